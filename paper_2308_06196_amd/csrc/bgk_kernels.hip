// bgk_kernels.hip -- kernel instantiations and launchers (gfx950).
//
// Kernels: the fused stage (transport + relaxation + RK + limiter + moment
// partials), the residual, stand-alone moment partials, the per-node Newton
// solve for the discretely conservative equilibrium, and state conversion /
// Maxwellian initialisation. All launched on the caller's stream.
#include <cmath>
#include <cstdlib>

#include "bgk_device.hpp"
#include "bgk_device3d.hpp"
#include "bgk_launch.hpp"

namespace bgk {

// ---------------------------------------------------------------------------
// Discretely conservative equilibrium, one thread per spatial node
// (Sec. 2.1: Maxwellian on a perturbed state whose discrete moments equal
// those of f; Newton's method with the closed-form Jacobian).
//
// g_j = exp(alpha . psi_j) and the trapezoid weights are products over the
// three velocity components, so every sum over the N_v nodes factorises into
// one-dimensional sums S_c^n = sum_b w_c[b] E_c[b] u_b^n (n = 0..4) with
// E_c[b] = exp(alpha_{1+c} u_b + alpha_4 u_b^2 / 2): O(3 N_1d) work per node.
// ---------------------------------------------------------------------------
__device__ static int chol5_solve(double J[5][5], const double* b, double* x) {
  double L[5][5], R[5];
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int k = 0; k < 5; ++k) L[i][k] = 0.0;
#pragma unroll
  for (int i = 0; i < 5; ++i) {
#pragma unroll
    for (int k = 0; k <= i; ++k) {
      double s = J[i][k];
#pragma unroll
      for (int m = 0; m < k; ++m) s -= L[i][m] * L[k][m];
      if (i == k) {
        if (!(s > 0.0)) return 1;
        L[i][i] = sqrt(s);
        R[i] = 1.0 / L[i][i];
      } else {
        L[i][k] = s * R[k];
      }
    }
  }
  double y[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    double s = b[i];
#pragma unroll
    for (int m = 0; m < i; ++m) s -= L[i][m] * y[m];
    y[i] = s * R[i];
  }
#pragma unroll
  for (int i = 4; i >= 0; --i) {
    double s = y[i];
#pragma unroll
    for (int m = i + 1; m < 5; ++m) s -= L[m][i] * x[m];
    x[i] = s * R[i];
  }
  return 0;
}

// All-reduce of one FP64 value over the T lanes of a team (T = 16: one DPP
// row, partners lane ^ 8, the mirror inside 8 lanes, lane ^ 2, lane ^ 1;
// T = 8 from the mirror on; T = 4: one quad; T = 2: a lane pair). Each step
// pairs lanes symmetrically, so every lane ends with the same bits.
template <int T>
__device__ __forceinline__ double team_sum(double x) {
  if constexpr (T == 16) x += dpp_partner<8>(x);
  if constexpr (T >= 8) x += dpp_partner<4>(x);
  if constexpr (T >= 4) x += dpp_partner<2>(x);
  x += dpp_partner<1>(x);
  return x;
}

// One team of kTeam lanes per spatial node. The lanes split the velocity
// chunks of the moment partials and the nodes of each one-dimensional sum;
// the 5x5 solve is repeated identically in every lane of the team. Large
// meshes use 2- or 4-lane teams (less redundant solve work), small ones
// 16-lane teams (enough waves to fill the device).
template <int kTeam>
__device__ __forceinline__ void newton_item(const NewtonArgs& A, const int64_t node_raw) {
  const DevGeom& g = A.g;
  const int r = threadIdx.x % kTeam;
  // teams past the last node work on the last node and store nothing, so that
  // every lane reaches the wave-level counter reduction at the end
  const bool active = node_raw < g.nx;
  const int64_t node = active ? node_raw : g.nx - 1;
  double Q[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const double* pp = A.partials + node * 5;  // chunk c at pp[c * nx * 5]
  // chunk partials: batches of 4 chunks per lane, all loads of a batch in flight
  for (int c0 = 0; c0 < g.nchunk; c0 += 4 * kTeam) {
    double v[4][5];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int c = c0 + u * kTeam + r;
#pragma unroll
      for (int m = 0; m < 5; ++m) v[u][m] = c < g.nchunk ? pp[(int64_t)c * g.nx * 5 + m] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int m = 0; m < 5; ++m) Q[m] += v[u][m];
  }
#pragma unroll
  for (int m = 0; m < 5; ++m) Q[m] = team_sum<kTeam>(Q[m]);
  if (A.Q && r == 0 && active) {
#pragma unroll
    for (int m = 0; m < 5; ++m) A.Q[node * 5 + m] = Q[m];
  }
  double* out = A.params + node * 8;
  if (!A.collide) {  // uniform over the grid
    if (r == 0 && active) {
#pragma unroll
      for (int m = 0; m < 8; ++m) out[m] = 0.0;
    }
    return;
  }
  const double rho = Q[0];
  const double UU = (Q[1] * Q[1] + Q[2] * Q[2] + Q[3] * Q[3]) / (rho * rho);
  const double P = (A.gamma - 1.0) * (Q[4] - 0.5 * rho * UU);
  const double th = P / rho;
  int status = 0, iters = 0;
  double al[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (!(rho > 0.0) || !(th > 0.0)) {
    status = 2;
  } else {
    const double tpt = 2.0 * M_PI * th;
    al[0] = log(rho / (tpt * sqrt(tpt))) - UU / (2.0 * th);
    al[1] = Q[1] / rho / th;
    al[2] = Q[2] / rho / th;
    al[3] = Q[3] / rho / th;
    al[4] = -1.0 / th;
    const double sq = rho * sqrt(th);
    const double sc[5] = {rho, sq, sq, sq, Q[4]};
    // the non-conservative model keeps the continuous Maxwellian (no solve)
    for (int it = 0; !A.continuous; ++it) {
      double S[3][5];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
#pragma unroll
        for (int n = 0; n < 5; ++n) S[c][n] = 0.0;
        const int N = g.nv1[c];
        for (int b = r; b < N; b += kTeam) {
          const double u = g.vlo[c] + b * g.du[c];
          double wc = g.du[c];
          if (b == 0 || b == N - 1) wc *= 0.5;
          const double t = wc * exp(al[1 + c] * u + al[4] * (0.5 * u * u));
          const double u2 = u * u;
          S[c][0] += t;
          S[c][1] += t * u;
          S[c][2] += t * u2;
          S[c][3] += t * u2 * u;
          S[c][4] += t * u2 * u2;
        }
#pragma unroll
        for (int n = 0; n < 5; ++n) S[c][n] = team_sum<kTeam>(S[c][n]);
      }
      double m[3][5];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double inv = 1.0 / S[c][0];
        m[c][0] = 1.0;
#pragma unroll
        for (int n = 1; n < 5; ++n) m[c][n] = S[c][n] * inv;
      }
      const double A0 = exp(al[0]) * S[0][0] * S[1][0] * S[2][0];
      double G[5], J[5][5];
      G[0] = A0;
      G[1] = A0 * m[0][1];
      G[2] = A0 * m[1][1];
      G[3] = A0 * m[2][1];
      G[4] = A0 * 0.5 * (m[0][2] + m[1][2] + m[2][2]);
#pragma unroll
      for (int a = 0; a < 5; ++a) {
        J[0][a] = G[a];
        J[a][0] = G[a];
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
#pragma unroll
        for (int c2 = 0; c2 < 3; ++c2)
          J[1 + c][1 + c2] = (c == c2) ? A0 * m[c][2] : A0 * m[c][1] * m[c2][1];
        double t = m[c][3];
#pragma unroll
        for (int c2 = 0; c2 < 3; ++c2)
          if (c2 != c) t += m[c][1] * m[c2][2];
        J[1 + c][4] = J[4][1 + c] = A0 * 0.5 * t;
      }
      J[4][4] = A0 * 0.25 *
                (m[0][4] + m[1][4] + m[2][4] +
                 2.0 * (m[0][2] * m[1][2] + m[0][2] * m[2][2] + m[1][2] * m[2][2]));
      double F[5], res = 0.0;
#pragma unroll
      for (int a = 0; a < 5; ++a) {
        F[a] = G[a] - Q[a];
        const double ra = fabs(F[a]) / sc[a];
        if (!(ra <= res)) res = ra;
      }
      iters = it + 1;
      const bool conv = res <= A.tol;
      if (!conv && it >= A.maxit) {
        status = 1;
        break;
      }
      double d[5];
      if (chol5_solve(J, F, d)) {
        status = 2;
        break;
      }
      double an[5];
#pragma unroll
      for (int a = 0; a < 5; ++a) an[a] = al[a] - d[a];
      for (int h = 0; h < 60 && !(an[4] < 0.0); ++h) {
#pragma unroll
        for (int a = 0; a < 5; ++a) {
          d[a] *= 0.5;
          an[a] = al[a] - d[a];
        }
      }
      if (!(an[4] < 0.0)) {
        status = 2;
        break;
      }
#pragma unroll
      for (int a = 0; a < 5; ++a) al[a] = an[a];
      if (conv) break;  // that was the polishing step
    }
  }
  if (status) {
#pragma unroll
    for (int a = 0; a < 5; ++a) al[a] = __builtin_nan("");
  }
  // relaxation time tau = mu / P (Sec. 2) with mu from the temperature law
  const double tr = th / A.theta_ref;
  const double mu = A.sutherland > 0.0
                        ? A.mu_ref * tr * sqrt(tr) * (A.theta_ref + A.sutherland) / (th + A.sutherland)
                        : A.mu_ref * pow(tr, A.omega);
  const double itau = P / mu;  // 1 / tau
  // one-dimensional factors of the equilibrium in FP64 for every storage
  // precision: exp(alpha_0) and 1/tau folded into x, so that the stage kernels
  // form the collision term as Ex[bx] Ey[by] Ez[bz] - f / tau
  double* row = (double*)A.etab + node * g.tabw;
  int off = 0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int N = g.nv1[c];
    const double a0 = c == 0 ? al[0] : 0.0;
    if (active) {
      for (int b = r; b < N; b += kTeam) {
        const double u = g.vlo[c] + b * g.du[c];
        const double v = exp(a0 + al[1 + c] * u + al[4] * (0.5 * u * u));
        row[off + b] = c == 0 ? v * itau : v;
      }
    }
    off += N;
  }
  if (r == 0 && active) {
#pragma unroll
    for (int a = 0; a < 5; ++a) out[a] = al[a];
    out[5] = itau;
    out[6] = 1.0 / itau;
    out[7] = (double)status;
    row[off] = itau;  // 1/tau closes the node's row
  }
  // counters: one atomic per wave (the four teams of a wave reduced first)
  int itw = active ? iters : 0;
  for (int o = kTeam; o < 64; o <<= 1) itw = max(itw, __shfl_xor(itw, o, 64));
  const unsigned long long nfail = __popcll(__ballot(active && r == 0 && status != 0));
  if ((threadIdx.x & 63) == 0) {
    if (itw > 0) atomicMax(&A.diag[0], (unsigned long long)itw);
    if (nfail) atomicAdd(&A.diag[1], nfail);
  }
}

template <int kTeam>
__global__ void __launch_bounds__(256) k_newton(const NewtonArgs A) {
  newton_item<kTeam>(A, ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kTeam);
}

// Equilibrium solves of the batch members of one team size: whole work-groups
// of 256 lanes per member, so that a work-group's arguments are uniform; the
// grid is the list's work-group count.
template <int kTeam>
__global__ void __launch_bounds__(256) k_newton_batch(table_ptr<NewtonArgs> args,
                                                      table_ptr<BatchList> list) {
  const int32_t t = blockIdx.x;
  const int m = batch_member(list->newton_off, list->n, t);
  newton_item<kTeam>(table_entry(args, list->slot[m]),
                     ((int64_t)(t - list->newton_off[m]) * 256 + threadIdx.x) / kTeam);
}

// Q[node][5] from the partials (no Newton solve).
__global__ void __launch_bounds__(256) k_reduce_partials(const DevGeom g, const double* partials,
                                                         double* Q) {
  const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= g.nx) return;
  double q[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const double* pp = partials + node * 5;
  for (int c = 0; c < g.nchunk; ++c)
#pragma unroll
    for (int m = 0; m < 5; ++m) q[m] += pp[(int64_t)c * g.nx * 5 + m];
#pragma unroll
  for (int m = 0; m < 5; ++m) Q[node * 5 + m] = q[m];
}

// Discrete moments of the collision term of a stored state, per node and
// chunk of kBlock velocities: sum_j w_j psi_j C_j with C_j formed by
// collision_term from the FP64 equilibrium rows and the stored values, as in
// the stage kernels. One work-group = one element x one chunk; lanes are
// summed by an xor butterfly and the four waves in a fixed order.
template <typename ST>
__global__ void __launch_bounds__(kBlock) k_collision_moments(const StageArgs A, int nchunk) {
  __shared__ double red[kBlock / 64][5];
  const DevGeom& g = A.g;
  const int64_t e = (int64_t)blockIdx.x / nchunk;
  const int chunk = (int)(blockIdx.x % nchunk);
  const int j = chunk * kBlock + (int)threadIdx.x;
  const bool valid = j < g.nv;
  const int jj = valid ? j : (int)g.nv - 1;
  const Vel vel = velocity_of(g, jj);
  const double wt = valid ? vel.w : 0.0;
  const double psi4 = 0.5 * (vel.u[0] * vel.u[0] + vel.u[1] * vel.u[1] + vel.u[2] * vel.u[2]);
  const int S = g.tabw;
  const int oy = g.nv1[0] + vel.b[1], oz = g.nv1[0] + g.nv1[1] + vel.b[2];
  const ST* fin = (const ST*)A.fin;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int i = 0; i < g.ns; ++i) {
    const int64_t node = e * g.ns + i;
    const double fv = (double)fin[f_offset(g, e, i, jj)];
    const double c = wt * collision_term(A.etab + node * S, vel.b[0], oy, oz, S, fv);
    double m[5] = {c, c * vel.u[0], c * vel.u[1], c * vel.u[2], c * psi4};
#pragma unroll
    for (int q = 0; q < 5; ++q)
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) m[q] += __shfl_xor(m[q], o, 64);
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < 5; ++q) red[wave][q] = m[q];
    }
    __syncthreads();
    if (threadIdx.x < 5) {
      double sum = 0.0;
#pragma unroll
      for (int w = 0; w < kBlock / 64; ++w) sum += red[w][threadIdx.x];
      A.partials[((int64_t)chunk * g.nx + node) * 5 + threadIdx.x] = sum;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Diffuse walls. At a flux point of a wall face the gas leaving the domain
// carries the discrete mass flux sum_{outgoing j} w_j |u_k| f_trace; the wall
// re-emits rho_w times the unit wall Maxwellian into the incoming velocities,
// with rho_w = that flux / (incoming flux of the unit wall Maxwellian), so the
// net mass flux through the wall vanishes.
// ---------------------------------------------------------------------------

// One work-group = one wall-face element x one chunk of 256 velocities; the
// flux points' partial sums are reduced in a fixed order (lanes by an xor
// butterfly, then the four waves in LDS).
template <int DIM, int P, typename ST>
__device__ __forceinline__ void wall_flux_item(const WallArgs& W, const int b) {
  constexpr int N1 = P + 1;
  constexpr int NF = ipow(N1, DIM - 1);
  __shared__ double red[kBlock / 64][NF];
  const DevGeom& g = W.g;
  int q = 0;
  while (q + 1 < W.nside && b >= W.blk0[q + 1]) ++q;
  const int k = W.side_k[q], side = W.side_s[q];
  const int local = b - W.blk0[q];
  const int face = local / g.nchunk, chunk = local % g.nchunk;
  // element: coordinate k on the wall, the other coordinate (2-D) = face
  int ek[2] = {0, 0};
  ek[k] = side == 0 ? 0 : g.nelem[k] - 1;
  if (DIM == 2) ek[1 - k] = face;
  const int64_t e = ek[0] + (int64_t)g.nelem[0] * ek[1];
  const int64_t nv = g.nv;
  const int j = chunk * kBlock + (int)threadIdx.x;
  const bool valid = j < nv;
  const int jj = valid ? j : (int)nv - 1;
  const Vel vel = velocity_of(g, jj);
  const double a = vel.u[k];
  const bool outgoing = valid && (side == 0 ? a < 0.0 : a > 0.0);
  const double wt = outgoing ? vel.w * fabs(a) : 0.0;
  const int S1 = k == 0 ? 1 : N1;
  const ST* fe = (const ST*)W.fin + f_offset(g, e, 0, jj);
  double v[NF];
#pragma unroll
  for (int fp = 0; fp < NF; ++fp) {
    const int base = (fp % S1) + (fp / S1) * S1 * N1;
    double tr = 0.0;
#pragma unroll
    for (int bb = 0; bb < N1; ++bb)
      tr += (side == 0 ? W.lamL[bb] : W.lamR[bb]) * (double)fe[(base + bb * S1) * kVB];
    v[fp] = wt * tr;
  }
#pragma unroll
  for (int fp = 0; fp < NF; ++fp) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v[fp] += __shfl_xor(v[fp], o, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int fp = 0; fp < NF; ++fp) red[wave][fp] = v[fp];
  }
  __syncthreads();
  if ((int)threadIdx.x < NF) {
    double sum = 0.0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) sum += red[w][threadIdx.x];
    W.part[((int64_t)W.off[q] + face * NF + threadIdx.x) * g.nchunk + chunk] = sum;
  }
}

template <int DIM, int P, typename ST>
__global__ void __launch_bounds__(kBlock) k_wall_flux(const WallArgs W) {
  wall_flux_item<DIM, P, ST>(W, blockIdx.x);
}

template <int DIM, int P, typename ST>
__global__ void __launch_bounds__(kBlock) k_wall_flux_batch(table_ptr<WallArgs> args,
                                                            table_ptr<BatchList> list, int stage) {
  const int32_t t = blockIdx.x;  // grid: the list's wall-flux work-groups
  const int m = batch_member(list->wflux_off, list->n, t);
  wall_flux_item<DIM, P, ST>(table_entry(args, list->slot[m] * 3 + stage),
                             (int)(t - list->wflux_off[m]));
}

// rho_w per wall flux point: the chunk partials summed in order, times the
// inverse incoming flux of the side's unit wall Maxwellian.
__device__ __forceinline__ void wall_rho_item(const WallArgs& W, const int t) {
  if (t >= W.npoints) return;
  int q = 0;
  while (q + 1 < W.nside && t >= W.off[q + 1]) ++q;
  const double* p = W.part + (int64_t)t * W.g.nchunk;
  double sum = 0.0;
  for (int c = 0; c < W.g.nchunk; ++c) sum += p[c];
  W.rho[t] = sum * W.wallp[(W.side_k[q] * 2 + W.side_s[q]) * 8 + 5];
}

__global__ void __launch_bounds__(256) k_wall_rho(const WallArgs W) {
  wall_rho_item(W, blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ void __launch_bounds__(256) k_wall_rho_batch(table_ptr<WallArgs> args,
                                                        table_ptr<BatchList> list, int stage) {
  const int32_t t = blockIdx.x;  // grid: the list's wall-density work-groups
  const int m = batch_member(list->wrho_off, list->n, t);
  wall_rho_item(table_entry(args, list->slot[m] * 3 + stage),
                (int)((t - list->wrho_off[m]) * 256 + threadIdx.x));
}

// Continuous Maxwellian sampled at every (node, velocity); one work-group =
// one node x one velocity chunk.
// grid-stride over (node, velocity chunk) work items: the number of work
// items can exceed what one launch dimension holds
template <typename ST>
__global__ void __launch_bounds__(kBlock) k_maxwellian(const DevGeom g, const double* prim, ST* f) {
  const int64_t nw = g.nx * g.nchunk;
  for (int64_t w = blockIdx.x; w < nw; w += gridDim.x) {
    const int64_t node = w / g.nchunk;
    const int chunk = (int)(w % g.nchunk);
    const int j = chunk * kBlock + (int)threadIdx.x;
    if (j >= g.nv) continue;
    const Vel v = velocity_of(g, j);
    const double* q = prim + node * 5;
    const double rho = q[0], th = q[4];
    const double nrm = rho / pow(2.0 * M_PI * th, 1.5);
    const double dx = v.u[0] - q[1], dy = v.u[1] - q[2], dz = v.u[2] - q[3];
    f[f_offset(g, node / g.ns, (int)(node % g.ns), j)] =
        (ST)(nrm * exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * th)));
  }
}

// Exchange between the canonical FP64 layout f[elem][node][vel] and the
// internal layout in storage precision (velocity blocks, velocities in slot
// order): entries i0 .. i0+m-1 of the canonical
// array, held at canon[0 .. m-1] (a staging window or the whole array).
template <typename DST>
__global__ void __launch_bounds__(256) k_to_internal(const DevGeom g, const double* canon, DST* f,
                                                     int64_t i0, int64_t m) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x, per_e = (int64_t)g.ns * g.nv;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m; t += stride) {
    const int64_t i = i0 + t, e = i / per_e, r = i - e * per_e, a = r / g.nv;
    f[f_offset(g, e, (int)a, vel_slot_of_canonical(g, (int)(r - a * g.nv)))] = (DST)canon[t];
  }
}

template <typename SRC>
__global__ void __launch_bounds__(256) k_to_canonical(const DevGeom g, const SRC* f, double* canon,
                                                      int64_t i0, int64_t m) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x, per_e = (int64_t)g.ns * g.nv;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m; t += stride) {
    const int64_t i = i0 + t, e = i / per_e, r = i - e * per_e, a = r / g.nv;
    canon[t] = (double)f[f_offset(g, e, (int)a, vel_slot_of_canonical(g, (int)(r - a * g.nv)))];
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static inline unsigned grid_of(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// Hexahedra. The one-lane-per-velocity kernels (k_stage<3, ...>: all
// (p+1)^3 nodes of a velocity in one lane's registers) run FP32 storage at
// every order and FP64 storage and BF16 increments at p <= 2; the
// plane-split kernels (k_stage3: four lanes per velocity, one z-plane each)
// run FP64 storage and BF16 increments at p = 3, where one lane cannot hold
// the element (FP64) or the second value per neighbour node (BF16: 137
// spilled registers). On the 16^3-element Taylor-Green box, ms per stage,
// plane-split against one-lane: FP64 p = 1 1.18 / 0.82, p = 2 4.95 / 2.50
// (two waves per SIMD; 6.22 at three, which spill); BF16 p = 1 0.90 / 0.51,
// p = 2 3.31 / 1.62, p = 3 6.83 / 7.72; FP32 p = 3 5.49 / 3.61.
// The choice (hex_one_lane) is per solver, so that all its kernels share one
// velocity-chunk width; it must agree with kHexOneLane below.
template <int P, typename ST>
constexpr bool kHexOneLane(bool inc) {
  return sizeof(ST) == 8 ? P <= 2 : (P <= 2 || !inc);
}

// RK stages over the whole mesh run as column sweeps along the last axis
// (k_stage_sweep, k_stage3_sweep) when the solver chose a segment length and
// the mesh has no diffuse wall.
static bool use_sweep(int mode, const StageArgs& A) {
  if (mode != 0 || A.sweep_seg <= 0 || A.g.dim < 2) return false;
  if (A.e0 != 0 || A.ecount != A.g.ne || A.g.nelem[A.g.dim - 1] % A.sweep_seg != 0) return false;
  for (int k = 0; k < 2; ++k)
    if (A.wall_off[k][0] >= 0 || A.wall_off[k][1] >= 0) return false;
  return true;
}

static dim3 sweep_grid(const StageArgs& A) {
  return dim3((unsigned)(A.g.nchunk * (A.g.ne / A.sweep_seg)));
}

template <int D, int P, typename ST, bool kIncBuilt = true>
static void launch_sweep(bool inc, const StageArgs& A, size_t lds, hipStream_t s) {
  const dim3 grid = sweep_grid(A), block(kBlock);
  if constexpr (sizeof(ST) == 4 && kIncBuilt) {
    if (inc) {
      if (A.din)
        hipLaunchKernelGGL((k_stage_sweep<D, P, ST, 0, true>), grid, block, lds, s, A);
      else
        hipLaunchKernelGGL((k_stage_sweep<D, P, ST, 3, true>), grid, block, lds, s, A);
      return;
    }
  }
  if (A.a != 0.0)
    hipLaunchKernelGGL((k_stage_sweep<D, P, ST, 0>), grid, block, lds, s, A);
  else
    hipLaunchKernelGGL((k_stage_sweep<D, P, ST, 3>), grid, block, lds, s, A);
}

template <int P, typename ST>
static void launch_sweep3(bool inc, const StageArgs& A, size_t lds, hipStream_t s) {
  const dim3 grid = sweep_grid(A), block(kBlock);
  // BF16 increments on planes of whole node pairs (odd p; p = 3 is the one
  // that runs plane-split, kHexOneLane)
  if constexpr (sizeof(ST) == 4 && Plane3<P>::P2 % 2 == 0) {
    if (inc) {
      if (A.din)
        hipLaunchKernelGGL((k_stage3_sweep<P, ST, 0, true>), grid, block, lds, s, A);
      else
        hipLaunchKernelGGL((k_stage3_sweep<P, ST, 3, true>), grid, block, lds, s, A);
      return;
    }
  }
  if (A.a != 0.0)
    hipLaunchKernelGGL((k_stage3_sweep<P, ST, 0>), grid, block, lds, s, A);
  else
    hipLaunchKernelGGL((k_stage3_sweep<P, ST, 3>), grid, block, lds, s, A);
}

template <int P, typename ST>
static hipError_t hex_dispatch(int mode, bool inc, const StageArgs& A, size_t tab, size_t lds,
                               dim3 grid, dim3 block, hipStream_t s) {
  const bool sweep = use_sweep(mode, A);
  if (kHexOneLane<P, ST>(inc)) {
    if constexpr (sizeof(ST) == 8 && P > 2) return hipErrorInvalidValue;  // not built
    else {
      if (sweep) {
        launch_sweep<3, P, ST, (P <= 2)>(inc, A, lds, s);  // one-lane increments: p <= 2
      } else if (mode == 0 && inc) {
        if constexpr (sizeof(ST) == 4 && P <= 2) {
          if (A.din)
            hipLaunchKernelGGL((k_stage<3, P, ST, 0, true>), grid, block, lds, s, A);
          else
            hipLaunchKernelGGL((k_stage<3, P, ST, 3, true>), grid, block, lds, s, A);
        }
      } else if (mode == 0 && A.a != 0.0) {
        hipLaunchKernelGGL((k_stage<3, P, ST, 0>), grid, block, lds, s, A);
      } else if (mode == 0) {
        hipLaunchKernelGGL((k_stage<3, P, ST, 3>), grid, block, lds, s, A);
      } else if (mode == 1) {
        hipLaunchKernelGGL((k_stage<3, P, ST, 1>), grid, block, lds, s, A);
      } else {
        hipLaunchKernelGGL((k_moments<3, P, ST>), grid, block, lds, s, A);
      }
      return hipGetLastError();
    }
  }
  // plane-split; the FP64 ones decode lexicographic slots (one octant)
  if (sizeof(ST) == 8 && A.g.voct[7] != 0) return hipErrorInvalidValue;
  const size_t lds3 = mode != 1 ? std::max(tab, (size_t)mfma3_lds_bytes<P, ST>()) : tab;
  if (sweep) {
    launch_sweep3<P, ST>(inc, A, lds3, s);
  } else if (mode == 0 && inc) {
    if constexpr (sizeof(ST) == 4 && Plane3<P>::P2 % 2 == 0) {
      if (A.din)
        hipLaunchKernelGGL((k_stage3<P, ST, 0, true>), grid, block, lds3, s, A);
      else
        hipLaunchKernelGGL((k_stage3<P, ST, 3, true>), grid, block, lds3, s, A);
    }
  } else if (mode == 0 && A.a != 0.0) {
    hipLaunchKernelGGL((k_stage3<P, ST, 0>), grid, block, lds3, s, A);
  } else if (mode == 0) {
    hipLaunchKernelGGL((k_stage3<P, ST, 3>), grid, block, lds3, s, A);
  } else if (mode == 1) {
    hipLaunchKernelGGL((k_stage3<P, ST, 1>), grid, block, lds3, s, A);
  } else {
    hipLaunchKernelGGL((k_moments3<P, ST>), grid, block, lds3, s, A);
  }
  return hipGetLastError();
}

template <typename ST>
static hipError_t stage_dispatch(int mode, bool inc, const StageArgs& A, hipStream_t s) {
  const dim3 grid((unsigned)(A.g.nchunk * A.ecount)), block(kBlock);
  const int key = A.g.dim * 10 + (A.g.n1 - 1);
  // dynamic LDS: equilibrium rows (relaxation), then, in the 1-D/2-D
  // kernels, the MFMA staging of the moment partials in the same bytes
  const size_t tab = A.collide ? (size_t)A.g.ns * A.g.tabw * sizeof(double) : 0;
  const size_t lds = mode != 1 ? std::max(tab, (size_t)mfma_lds_bytes<ST>()) : tab;
#define BGK_CASE(D, P)                                                     \
  case D * 10 + P:                                                         \
    if (D >= 2 && use_sweep(mode, A)) {                                    \
      launch_sweep<(D >= 2 ? D : 2), P, ST>(inc, A, lds, s);               \
      break;                                                               \
    }                                                                      \
    if constexpr (sizeof(ST) == 4) {                                       \
      if (mode == 0 && inc) {                                              \
        if (A.din)                                                         \
          hipLaunchKernelGGL((k_stage<D, P, ST, 0, true>), grid, block, lds, s, A); \
        else                                                               \
          hipLaunchKernelGGL((k_stage<D, P, ST, 3, true>), grid, block, lds, s, A); \
        break;                                                             \
      }                                                                    \
    }                                                                      \
    if (mode == 0 && A.a != 0.0)                                           \
      hipLaunchKernelGGL((k_stage<D, P, ST, 0>), grid, block, lds, s, A);  \
    else if (mode == 0)                                                    \
      hipLaunchKernelGGL((k_stage<D, P, ST, 3>), grid, block, lds, s, A);  \
    else if (mode == 1)                                                    \
      hipLaunchKernelGGL((k_stage<D, P, ST, 1>), grid, block, lds, s, A);  \
    else                                                                   \
      hipLaunchKernelGGL((k_moments<D, P, ST>), grid, block, lds, s, A);   \
    break;
#define BGK_CASE3(P)                                                       \
  case 30 + P:                                                             \
    return hex_dispatch<P, ST>(mode, inc, A, tab, lds, grid, block, s);
  switch (key) {
    BGK_CASE(1, 1) BGK_CASE(1, 2) BGK_CASE(1, 3)
    BGK_CASE(2, 1) BGK_CASE(2, 2) BGK_CASE(2, 3)
    BGK_CASE3(1) BGK_CASE3(2) BGK_CASE3(3)
    default:
      return hipErrorInvalidValue;
  }
#undef BGK_CASE
#undef BGK_CASE3
  return hipGetLastError();
}

// Work-groups of kernel k (256 lanes, lds bytes of dynamic LDS) that one CU
// holds at once.
template <typename K>
static int groups_per_cu(K k, size_t lds) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, kBlock, lds) != hipSuccess) return 0;
  return n;
}

template <int D, int P, typename ST>
static int sweep_groups_per_cu(bool inc, size_t tab) {
  if constexpr (D == 3) {
    if (!kHexOneLane<P, ST>(inc)) {
      const size_t lds = std::max(tab, (size_t)mfma3_lds_bytes<P, ST>());
      if constexpr (sizeof(ST) == 4 && Plane3<P>::P2 % 2 == 0) {
        if (inc) return groups_per_cu(k_stage3_sweep<P, ST, 0, true>, lds);
      }
      return groups_per_cu(k_stage3_sweep<P, ST, 0>, lds);
    }
    if constexpr (sizeof(ST) == 8 && P > 2) return 0;  // not built
  }
  const size_t lds = std::max(tab, (size_t)mfma_lds_bytes<ST>());
  if constexpr (sizeof(ST) == 4 && (D == 2 || P <= 2)) {
    if (inc) return groups_per_cu(k_stage_sweep<D, P, ST, 0, true>, lds);
  }
  if constexpr (sizeof(ST) == 8 && D == 3 && P > 2) return 0;
  else return groups_per_cu(k_stage_sweep<D, P, ST, 0>, lds);
}

template <typename ST>
static int sweep_groups(int dim, int order, bool inc, size_t tab) {
  switch (dim * 10 + order) {
    case 21: return sweep_groups_per_cu<2, 1, ST>(inc, tab);
    case 22: return sweep_groups_per_cu<2, 2, ST>(inc, tab);
    case 23: return sweep_groups_per_cu<2, 3, ST>(inc, tab);
    case 31: return sweep_groups_per_cu<3, 1, ST>(inc, tab);
    case 32: return sweep_groups_per_cu<3, 2, ST>(inc, tab);
    case 33: return sweep_groups_per_cu<3, 3, ST>(inc, tab);
    default: return 0;
  }
}

// Elements per column-sweep work item (0: no sweep). A work-group walks its
// segment one element after another, so long segments leave the last wave
// of work-groups part of the device idle; each segment's first element reads
// its upwind neighbour's nodes. The choice minimises (1 + 0.2 / seg) / eff,
// eff = R / ceil(R) for R = work items / work-groups resident on the device
// (from the kernel's occupancy), over the divisors seg >= 2 of the number of
// elements along the last axis; seg = 1 (no sweep) when that is cheaper.
// The environment variable BGK_SWEEP_SEG overrides the choice (0: no sweep;
// a length that does not divide the column length means no sweep).
// Sweeps are used where they measured faster than the per-element kernels
// (ms per stage launch, sweep / per element): quadrilaterals in FP64 (32^2
// box, p = 3: 1.021 / 1.039) and p = 3 hexahedra in FP32 (Taylor-Green box,
// one lane per velocity: 3.26 / 3.50; the sweep's last axis loads nothing,
// and without its loads the element fits the registers). Not for FP32 and
// BF16 quadrilaterals (0.626 / 0.588, the loop costs registers at five waves
// per SIMD), p = 2 hexahedra (Mach-2 box at four waves per SIMD: spills),
// FP64 p = 3 hexahedra (the plane-split sweep needs two waves per SIMD where
// the per-element kernel runs three: 10.2 / 9.88) or BF16 increments at
// p = 3 (plane-split at four waves per SIMD: 7.36 / 5.84).
static bool sweep_pays(const DevGeom& g, int precision) {
  if (g.dim == 2) return precision == 0;
  return g.dim == 3 && g.n1 == 4 && precision == 1;
}

int sweep_segment(const DevGeom& g, int precision, bool collide) {
  if (g.dim < 2) return 0;
  const int nl = g.nelem[g.dim - 1];
  if (const char* env = getenv("BGK_SWEEP_SEG")) {
    const int v = atoi(env);
    return v >= 1 && nl % v == 0 ? v : 0;
  }
  if (!sweep_pays(g, precision)) return 0;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  const size_t tab = collide ? (size_t)g.ns * g.tabw * sizeof(double) : 0;
  const bool inc = precision == 2;
  const int per_cu = precision == 0 ? sweep_groups<double>(g.dim, g.n1 - 1, false, tab)
                                    : sweep_groups<float>(g.dim, g.n1 - 1, inc, tab);
  (void)hipGetLastError();
  if (per_cu <= 0 || cus <= 0) return 0;
  const double resident = (double)per_cu * cus;
  const double cols = (double)(g.ne / nl) * g.nchunk;
  int best = 0;
  double best_cost = 0.0;
  for (int seg = 1; seg <= nl; ++seg) {
    if (nl % seg) continue;
    const double R = cols * (nl / seg) / resident;
    const double eff = R / std::ceil(R);
    const double cost = (1.0 + 0.2 / seg) / eff;
    if (best == 0 || cost < best_cost) {
      best = seg;
      best_cost = cost;
    }
  }
  return best >= 2 ? best : 0;
}

bool hex_one_lane(int order, int precision) {
  return precision != 2 ? (precision == 1 || order <= 2) : order <= 2;
}

int velocities_per_block(int dim, int order, int precision) {
  if (dim < 3 || hex_one_lane(order, precision)) return kBlock;
  return order + 1 <= 2 ? Plane3<1>::VB : Plane3<3>::VB;
}

hipError_t launch_stage(int precision, int mode, const StageArgs& A, hipStream_t s) {
  if (A.ecount <= 0) return hipSuccess;
  // BF16 storage (precision 2): FP32 state with BF16 stage increments; the
  // RK stages use the increment kernels, everything else the FP32 ones
  return precision == 0 ? stage_dispatch<double>(mode, false, A, s)
                        : stage_dispatch<float>(mode, precision == 2, A, s);
}

template <typename ST>
static hipError_t wall_dispatch(const WallArgs& W, hipStream_t s) {
  const dim3 grid((unsigned)W.blk0[W.nside]), block(kBlock);
  switch (W.g.dim * 10 + (W.g.n1 - 1)) {
#define BGK_WALL(D, P)                                                          \
  case D * 10 + P:                                                              \
    hipLaunchKernelGGL((k_wall_flux<D, P, ST>), grid, block, 0, s, W);          \
    break;
    BGK_WALL(1, 1) BGK_WALL(1, 2) BGK_WALL(1, 3)
    BGK_WALL(2, 1) BGK_WALL(2, 2) BGK_WALL(2, 3)
#undef BGK_WALL
    default:
      return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_wall_rho, dim3(grid_of(W.npoints, 256)), dim3(256), 0, s, W);
  return hipGetLastError();
}

hipError_t launch_wall(int precision, const WallArgs& W, hipStream_t s) {
  if (W.nside == 0) return hipSuccess;
  return precision == 0 ? wall_dispatch<double>(W, s) : wall_dispatch<float>(W, s);
}

hipError_t launch_newton(const NewtonArgs& A, hipStream_t s) {
  // teams of 4 lanes per node once there are enough nodes to fill the GPU
  // (measured on 16,384 nodes: 0.045 ms against 0.076 ms with 16 lanes and
  // 0.047 ms with 2), of 2 lanes on large meshes (262,144 nodes: 0.146 ms
  // against 0.240 ms with 4; 884,736 nodes: 0.54 ms against 0.72 ms)
  const int team = newton_team(A.g.nx);
  if (team == 2)
    hipLaunchKernelGGL(k_newton<2>, dim3(grid_of(A.g.nx * 2, 256)), dim3(256), 0, s, A);
  else if (team == 4)
    hipLaunchKernelGGL(k_newton<4>, dim3(grid_of(A.g.nx * 4, 256)), dim3(256), 0, s, A);
  else
    hipLaunchKernelGGL(k_newton<16>, dim3(grid_of(A.g.nx * 16, 256)), dim3(256), 0, s, A);
  return hipGetLastError();
}

hipError_t launch_collision_moments(int precision, const StageArgs& A, double* Cm,
                                    hipStream_t s) {
  const int nchunk = (int)((A.g.nv + kBlock - 1) / kBlock);
  const dim3 grid((unsigned)(A.g.ne * nchunk)), block(kBlock);
  if (precision == 0)
    hipLaunchKernelGGL(k_collision_moments<double>, grid, block, 0, s, A, nchunk);
  else
    hipLaunchKernelGGL(k_collision_moments<float>, grid, block, 0, s, A, nchunk);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  DevGeom g = A.g;
  g.nchunk = nchunk;
  return launch_reduce_partials(g, A.partials, Cm, s);
}

hipError_t launch_stage_batch(int precision, int dim, int order, int stage, const StageArgs* args,
                              const BatchList* list, size_t tab_bytes, unsigned grid,
                              hipStream_t s) {
  if (grid == 0) return hipSuccess;
  const size_t lds = std::max(tab_bytes, (size_t)(precision == 0 ? mfma_lds_bytes<double>()
                                                                  : mfma_lds_bytes<float>()));
#define BGK_BATCH(D, P)                                                                       \
  case D * 10 + P:                                                                          \
    if (precision == 0) {                                                                   \
      if (stage == 0)                                                                       \
        hipLaunchKernelGGL((k_stage_batch<D, P, double, 3>), dim3(grid), dim3(kBlock), lds, s, \
                           (table_ptr<StageArgs>)args, (table_ptr<BatchList>)list, stage);                                              \
      else                                                                                  \
        hipLaunchKernelGGL((k_stage_batch<D, P, double, 0>), dim3(grid), dim3(kBlock), lds, s, \
                           (table_ptr<StageArgs>)args, (table_ptr<BatchList>)list, stage);                                              \
    } else {                                                                                \
      if (stage == 0)                                                                       \
        hipLaunchKernelGGL((k_stage_batch<D, P, float, 3>), dim3(grid), dim3(kBlock), lds, s, \
                           (table_ptr<StageArgs>)args, (table_ptr<BatchList>)list, stage);                                              \
      else                                                                                  \
        hipLaunchKernelGGL((k_stage_batch<D, P, float, 0>), dim3(grid), dim3(kBlock), lds, s, \
                           (table_ptr<StageArgs>)args, (table_ptr<BatchList>)list, stage);                                              \
    }                                                                                       \
    break;
  switch (dim * 10 + order) {
    BGK_BATCH(1, 1) BGK_BATCH(1, 2) BGK_BATCH(1, 3)
    BGK_BATCH(2, 1) BGK_BATCH(2, 2) BGK_BATCH(2, 3)
    default:
      return hipErrorInvalidValue;
  }
#undef BGK_BATCH
  return hipGetLastError();
}

hipError_t launch_newton_batch(int team, const NewtonArgs* args, const BatchList* list,
                               unsigned grid, hipStream_t s) {
  if (grid == 0) return hipSuccess;
  if (team == 16)
    hipLaunchKernelGGL(k_newton_batch<16>, dim3(grid), dim3(256), 0, s, (table_ptr<NewtonArgs>)args,
                       (table_ptr<BatchList>)list);
  else if (team == 4)
    hipLaunchKernelGGL(k_newton_batch<4>, dim3(grid), dim3(256), 0, s, (table_ptr<NewtonArgs>)args,
                       (table_ptr<BatchList>)list);
  else
    hipLaunchKernelGGL(k_newton_batch<2>, dim3(grid), dim3(256), 0, s, (table_ptr<NewtonArgs>)args,
                       (table_ptr<BatchList>)list);
  return hipGetLastError();
}

hipError_t launch_wall_flux_batch(int precision, int dim, int order, int stage,
                                  const WallArgs* args, const BatchList* list, unsigned grid,
                                  hipStream_t s) {
  if (grid == 0) return hipSuccess;
#define BGK_WBATCH(D, P)                                                                        \
  case D * 10 + P:                                                                            \
    if (precision == 0)                                                                       \
      hipLaunchKernelGGL((k_wall_flux_batch<D, P, double>), dim3(grid), dim3(kBlock), 0, s, \
                         (table_ptr<WallArgs>)args, (table_ptr<BatchList>)list, stage);                                                        \
    else                                                                                      \
      hipLaunchKernelGGL((k_wall_flux_batch<D, P, float>), dim3(grid), dim3(kBlock), 0, s, \
                         (table_ptr<WallArgs>)args, (table_ptr<BatchList>)list, stage);                                                        \
    break;
  switch (dim * 10 + order) {
    BGK_WBATCH(1, 1) BGK_WBATCH(1, 2) BGK_WBATCH(1, 3)
    BGK_WBATCH(2, 1) BGK_WBATCH(2, 2) BGK_WBATCH(2, 3)
    default:
      return hipErrorInvalidValue;
  }
#undef BGK_WBATCH
  return hipGetLastError();
}

hipError_t launch_wall_rho_batch(int stage, const WallArgs* args, const BatchList* list,
                                 unsigned grid, hipStream_t s) {
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL(k_wall_rho_batch, dim3(grid), dim3(256), 0, s, (table_ptr<WallArgs>)args,
                     (table_ptr<BatchList>)list, stage);
  return hipGetLastError();
}

int newton_team(int64_t nx) { return nx >= 131072 ? 2 : nx >= 8192 ? 4 : 16; }

hipError_t launch_reduce_partials(const DevGeom& g, const double* partials, double* Q,
                                  hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_partials, dim3(grid_of(g.nx, 256)), dim3(256), 0, s, g, partials,
                     Q);
  return hipGetLastError();
}

hipError_t launch_maxwellian(int precision, const DevGeom& g, const double* prim, void* f,
                             hipStream_t s) {
  const dim3 grid((unsigned)std::min<int64_t>(g.nx * g.nchunk, 1 << 20));
  if (precision == 0)
    hipLaunchKernelGGL(k_maxwellian<double>, grid, dim3(kBlock), 0, s, g, prim, (double*)f);
  else
    hipLaunchKernelGGL(k_maxwellian<float>, grid, dim3(kBlock), 0, s, g, prim, (float*)f);
  return hipGetLastError();
}

hipError_t launch_to_storage(int precision, const DevGeom& g, const double* in, void* out,
                             int64_t i0, int64_t m, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  const unsigned grid = (unsigned)std::min<int64_t>(grid_of(m, 256), 65536);
  if (precision == 0)
    hipLaunchKernelGGL(k_to_internal<double>, dim3(grid), dim3(256), 0, s, g, in, (double*)out, i0, m);
  else
    hipLaunchKernelGGL(k_to_internal<float>, dim3(grid), dim3(256), 0, s, g, in, (float*)out, i0, m);
  return hipGetLastError();
}

hipError_t launch_from_storage(int precision, const DevGeom& g, const void* in, double* out,
                               int64_t i0, int64_t m, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  const unsigned grid = (unsigned)std::min<int64_t>(grid_of(m, 256), 65536);
  if (precision == 0)
    hipLaunchKernelGGL(k_to_canonical<double>, dim3(grid), dim3(256), 0, s, g, (const double*)in,
                       out, i0, m);
  else
    hipLaunchKernelGGL(k_to_canonical<float>, dim3(grid), dim3(256), 0, s, g, (const float*)in,
                       out, i0, m);
  return hipGetLastError();
}

}  // namespace bgk
