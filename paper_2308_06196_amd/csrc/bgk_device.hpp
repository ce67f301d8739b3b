// bgk_device.hpp -- gfx950 kernels of the discrete-velocity Boltzmann-BGK
// hot path (Dzanic & Martinelli, arXiv 2308.06196, Sec. 2 and Sec. 2.1).
//
// Data layout in HBM (one solver):
//   f[elem][node][vel]   storage precision, velocity fastest (coalesced rows
//                        of nv values per spatial node)
//   partials[node][chunk][5]  FP64 moment partial sums of one stage output,
//                        one entry per 256-wide velocity chunk
//   params[node][8]      FP64 (alpha_0..alpha_4, 1/tau, tau, flag) of the
//                        discretely conservative equilibrium
//
// Thread mapping of the stage kernel: one work-group = one element x one
// chunk of 256 consecutive velocities; one thread = one velocity j and all
// (p+1)^d nodes of the element, held in registers. The FR operators are
// (p+1)-point contractions along element lines (sum factorisation, VALU);
// they are far below the FP64/FP32 ridge point, so the kernel is bound by
// HBM traffic, not by arithmetic.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bgk {

constexpr int kMaxN1 = 4;      // p <= 3
constexpr int kMaxNS = 64;     // (p+1)^d <= 64
constexpr int kBlock = 256;    // velocities per work-group
constexpr int kNumXCD = 8;     // MI355X: 8 accelerator complex dies

struct DevGeom {
  int32_t dim, n1, ns;
  int32_t nelem[3];
  int32_t bc[3][2];
  int32_t nv1[3];
  int64_t ne, nx, nv;
  int32_t nchunk;
  double vlo[3], du[3];
  double scale[3];  // 2 / h_k
};

struct DevOps {
  double D[kMaxN1][kMaxN1];  // D[a][b] = l_b'(xi_a)
  double lamL[kMaxN1], lamR[kMaxN1];
  double GL[kMaxN1], GR[kMaxN1];  // correction-function slopes at the nodes
  double W[kMaxNS];               // tensor-product Gauss weights per node
  double Wsum;
};

struct StageArgs {
  DevGeom g;
  DevOps op;
  const void* fin;   // stage input (storage precision)
  const void* fn;    // f^n (storage precision), read when a != 0
  void* out;         // stage output (storage precision), or FP64 residual
  const double* params;
  double* partials;
  unsigned long long* diag;  // [0] newton it max, [1] newton fail, [2] lim hits, [3] lim bad
  double dt, a, b;
  int64_t e0, ecount, out_e0;
  int32_t limiter, collide;
};

struct NewtonArgs {
  DevGeom g;
  const double* partials;
  double* params;
  double* Q;  // optional [nx][5] output of the reduced moments
  unsigned long long* diag;
  double gamma, mu_ref, theta_ref, omega, tol;
  int32_t maxit, collide;
};

constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

// Linear block id -> work id such that each XCD (blocks are dealt to the 8
// XCDs round-robin) walks one contiguous range of work ids, so that blocks
// of neighbouring elements share an L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t nb) {
  const int64_t x = bid % kNumXCD, k = bid / kNumXCD;
  const int64_t per = nb / kNumXCD, rem = nb % kNumXCD;
  return x * per + (x < rem ? x : rem) + k;
}

// ---------------------------------------------------------------------------
// Work-group reduction of M per-lane FP64 values (fixed order, no atomics).
// Butterfly reduce-scatter across the 64 lanes while the count is even,
// all-reduce for the remaining lane bits, then a sum over the 4 waves in LDS.
// ---------------------------------------------------------------------------
constexpr int shuffle_cost(int m) {
  int c = 0;
  for (int o = 32; o >= 1; o >>= 1) {
    if ((m & 1) == 0) { m >>= 1; c += m; } else { c += m; }
  }
  return c;
}
// nodes per reduction group: the largest divisor of NS not above 9
constexpr int group_of(int ns) {
  int g = 1;
  for (int d = 1; d <= 9 && d <= ns; ++d)
    if (ns % d == 0) g = d;
  return g;
}
constexpr int best_pad(int m) {
  int best = m, bc = shuffle_cost(m);
  for (int k = 1; k <= 64; k <<= 1) {
    int mp = (m + k - 1) / k * k;
    if (shuffle_cost(mp) < bc) { bc = shuffle_cost(mp); best = mp; }
  }
  return best;
}

// Butterfly step across lane bit 32 (16): lanes with the bit clear return
// x + x(partner), lanes with it set return y(partner) + y. gfx950's
// v_permlane32_swap / v_permlane16_swap exchange the odd 32- (16-) lane rows
// of the first operand with the even rows of the second.
template <int O>
__device__ __forceinline__ double swap_sum(double x, double y) {
  const unsigned xl = (unsigned)__double2loint(x), xh = (unsigned)__double2hiint(x);
  const unsigned yl = (unsigned)__double2loint(y), yh = (unsigned)__double2hiint(y);
  if constexpr (O == 32) {
    const auto rl = __builtin_amdgcn_permlane32_swap(xl, yl, false, false);
    const auto rh = __builtin_amdgcn_permlane32_swap(xh, yh, false, false);
    return __hiloint2double((int)rh[0], (int)rl[0]) + __hiloint2double((int)rh[1], (int)rl[1]);
  } else {
    const auto rl = __builtin_amdgcn_permlane16_swap(xl, yl, false, false);
    const auto rh = __builtin_amdgcn_permlane16_swap(xh, yh, false, false);
    return __hiloint2double((int)rh[0], (int)rl[0]) + __hiloint2double((int)rh[1], (int)rl[1]);
  }
}

// One butterfly level per template instance (each level owns a fresh,
// statically indexed array, which keeps every value in registers).
// v[0..H) per lane at level STEP (lane bit 32 >> STEP is reduced next);
// after the last level lds_wave[base + q] holds the wave total of index
// base + q, written by the lanes whose all-reduced bits (dup) are zero.
template <int H, int STEP>
__device__ __forceinline__ void wave_level(const double (&v)[H], double* lds_wave, int lane,
                                           int base, int dup) {
  if constexpr (STEP == 6) {
    if ((lane & dup) == 0) {
#pragma unroll
      for (int q = 0; q < H; ++q) lds_wave[base + q] = v[q];
    }
  } else {
    constexpr int O = 32 >> STEP;
    if constexpr (H % 2 == 0) {
      constexpr int HH = H / 2;
      const bool up = (lane & O) != 0;
      double w[HH];
      if constexpr (O == 32 || O == 16) {
#pragma unroll
        for (int q = 0; q < HH; ++q) w[q] = swap_sum<O>(v[q], v[q + HH]);
      } else {
#pragma unroll
        for (int q = 0; q < HH; ++q) {
          const double xs = v[q] + __shfl_xor(v[q], O, 64);
          const double ys = v[q + HH] + __shfl_xor(v[q + HH], O, 64);
          w[q] = up ? ys : xs;
        }
      }
      wave_level<HH, STEP + 1>(w, lds_wave, lane, base + (up ? HH : 0), dup);
    } else {
      double w[H];
#pragma unroll
      for (int q = 0; q < H; ++q) w[q] = v[q] + __shfl_xor(v[q], O, 64);
      wave_level<H, STEP + 1>(w, lds_wave, lane, base, dup | O);
    }
  }
}

// v[0..MP) per lane; on return lds_wave[idx] holds the wave total of idx.
template <int MP>
__device__ __forceinline__ void wave_reduce_to_lds(const double (&v)[MP], double* lds_wave,
                                                   int lane) {
  wave_level<MP, 0>(v, lds_wave, lane, 0, 0);
}

// ---------------------------------------------------------------------------
// Per-thread velocity of velocity index j.
// ---------------------------------------------------------------------------
struct Vel {
  int b[3];
  double u[3];
  double w;  // trapezoid weight
};

__device__ __forceinline__ Vel velocity_of(const DevGeom& g, int64_t j) {
  Vel v;
  v.b[0] = (int)(j % g.nv1[0]);
  v.b[1] = (int)((j / g.nv1[0]) % g.nv1[1]);
  v.b[2] = (int)(j / ((int64_t)g.nv1[0] * g.nv1[1]));
  double w = 1.0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    v.u[c] = g.vlo[c] + v.b[c] * g.du[c];
    double wc = g.du[c];
    if (v.b[c] == 0 || v.b[c] == g.nv1[c] - 1) wc *= 0.5;
    w *= wc;
  }
  v.w = w;
  return v;
}

template <typename ST> struct Compute;
template <> struct Compute<double> { using T = double; };
template <> struct Compute<float> { using T = float; };

// Moment partials of one element's NS node values (per lane), written for
// this work-group's velocity chunk into partials[(node)*nchunk + chunk][5].
// Values of lanes outside the grid must enter with w = 0.
template <int NS, typename CT>
__device__ __forceinline__ void element_partials(const CT (&fv)[NS], const Vel& vel,
                                                 double* __restrict__ partials, int64_t node0,
                                                 int nchunk, int chunk, double* lds) {
  // groups of nodes bound the register footprint of the reduction
  constexpr int G = group_of(NS);
  constexpr int M = 5 * G;
  constexpr int MP = best_pad(M);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double psi4 = 0.5 * (vel.u[0] * vel.u[0] + vel.u[1] * vel.u[1] + vel.u[2] * vel.u[2]);
#pragma unroll
  for (int g0 = 0; g0 < NS; g0 += G) {
    double v[MP];
#pragma unroll
    for (int q = 0; q < G; ++q) {
      const double wf = vel.w * (double)fv[g0 + q];
      v[5 * q + 0] = wf;
      v[5 * q + 1] = wf * vel.u[0];
      v[5 * q + 2] = wf * vel.u[1];
      v[5 * q + 3] = wf * vel.u[2];
      v[5 * q + 4] = wf * psi4;
    }
#pragma unroll
    for (int q = M; q < MP; ++q) v[q] = 0.0;
    wave_reduce_to_lds<MP>(v, lds + wave * MP, lane);
    __syncthreads();
    for (int t = threadIdx.x; t < M; t += blockDim.x) {
      double s = lds[t];
      for (int w = 1; w < (int)(blockDim.x >> 6); ++w) s += lds[w * MP + t];
      const int q = t / 5, m = t % 5;
      partials[((node0 + g0 + q) * nchunk + chunk) * 5 + m] = s;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Stage kernel: FR transport (volume + upwind inflow-face lift) + BGK
// relaxation + SSP-RK combine + positivity limiter + next-stage moment
// partials (MODE 0), or the plain residual L(f) in FP64 (MODE 1).
// ---------------------------------------------------------------------------
template <int DIM, int P, typename ST, int MODE>
__global__ void __launch_bounds__(kBlock) k_stage(const StageArgs A) {
  using CT = typename Compute<ST>::T;
  constexpr int N1 = P + 1;
  constexpr int NS = ipow(N1, DIM);
  __shared__ double lds[(kBlock / 64) * best_pad(5 * group_of(NS))];

  const DevGeom& g = A.g;
  const int64_t w = xcd_remap(blockIdx.x, gridDim.x);
  const int chunk = (int)(w / A.ecount);
  const int64_t e = A.e0 + (w % A.ecount);
  const int64_t nv = g.nv;
  const int64_t j = (int64_t)chunk * kBlock + threadIdx.x;
  const bool valid = j < nv;
  const int64_t jj = valid ? j : nv - 1;
  Vel vel = velocity_of(g, jj);
  if (!valid) vel.w = 0.0;

  const ST* __restrict__ fin = (const ST*)A.fin;
  const ST* fe = fin + (e * NS) * nv + jj;
  CT f[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) f[i] = (CT)fe[(int64_t)i * nv];

  CT acc[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) acc[i] = (CT)0;

  // element coordinates (uniform over the work-group)
  int ek[3] = {0, 0, 0};
  {
    int64_t r = e;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      ek[k] = (int)(r % g.nelem[k]);
      r /= g.nelem[k];
    }
  }

#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    int S = 1;
#pragma unroll
    for (int m = 0; m < k; ++m) S *= N1;
    const CT a = (CT)(vel.u[k] * g.scale[k]);
    const bool pos = a > (CT)0;
    // upwind neighbour along k: left one when a > 0, right one otherwise
    const int side = pos ? 0 : 1;
    int nk = ek[k] + (pos ? -1 : 1);
    bool wall = false;
    if (nk < 0 || nk >= g.nelem[k]) {
      if (g.bc[k][side] != 0) wall = true;
      nk = (nk + g.nelem[k]) % g.nelem[k];
    }
    int64_t src_e = e;
    int64_t src_j = jj;
    if (wall) {
      // specular wall: own element at the velocity with component k mirrored
      int bm[3] = {vel.b[0], vel.b[1], vel.b[2]};
      bm[k] = g.nv1[k] - 1 - bm[k];
      src_j = bm[0] + (int64_t)g.nv1[0] * (bm[1] + (int64_t)g.nv1[1] * bm[2]);
    } else {
      int64_t stride = 1;
      for (int m = 0; m < k; ++m) stride *= g.nelem[m];
      src_e = e + (int64_t)(nk - ek[k]) * stride;
    }
    // exterior trace: right trace of the left neighbour (a > 0), left trace
    // of the right neighbour (a < 0); at a wall the own trace on that side
    const bool use_right = (pos != wall);
    const ST* src = fin + (src_e * NS) * nv + src_j;
#pragma unroll
    for (int base = 0; base < NS; ++base) {
      if ((base / S) % N1 != 0) continue;
      CT line[N1];
#pragma unroll
      for (int bb = 0; bb < N1; ++bb) line[bb] = f[base + bb * S];
      CT own = (CT)0, ext = (CT)0;
#pragma unroll
      for (int bb = 0; bb < N1; ++bb) {
        const CT lL = (CT)A.op.lamL[bb], lR = (CT)A.op.lamR[bb];
        own += (pos ? lL : lR) * line[bb];
        ext += (use_right ? lR : lL) * (CT)src[(int64_t)(base + bb * S) * nv];
      }
      const CT jump = a * (ext - own);
#pragma unroll
      for (int ia = 0; ia < N1; ++ia) {
        CT df = (CT)0;
#pragma unroll
        for (int bb = 0; bb < N1; ++bb) df += (CT)A.op.D[ia][bb] * line[bb];
        const CT G = pos ? (CT)A.op.GL[ia] : (CT)A.op.GR[ia];
        acc[base + ia * S] += a * df + jump * G;
      }
    }
  }

  // BGK relaxation towards the discretely conservative equilibrium
  // g = exp(alpha . psi) (FP64 argument and exponential)
  const double psi4 = 0.5 * (vel.u[0] * vel.u[0] + vel.u[1] * vel.u[1] + vel.u[2] * vel.u[2]);
  const int64_t node0 = e * NS;
  CT L[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    CT c = (CT)0;
    if (A.collide) {
      const double* pr = A.params + (node0 + i) * 8;
      const double arg = pr[0] + pr[1] * vel.u[0] + pr[2] * vel.u[1] + pr[3] * vel.u[2] + pr[4] * psi4;
      const CT gq = (CT)exp(arg);
      c = (gq - f[i]) * (CT)pr[5];
    }
    L[i] = -acc[i] + c;
  }

  if constexpr (MODE == 1) {
    double* out = (double*)A.out;
    if (valid) {
      double* oe = out + ((e - A.out_e0) * NS) * nv + j;
#pragma unroll
      for (int i = 0; i < NS; ++i) oe[(int64_t)i * nv] = (double)L[i];
    }
    if (threadIdx.x == 0 && blockIdx.x == 0) atomicAdd(&A.diag[4], 1ull);
  } else {
    const CT dt = (CT)A.dt, ca = (CT)A.a, cb = (CT)A.b;
    CT o[NS];
    if (A.a != 0.0) {
      const ST* fn = (const ST*)A.fn + (e * NS) * nv + jj;
#pragma unroll
      for (int i = 0; i < NS; ++i) o[i] = ca * (CT)fn[(int64_t)i * nv] + cb * (f[i] + dt * L[i]);
    } else {
#pragma unroll
      for (int i = 0; i < NS; ++i) o[i] = cb * (f[i] + dt * L[i]);
    }
    if (A.limiter) {
      double mean = 0.0;
      CT fmin = o[0];
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        mean += A.op.W[i] * (double)o[i];
        fmin = o[i] < fmin ? o[i] : fmin;
      }
      mean /= A.op.Wsum;
      const bool hit = valid && (fmin < (CT)0);
      if (hit && mean != (double)fmin) {
        double beta = fabs(mean / (mean - (double)fmin));
        beta = beta > 1.0 ? 1.0 : beta;
#pragma unroll
        for (int i = 0; i < NS; ++i) o[i] = (CT)(mean + beta * ((double)o[i] - mean));
      }
      const unsigned long long nh = __popcll(__ballot(hit));
      const unsigned long long nb = __popcll(__ballot(hit && !(mean > 0.0)));
      if ((threadIdx.x & 63) == 0 && nh) {
        atomicAdd(&A.diag[2], nh);
        if (nb) atomicAdd(&A.diag[3], nb);
      }
    }
    ST* out = (ST*)A.out;
    if (valid) {
      ST* oe = out + (e * NS) * nv + j;
#pragma unroll
      for (int i = 0; i < NS; ++i) oe[(int64_t)i * nv] = (ST)o[i];
    }
    // moment partials of what was stored (FP64 sums)
    CT os[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) os[i] = (CT)(ST)o[i];
    element_partials<NS, CT>(os, vel, A.partials, node0, g.nchunk, chunk, lds);
    if (threadIdx.x == 0 && blockIdx.x == 0) atomicAdd(&A.diag[4], 1ull);
  }
}

// Moment partials of a stored state (first stage after installation).
template <int DIM, int P, typename ST>
__global__ void __launch_bounds__(kBlock) k_moments(const StageArgs A) {
  using CT = typename Compute<ST>::T;
  constexpr int N1 = P + 1;
  constexpr int NS = ipow(N1, DIM);
  __shared__ double lds[(kBlock / 64) * best_pad(5 * group_of(NS))];
  const DevGeom& g = A.g;
  const int64_t w = xcd_remap(blockIdx.x, gridDim.x);
  const int chunk = (int)(w / A.ecount);
  const int64_t e = A.e0 + (w % A.ecount);
  const int64_t nv = g.nv;
  const int64_t j = (int64_t)chunk * kBlock + threadIdx.x;
  const bool valid = j < nv;
  const int64_t jj = valid ? j : nv - 1;
  Vel vel = velocity_of(g, jj);
  if (!valid) vel.w = 0.0;
  const ST* fe = (const ST*)A.fin + (e * NS) * nv + jj;
  CT f[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) f[i] = (CT)fe[(int64_t)i * nv];
  element_partials<NS, CT>(f, vel, A.partials, e * NS, g.nchunk, chunk, lds);
}

}  // namespace bgk
