// bgk_device3d.hpp -- stage and moment kernels for hexahedral (d = 3)
// elements on gfx950 (Dzanic & Martinelli, arXiv 2308.06196, Sec. 2.1).
//
// Plane-split kernels, used where a (p+1)^3-node element does not fit one
// lane's registers: FP64 storage, and the BF16-increment stages (which hold a
// second value per neighbour node). FP32 hexahedra run the one-lane-per-
// velocity k_stage<3, ...> of bgk_device.hpp instead. Here a group of G lanes
// (G = 2 for p = 1, 4 for p = 2, 3) shares one velocity and lane g of the
// group owns the z-plane a_z = g of the element: (p+1)^2 nodes. The x and
// y operators are lane-local exactly as for quadrilaterals; the z-derivative
// and the z-face traces need the other planes of the same column, which come
// from the other lanes of the group by DPP quad permutations (no LDS, no
// barriers). A work-group of 256 lanes covers 256 / G consecutive velocity slots
// of one element. Lanes with g >= p+1 (p = 2) load nothing and store nothing.
#pragma once

#include "bgk_device.hpp"

namespace bgk {

template <int P> struct Plane3 {
  static constexpr int N1 = P + 1;
  static constexpr int G = N1 <= 2 ? 2 : 4;   // lanes per velocity
  static constexpr int VB = kBlock / G;        // velocities per work-group
  static constexpr int P2 = N1 * N1;           // nodes per plane
  static constexpr int NS = N1 * N1 * N1;
};

// Sum / min over the G lanes of a group (partners lane ^ 1, lane ^ 2; every
// lane ends with the same bits).
template <int G, typename T>
__device__ __forceinline__ T group_allsum(T x) {
  x += quad_xor<1>(x);
  if constexpr (G == 4) x += quad_xor<2>(x);
  return x;
}
template <int G, typename T>
__device__ __forceinline__ T group_allmin(T x) {
  T y = quad_xor<1>(x);
  x = y < x ? y : x;
  if constexpr (G == 4) {
    y = quad_xor<2>(x);
    x = y < x ? y : x;
  }
  return x;
}

// Moment partials of one element on the matrix cores (FP64 MFMA), as in the
// 1-D/2-D kernels: per wave and per plane pl, P[q][m] = sum over the wave's
// 64 / G velocities v of f[pl][q][v] (w psi_m)(v), a (p+1)^2 x K by K x 5
// contraction on the matrix cores (wave_moments_4x4, one 16-row tile per
// plane). Every lane stages its plane's values, the first lane of each
// velocity group stages w psi of that velocity; the four waves' results are
// added in a fixed order. `stage` is mfma3_lds_bytes<P, ST>() bytes, `red`
// 4 x NS x 5 doubles.
template <int P, typename ST>
constexpr int mfma3_lds_bytes() {
  constexpr int G = Plane3<P>::G, K = 64 / G, RS = K + 2;
  return (kBlock / 64) * (K * 5 * (int)sizeof(double) + G * 16 * RS * (int)sizeof(ST));
}

template <int P, typename ST, typename CT>
__device__ __forceinline__ void plane_partials_mfma(const CT (&fv)[Plane3<P>::P2], const Vel& vel,
                                                    double* __restrict__ partials, int64_t node0,
                                                    int64_t nx, int chunk, int lp,
                                                    unsigned char* stage, double* red,
                                                    const int tid) {
  using PL = Plane3<P>;
  constexpr int N1 = PL::N1, G = PL::G, P2 = PL::P2, NS = PL::NS;
  constexpr int K = 64 / G, RS = K + 2;
  static_assert(P2 <= 16, "the nodes of a plane fill at most one 16-row tile");
  const int lane = tid & 63, wave = tid >> 6;
  const int vw = lane / G;  // velocity of this lane inside the wave
  double* ps = reinterpret_cast<double*>(stage) + wave * K * 5;
  ST* gw = reinterpret_cast<ST*>(stage + (kBlock / 64) * K * 5 * sizeof(double)) +
           wave * G * 16 * RS;
  if (lp < N1) {
#pragma unroll
    for (int q = 0; q < P2; ++q) gw[(lp * 16 + q) * RS + vw] = (ST)fv[q];
  }
  if (lp == 0) {
    const double psi4 = 0.5 * (vel.u[0] * vel.u[0] + vel.u[1] * vel.u[1] + vel.u[2] * vel.u[2]);
    ps[vw * 5 + 0] = vel.w;
    ps[vw * 5 + 1] = vel.w * vel.u[0];
    ps[vw * 5 + 2] = vel.w * vel.u[1];
    ps[vw * 5 + 3] = vel.w * vel.u[2];
    ps[vw * 5 + 4] = vel.w * psi4;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
  wave_moments_4x4<N1, P2, K, ST>(gw, RS, ps, red + wave * NS * 5, tid);
  lds_barrier();
  for (int t = tid; t < NS * 5; t += kBlock) {
    const int node = t / 5, m = t - node * 5;
    double sum = red[node * 5 + m];
#pragma unroll
    for (int w = 1; w < kBlock / 64; ++w) sum += red[(w * NS + node) * 5 + m];
    partials[((int64_t)chunk * nx + node0 + node) * 5 + m] = sum;
  }
}


// One work item (element e x velocity chunk) of the plane-split stage. With
// SW (column sweep along z, see stage_item) the group's z-outflow traces are
// carried from the previous element of the column in LDS (one value per
// velocity and z-line, written by the group's first lane).
// The (p+1)^2 values of one plane of a neighbour (BF16-increment stages:
// F + increment).
template <int P2, bool DIN, typename CT, typename ST>
__device__ __forceinline__ void load_planes(CT (&v)[P2], const ST* src, const ST* fin,
                                            const uint16_t* din) {
#pragma unroll
  for (int q = 0; q < P2; ++q) v[q] = (CT)src[q * kVB];
  if constexpr (DIN) add_increments(v, din, src - fin);
}

template <int P, typename ST, int MODE, bool INC = false, bool SW = false>
__device__ __forceinline__ void stage3_item(const StageArgs& A, const int chunk, const int64_t e,
                                            const bool count, const bool carry, const bool up) {
  static_assert(!INC || (MODE != 1 && sizeof(ST) == 4), "increment stages: FP32 state, RK modes");
  static_assert(!SW || MODE != 1, "column sweeps: RK modes");
  using CT = typename Compute<ST>::T;
  using PL = Plane3<P>;
  constexpr bool kMfma = sizeof(CT) == 4;
  constexpr int N1 = PL::N1, G = PL::G, VB = PL::VB, P2 = PL::P2, NS = PL::NS;
  __shared__ double red[(kBlock / 64) * NS * 5];
  __shared__ FaceRows<CT> frows[kBlock / 64];
  __shared__ LineOps lops[kMfma ? kBlock / 64 : 1];
  __shared__ CT trl[SW ? P2 * VB : 1];  // carried z-traces, [line][velocity of the work-group]
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  double* tab = reinterpret_cast<double*>(dyn_lds);

  // thread index, opaque per element in a sweep (see stage_item)
  int tid = (int)threadIdx.x;
  if constexpr (SW) asm volatile("" : "+v"(tid));
  const DevGeom& g = A.g;
  const DevOpsT<CT>& OP = ops_of<CT>(A);
  FaceRows<CT>& fr = frows[tid >> 6];
  face_rows_store<CT, N1, true>(fr, OP, tid);
  LineOps& lo = lops[kMfma ? tid >> 6 : 0];
  if constexpr (kMfma) line_ops_store(lo, A.lops, tid);
  const int64_t nv = g.nv;
  const int S = g.tabw;
  const int64_t node0 = e * NS;

  const int lp = tid % G;                        // plane owned by this lane
  const bool live = lp < N1;
  const int pl = live ? lp : N1 - 1;             // address plane (idle lanes)
  const int j = chunk * VB + tid / G;
  const bool valid = j < nv;
  const bool act = valid && live;
  const int jj = valid ? j : (int)nv - 1;
  Vel vel = velocity_of<sizeof(ST) == 8>(g, jj);  // FP64: lexicographic slots
  if (!act) vel.w = 0.0;

  int ek[3];
  {
    int64_t r = e;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      ek[k] = (int)(r % g.nelem[k]);
      r /= g.nelem[k];
    }
  }
  const ST* __restrict__ fin = (const ST*)A.fin;
  const ST* src[3];
  bool pos[3], use_right[3], wall_in[3][2];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    pos[k] = vel.u[k] * g.scale[k] > 0.0;
    const int nek = sreg(g.nelem[k]);
    const bool wall_lo = sreg(g.bc[k][0]) != 0, wall_hi = sreg(g.bc[k][1]) != 0;
    wall_in[k][1] = ek[k] == 0 && wall_lo;
    wall_in[k][0] = ek[k] == nek - 1 && wall_hi;
    int nk = ek[k] + (pos[k] ? -1 : 1);
    bool wall = false;
    if (nk < 0 || nk >= nek) {
      wall = pos[k] ? wall_lo : wall_hi;
      nk = (nk + nek) % nek;
    }
    int64_t src_e = e;
    int src_j = jj;
    if (wall) {
      int bm[3] = {vel.b[0], vel.b[1], vel.b[2]};
      bm[k] = g.nv1[k] - 1 - bm[k];
      src_j = vel_slot(g, bm);
    } else {
      int64_t stride = 1;
      for (int m = 0; m < k; ++m) stride *= g.nelem[m];
      src_e = e + (int64_t)(nk - ek[k]) * stride;
    }
    use_right[k] = (pos[k] != wall);
    src[k] = fin + f_offset(g, src_e, pl * P2, src_j);
  }
  // sweep: groups whose upwind z-neighbour is the previous element of the
  // column take its carried traces; a wave loads the z-neighbour's planes only
  // when one of its groups does not (uniform)
  bool lane_carry = false, wave_load = true;
  if constexpr (SW) {
    lane_carry = carry && pos[2] == up;
    // every wave loads at the column's entry element, also one whose lanes
    // are all beyond the velocity count: their carried values must be finite
    // (they enter the moment partials with weight 0)
    wave_load = !carry || __ballot(valid && !lane_carry) != 0;
  }

  // loads: equilibrium rows (first batch), own plane, the x-, y- and
  // z-neighbours' planes, f^n plane
  // first batch of row loads: 4 x 256 entries for FP32 arithmetic, whose
  // registers are scarcer, 6 x 256 in FP64 (a 64-velocity chunk of the 16^3
  // grid at p = 3 needs 64 x 22)
  constexpr int kU = kMfma ? 4 : 6;
  const RowPick rp = row_pick(A, chunk, NS);
  const double* et = A.etab + node0 * S;
  double tv[kU];
  if (A.collide) {
#pragma unroll
    for (int u = 0; u < kU; ++u) {  // clamped, unconditional loads
      const int t = u * kBlock + tid;
      tv[u] = et[rp.offset(t < rp.count ? t : rp.count - 1)];
    }
  }
  // BF16-increment stages 2-3: the input is F + increment (same offsets)
  constexpr bool kDin = INC && MODE == 0;
  const uint16_t* __restrict__ din = A.din;
  const ST* fe = fin + f_offset(g, e, pl * P2, jj);
  CT f[P2];
#pragma unroll
  for (int q = 0; q < P2; ++q) f[q] = (CT)fe[q * kVB];
  // sweep: the z-neighbour's planes are not held (see the z part). The
  // neighbours' planes are loaded one axis at a time (the next axis' after
  // this axis' transport), so that no more than one neighbour's planes are
  // held at once: FP64 fits three waves per SIMD (167 registers against 234
  // with all loaded up front), BF16 increments four (128 against 157).
  constexpr int NB = SW ? 2 : 3;
  constexpr bool kStaged = true;
  CT nb[NB][P2];
  if constexpr (kStaged) {
    load_planes<P2, kDin>(nb[0], src[0], fin, din);
  } else {
#pragma unroll
    for (int k = 0; k < NB; ++k)
#pragma unroll
      for (int q = 0; q < P2; ++q) nb[k][q] = (CT)src[k][q * kVB];
  }
  if constexpr (kDin) {
    add_increments(f, din, fe - fin);
    if constexpr (!kStaged) {
#pragma unroll
      for (int k = 0; k < NB; ++k) add_increments(nb[k], din, src[k] - fin);
    }
  }

  if (A.collide) {
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int t = u * kBlock + tid;
      if (t < rp.count) tab[t] = tv[u];
    }
  }

  CT acc[P2];
#pragma unroll
  for (int q = 0; q < P2; ++q) acc[q] = (CT)0;

  // x and y: lines inside the plane, lane-local (FP32 arithmetic on the matrix
  // cores, see line_mfma: a block of four lanes is one velocity's planes for
  // p >= 2, two velocities for p = 1)
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    if (kStaged && k > 0) {  // keep the scheduler from hoisting these loads
      __builtin_amdgcn_sched_barrier(0);
      load_planes<P2, kDin>(nb[k], src[k], fin, din);
    }
    const int S1 = k == 0 ? 1 : N1;
    const CT a = (CT)(vel.u[k] * g.scale[k]);
    if constexpr (kMfma) {
      const bool uni = quads_agree(pos[k]);
      const int npass = uni ? 1 : 2;
      for (int ps = 0; ps < npass; ++ps) {
        const int sg = uni ? (pos[k] ? 1 : 0) : ps;
        const int ur = sg ? (wall_in[k][1] ? 0 : 1) : (wall_in[k][0] ? 1 : 0);
        float dp[4], ev[4];
        line_ops_row(lo, sg, ur, tid, dp, ev);
        const CT as = (uni || (pos[k] ? 1 : 0) == sg) ? a : (CT)0;
#pragma unroll
        for (int base = 0; base < P2; ++base) {
          if ((base / S1) % N1 != 0) continue;
          float fl[N1], nl[N1];
#pragma unroll
          for (int bb = 0; bb < N1; ++bb) {
            fl[bb] = f[base + bb * S1];
            nl[bb] = nb[k][base + bb * S1];
          }
          const mfma_f4 c = line_mfma<N1>(dp, ev, fl, nl);
#pragma unroll
          for (int ia = 0; ia < N1; ++ia) acc[base + ia * S1] = fmaf(as, c[ia], acc[base + ia * S1]);
        }
      }
      continue;
    }
    CT lown[N1], lext[N1], Gin[N1];
    {
      const CT* ro = fr.r[pos[k] ? 1 : 0];
      const CT* re = fr.r[use_right[k] ? 0 : 1];
#pragma unroll
      for (int bb = 0; bb < N1; ++bb) {
        lown[bb] = ro[bb];
        Gin[bb] = ro[kMaxN1 + bb];
        lext[bb] = re[bb];
      }
    }
#pragma unroll
    for (int base = 0; base < P2; ++base) {
      if ((base / S1) % N1 != 0) continue;
      CT line[N1];
#pragma unroll
      for (int bb = 0; bb < N1; ++bb) line[bb] = f[base + bb * S1];
      CT own = (CT)0, ext = (CT)0;
#pragma unroll
      for (int bb = 0; bb < N1; ++bb) {
        own += lown[bb] * line[bb];
        ext += lext[bb] * nb[k][base + bb * S1];
      }
      const CT jump = a * (ext - own);
#pragma unroll
      for (int ia = 0; ia < N1; ++ia) {
        CT df = (CT)0;
#pragma unroll
        for (int bb = 0; bb < N1; ++bb) df += sreg(OP.D[ia][bb]) * line[bb];
        acc[base + ia * S1] += a * df + jump * Gin[ia];
      }
    }
  }
  if constexpr (kStaged && !SW) {
    __builtin_amdgcn_sched_barrier(0);
    load_planes<P2, kDin>(nb[NB - 1], src[2], fin, din);
  }
  // z: the column of node q is spread over the group's lanes; lane lp holds
  // plane lp and its partners lane ^ r the other planes. The derivative is
  // sum_r D[lp][lp ^ r] f(lp ^ r); the trace difference ext - own is one
  // group sum of lext(lp) f_nb - lown(lp) f (zero weights on idle lanes).
  {
    const CT a = (CT)(vel.u[2] * g.scale[2]);
    const CT* ro = fr.r[pos[2] ? 1 : 0];
    const CT* re = fr.r[use_right[2] ? 0 : 1];
    const CT lown_mine = live ? ro[pl] : (CT)0;
    const CT lext_mine = live ? re[pl] : (CT)0;
    const CT lout_mine = live ? fr.r[up ? 0 : 1][pl] : (CT)0;  // sweep: outflow trace weight
    const int vg = tid / G;                                 // velocity inside the work-group
    const CT ag = a * ro[kMaxN1 + pl];
    // sweep: every group takes its z-exterior traces from trl; where a wave
    // has groups that do not carry, those groups first put there the traces
    // formed from the z-neighbour's planes
    if constexpr (SW) {
      if (wave_load) {
#pragma unroll
        for (int q = 0; q < P2; ++q) {
          CT v = (CT)src[2][q * kVB];
          if constexpr (kDin) v += increment_of<P2>(din, src[2] - fin, q);
          const CT t = group_allsum<G>(lext_mine * v);
          if (!lane_carry) trl[q * VB + vg] = t;
        }
      }
    }
    CT Dr[G];
#pragma unroll
    for (int r = 0; r < G; ++r) {
      const int b = lp ^ r;
      Dr[r] = live && b < N1 ? fr.D[pl * kMaxN1 + b] : (CT)0;
    }
#pragma unroll
    for (int q = 0; q < P2; ++q) {
      const CT fq = f[q];
      CT df = Dr[0] * fq;
      df += Dr[1] * quad_xor<1>(fq);
      if constexpr (G == 4) {
        df += Dr[2] * quad_xor<2>(fq);
        df += Dr[3] * quad_xor<3>(fq);
      }
      CT jl;
      if constexpr (SW) {
        jl = trl[q * VB + vg] - group_allsum<G>(lown_mine * fq);
        // outflow trace of this line for the next element of the column
        // (every lane of the group writes the same value)
        trl[q * VB + vg] = group_allsum<G>(lout_mine * fq);
      } else {
        jl = group_allsum<G>(lext_mine * nb[NB - 1][q] - lown_mine * fq);
      }
      acc[q] += a * df + ag * jl;
    }
  }

  // relaxation folded with the transport into h = b (f - dt T) + b dt C
  // before f^n is loaded (as in stage_item: C in FP64 from the FP64 rows,
  // added in FP64), all inside the branch that loads the rows
  // positions of this velocity's factors in a node's LDS row (compact)
  const int cx = vel.b[0] - rp.x0, oy = rp.nx + vel.b[1] - rp.y0,
            oz = rp.nxy + vel.b[2] - rp.z0;
  const double* tp = tab + pl * P2 * rp.ncols;  // rows of this lane's plane
  double* oe1 = nullptr;                 // residual output (MODE 1)
  if constexpr (MODE == 1) {
    const int jc = vel.b[0] + g.nv1[0] * (vel.b[1] + g.nv1[1] * vel.b[2]);
    oe1 = (double*)A.out + ((e - A.out_e0) * NS + pl * P2) * nv + jc;
  }
  const CT dt = (CT)A.dt, ca = (CT)A.a, cb = (CT)A.b;
  const double wc = A.b * A.dt;
  if (A.collide) {  // uniform: rows beyond the first batch, then the relaxation
    table_rest<kU>(tab, et, rp, tid);
    lds_barrier();
#pragma unroll
    for (int q = 0; q < P2; ++q) {
      const double c = collision_term(tp + q * rp.ncols, cx, oy, oz, rp.ncols, (double)f[q]);
      if constexpr (MODE == 1) {
        if (act) oe1[(int64_t)q * nv] = c - (double)acc[q];
      } else if constexpr (sizeof(CT) == 8) {  // h, kept in acc
        acc[q] = fma(wc, c, cb * (f[q] - dt * acc[q]));
      } else {
        acc[q] = (CT)fma(wc, c, (double)(cb * (f[q] - dt * acc[q])));
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < P2; ++q) {
      if constexpr (MODE == 1) {
        if (act) oe1[(int64_t)q * nv] = -(double)acc[q];
      } else {
        acc[q] = cb * (f[q] - dt * acc[q]);
      }
    }
  }
  // f^n (MODE 0; a stream, see stage_item), or F of the own nodes, the base
  // of the BF16 increments (read again: a cache hit)
  CT fnv[P2];
  // keep the scheduler from hoisting these loads above the relaxation
  __builtin_amdgcn_sched_barrier(0);
  if constexpr (INC) {
#pragma unroll
    for (int q = 0; q < P2; ++q) fnv[q] = (CT)fe[q * kVB];
  } else if constexpr (MODE == 0) {
    const ST* fn = (const ST*)A.fn + f_offset(g, e, pl * P2, jj);
#pragma unroll
    for (int q = 0; q < P2; ++q) fnv[q] = (CT)__builtin_nontemporal_load(&fn[q * kVB]);
  }
  CT o[P2];
  if constexpr (MODE != 1) {
#pragma unroll
    for (int q = 0; q < P2; ++q) o[q] = MODE == 0 ? ca * fnv[q] + acc[q] : acc[q];
  }

  if constexpr (MODE == 1) {
    if (tid == 0 && count) atomicAdd(&A.diag[4], 1ull);
  } else {
    if (A.limiter) {
      // element mean and minimum over all planes of the velocity
      CT wz = (CT)0;  // Gauss weight of this lane's plane
#pragma unroll
      for (int bb = 0; bb < N1; ++bb) wz = bb == lp ? sreg(OP.w[bb]) : wz;
      CT part = wz * tensor_wsum<2, N1>(o, OP.w);
      CT fmin = o[0];
#pragma unroll
      for (int q = 0; q < P2; ++q) fmin = o[q] < fmin ? o[q] : fmin;
      if (!live) {
        part = (CT)0;
        fmin = (CT)INFINITY;
      }
      const CT mean = group_allsum<G>(part) / OP.Wsum;
      fmin = group_allmin<G>(fmin);
      const bool hit = valid && (fmin < (CT)0);
      if (hit && mean != fmin) {
        CT beta = fabs(mean / (mean - fmin));
        beta = beta > (CT)1 ? (CT)1 : beta;
#pragma unroll
        for (int q = 0; q < P2; ++q) o[q] = mean + beta * (o[q] - mean);
      }
      const unsigned long long nh = __popcll(__ballot(hit && lp == 0));
      const unsigned long long nb2 = __popcll(__ballot(hit && lp == 0 && !(mean > (CT)0)));
      if ((tid & 63) == 0 && nh) {
        atomicAdd(&A.diag[2], nh);
        if (nb2) atomicAdd(&A.diag[3], nb2);
      }
    }
    if constexpr (INC) {
      // the increment o - F in BF16, and the stored state F + increment for
      // the partials; the last stage stores o itself in FP32
      if (A.out_full) {
        if (act) {
          ST* oe = (ST*)A.out + f_offset(g, e, pl * P2, j);
#pragma unroll
          for (int q = 0; q < P2; ++q) __builtin_nontemporal_store((ST)o[q], &oe[q * kVB]);
        }
      } else {
        static_assert(P2 % 2 == 0, "BF16 planes hold whole node pairs");
        uint32_t* ow = inc_pairs((uint16_t*)A.out, f_offset(g, e, pl * P2, jj));
        float omin = INFINITY, smin = INFINITY;  // stage values / stored values
        uint32_t hp = 0;
#pragma unroll
        for (int q = 0; q < P2; ++q) {
          float stored;
          const uint16_t h = bf16_increment(o[q], fnv[q], stored);
          if (q % 2 == 0) {
            hp = h;
          } else if (act) {
            __builtin_nontemporal_store(hp | ((uint32_t)h << 16), &ow[(q >> 1) * kVB]);
          }
          omin = fminf(omin, o[q]);
          smin = fminf(smin, stored);
          o[q] = stored;
        }
        // (velocity, plane) pairs whose stored stage is negative where the
        // stage itself is not
        const unsigned long long nviol = __popcll(__ballot(act && smin < 0.0f && !(omin < 0.0f)));
        if ((tid & 63) == 0 && nviol) atomicAdd(&A.diag[5], nviol);
      }
    } else if (act) {
      ST* oe = (ST*)A.out + f_offset(g, e, pl * P2, j);
#pragma unroll
      for (int q = 0; q < P2; ++q) __builtin_nontemporal_store((ST)o[q], &oe[q * kVB]);
    }
    // moment partials on the matrix cores; the staging area reuses the
    // equilibrium rows' LDS once every wave is done with them
    if (A.collide) lds_barrier();
    plane_partials_mfma<P, ST, CT>(o, vel, A.partials, node0, g.nx, chunk, lp, dyn_lds, red, tid);
    if (tid == 0 && count) atomicAdd(&A.diag[4], 1ull);
  }
}

// Waves per SIMD of the plane-split kernels: three in FP64, four in FP32
// arithmetic (the neighbours' planes loaded one axis at a time); the FP64
// sweep keeps two (its loop spills at three).
template <typename CT, bool SW>
constexpr int plane_waves() {
  return sizeof(CT) == 8 ? (SW ? 2 : 3) : 4;
}

template <int P, typename ST, int MODE, bool INC = false>
__global__ void __launch_bounds__(kBlock)
    __attribute__((amdgpu_waves_per_eu(plane_waves<typename Compute<ST>::T, false>())))
    k_stage3(const StageArgs A) {
  const int64_t w = xcd_chunk_remap(blockIdx.x, gridDim.x, A.ecount, A.xcd_part);
  stage3_item<P, ST, MODE, INC>(A, (int)(w / A.ecount), work_element(A.order, A.e0, w, A.ecount),
                                w == 0, false, false);
}

// Plane-split stage as column sweeps along z (see k_stage_sweep).
template <int P, typename ST, int MODE, bool INC = false>
__global__ void __launch_bounds__(kBlock)
    __attribute__((amdgpu_waves_per_eu(plane_waves<typename Compute<ST>::T, true>())))
    k_stage3_sweep(const StageArgs A) {
  const DevGeom& g = A.g;
  const int nl = sreg(g.nelem[2]), seg = sreg(A.sweep_seg);
  const int64_t ncol = g.ne / nl, nseg = nl / seg, per_chunk = ncol * nseg;
  const int64_t w = xcd_chunk_remap(blockIdx.x, gridDim.x, per_chunk, A.xcd_part);
  const int chunk = (int)(w / per_chunk);
  const int64_t r = w - (int64_t)chunk * per_chunk;
  const int64_t sg = r / ncol, col = r - sg * ncol;
  const bool up = sweep_up(g, chunk * Plane3<P>::VB);
  // arguments re-read per element (see k_stage_sweep)
  table_ptr<StageArgs> ap = (table_ptr<StageArgs>)__builtin_amdgcn_kernarg_segment_ptr();
  for (int s = 0; s < seg; ++s) {
    const int el = (int)(sg * seg) + s;
    const int64_t e = col + (int64_t)(up ? el : nl - 1 - el) * ncol;
    if (s > 0 && !A.collide) lds_barrier();
    asm volatile("" : "+s"(ap));
    stage3_item<P, ST, MODE, INC, true>(table_entry(ap, 0), chunk, e, w == 0 && s == 0, s > 0, up);
  }
}

template <int P, typename ST>
__global__ void __launch_bounds__(kBlock) k_moments3(const StageArgs A) {
  using CT = typename Compute<ST>::T;
  using PL = Plane3<P>;
  constexpr int N1 = PL::N1, G = PL::G, VB = PL::VB, P2 = PL::P2, NS = PL::NS;
  __shared__ double red[(kBlock / 64) * NS * 5];
  extern __shared__ __align__(16) unsigned char dyn_lds[];  // MFMA staging
  const DevGeom& g = A.g;
  const int64_t w = xcd_remap(blockIdx.x, gridDim.x);
  const int chunk = (int)(w / A.ecount);
  const int64_t e = work_element(A.order, A.e0, w, A.ecount);
  const int64_t nv = g.nv;
  const int lp = (int)threadIdx.x % G;
  const bool live = lp < N1;
  const int pl = live ? lp : N1 - 1;
  const int j = chunk * VB + (int)threadIdx.x / G;
  const bool valid = j < nv;
  const int jj = valid ? j : (int)nv - 1;
  Vel vel = velocity_of<sizeof(ST) == 8>(g, jj);  // FP64: lexicographic slots
  if (!(valid && live)) vel.w = 0.0;
  const ST* fe = (const ST*)A.fin + f_offset(g, e, pl * P2, jj);
  CT f[P2];
#pragma unroll
  for (int q = 0; q < P2; ++q) f[q] = (CT)fe[q * kVB];
  plane_partials_mfma<P, ST, CT>(f, vel, A.partials, e * NS, g.nx, chunk, lp, dyn_lds, red,
                                 (int)threadIdx.x);
}

}  // namespace bgk
