// bgk_device.hpp -- gfx950 kernels of the discrete-velocity Boltzmann-BGK
// hot path (Dzanic & Martinelli, arXiv 2308.06196, Sec. 2 and Sec. 2.1).
//
// Data layout in HBM (one solver):
//   f[elem][vblock][node][64]  storage precision; velocities in blocks of
//                        kVB = 64 (f_offset), so a wave reads one contiguous
//                        block per element and node offsets are immediates
//                        (the ABI exchanges f[elem][node][vel], converted)
//   partials[chunk][node][5]  FP64 moment partial sums of one stage output,
//                        one entry per velocity chunk of a work-group (chunk
//                        major, so a work-group writes one contiguous block)
//   params[node][8]      FP64 (alpha_0..alpha_4, 1/tau, tau, status) of the
//                        discretely conservative equilibrium
//   etab[node][S]        one-dimensional factors of that equilibrium and
//                        1/tau, in the precision of the stage arithmetic,
//                        S = nv1[0] + nv1[1] + nv1[2] + 1:
//                        g(u) = Ex[bx] Ey[by] Ez[bz] with
//                        Ex[b] = exp(alpha_0 + alpha_1 u_b + alpha_4 u_b^2/2),
//                        Ey[b] = exp(alpha_2 u_b + alpha_4 u_b^2/2), Ez alike;
//                        the last entry of a row is 1/tau of the node
//
// Thread mapping of the stage kernel: one work-group = one element x one
// chunk of 256 consecutive velocity slots; one lane = one velocity slot j and all
// (p+1)^d nodes of the element, held in registers (quadrilaterals, and
// hexahedra in FP32; the plane-split hexahedral kernels are in
// bgk_device3d.hpp). The FR operators are
// (p+1)-point contractions along element lines (sum factorisation, VALU);
// they are far below the FP64/FP32 ridge point, so the kernel is bound by
// HBM traffic and instruction issue, not by arithmetic peak.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bgk {

constexpr int kMaxN1 = 4;            // p <= 3
constexpr int kBlock = 256;          // velocities per work-group
constexpr int kNumXCD = 8;           // MI355X: 8 accelerator complex dies
constexpr int kMaxTabBytes = 65536;  // LDS for one element's equilibrium factors

struct DevGeom {
  int32_t dim, n1, ns;
  int32_t nelem[3];
  int32_t bc[3][2];
  int32_t nv1[3];
  int32_t tabw;  // S = nv1[0] + nv1[1] + nv1[2] + 1 (factors, then 1/tau)
  int64_t ne, nx, nv;
  int64_t nvb;  // velocity blocks of kVB per element (internal layout)
  int32_t nchunk;
  double vlo[3], du[3];
  double scale[3];  // 2 / h_k
  // Internal velocity order (slots): the velocities are grouped by the signs
  // of their transported components, octant o = s0 + 2 s1 + 4 s2 after
  // octant, lexicographic (component 0 fastest) inside an octant. vsplit[k]
  // is the number of nodes with u_k <= 0 on a transported axis (0 on the
  // others: a single half), voct[o] the first slot of octant o (voct[8] = nv).
  // Every upwind choice is then uniform over runs of many slots, so a wave's
  // neighbour loads read whole cache lines of one element.
  int32_t vsplit[3];
  int32_t voct[9];
};

// Internal state layout: f[element][velocity block][node][kVB], blocks of
// kVB consecutive velocity slots (the slot order is described at DevGeom; the
// last block padded). The values one wave reads
// for one node are kVB consecutive entries and the nodes of an element are kVB
// entries apart, so a wave streams one contiguous block per element and node
// offsets fit in the load instructions. Offset of (element e, node a of the
// element, velocity slot j).
constexpr int kVB = 64;
__host__ __device__ __forceinline__ int64_t f_offset(const DevGeom& g, int64_t e, int a,
                                                     int64_t j) {
  return ((e * g.nvb + j / kVB) * g.ns + a) * kVB + j % kVB;
}

template <typename T>
struct DevOpsT {
  T D[kMaxN1][kMaxN1];  // D[a][b] = l_b'(xi_a)
  T lamL[kMaxN1], lamR[kMaxN1];
  T GL[kMaxN1], GR[kMaxN1];  // correction-function slopes at the nodes
  T w[kMaxN1];               // 1-D Gauss weights (node weights are products)
  T Wsum;                    // sum of the node weights
};
using DevOps = DevOpsT<double>;

// FR line operators for the matrix-core contraction (FP32 arithmetic). For a
// velocity with u_k > 0 (pos = 1) the inflow face of an element is its left
// face, and the transport of one line of p+1 nodes along axis k is
//   T = a (Dp f_own + E f_nb),   Dp = D - G_in lam_own^T,   E = G_in lam_ext^T,
// a = u_k 2/h_k, with (lam_own, G_in) = (lamL, GL) where pos and (lamR, GR)
// otherwise, and lam_ext = lamR where use_right (the upwind neighbour's right
// trace, or the own trace at a right wall), lamL otherwise: the volume
// derivative plus the inflow-face correction of the upwind common flux
// (Sec. 2.1, correction functions recovering nodal DG). Rows and columns
// beyond p+1 are zero.
struct alignas(16) LineOps {
  float Dp[2][4][4];    // [pos][row i][column k]
  float E[2][2][4][4];  // [pos][use_right][row i][column k]
  float G[2][4];        // [pos][row i]: G_in, for a given exterior trace
};
constexpr int kLineOpsFloats = (int)(sizeof(LineOps) / sizeof(float));

// Entries of an element's equilibrium rows that one work-group reads: the
// factors of the velocity nodes its slots use on each axis (node ranges
// [x0, x0 + nx), [y0, y0 + ny), [z0, z0 + nz)) and 1/tau; ncols = nx + ny +
// nz + 1 entries per spatial node, magic = ceil(2^32 / ncols) for the
// division of a compact index by ncols.
struct RowCols {
  int32_t x0, nx, y0, ny, z0, nz, ncols, magic;
};

struct StageArgs {
  DevGeom g;
  DevOps op;
  DevOpsT<float> opf;  // the same operators rounded to FP32 (FP32 arithmetic)
  const void* fin;  // stage input (storage precision)
  const void* fn;   // f^n (storage precision), read when a != 0
  void* out;        // stage output (storage precision), or FP64 residual
  const double* params;
  const double* etab;    // equilibrium factor rows (FP64)
  const int32_t* order;  // traversal order of the elements (null: lexicographic)
  double* partials;
  unsigned long long* diag;  // newton it max, newton fail, lim hits, lim bad, stages
  double dt, a, b;
  int64_t e0, ecount, out_e0;
  int32_t limiter, collide;
  // diffuse walls (1-D/2-D): wallp[k][s][8] = ((2 pi theta_w)^{-3/2},
  // 1/(2 theta_w), U_w, 1/(incoming flux of the unit wall Maxwellian)), the
  // re-emitted density of every wall flux point, and the offset of side
  // (k, s) in it (-1: not a diffuse wall)
  const double* wallp;
  const double* wall_rho;
  int32_t wall_off[2][2];
  // BF16-increment stages (FP32 state F, stage increments in BF16): the
  // stage input is F + din (din null in the first stage), and the output is
  // the increment o - F in BF16, or o itself in FP32 when out_full is set
  const uint16_t* din;
  int32_t out_full;
  LineOps lops;  // FR line operators for the matrix-core contraction (FP32)
  // row entries read by velocity chunk c: rcols[c & rc_mask] (rc_mask 0: one
  // entry for every chunk)
  const RowCols* rcols;
  int32_t rc_mask;
  int32_t sweep_seg;  // column sweeps: elements per work item along the last axis
  int32_t xcd_part;   // XCDs per chunk group of xcd_chunk_remap (else xcd_remap)
};

// BF16 <-> FP32: the upper half of the FP32 bit pattern; rounding to nearest,
// ties to even (finite inputs).
__device__ __forceinline__ float bf16_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// BF16 increment buffers pair the nodes of a velocity block: the increments
// of nodes 2m and 2m + 1 of a velocity share one 32-bit word (node 2m in the
// low half), word m * 64 + lane of the pair's 128 halves, so that a lane
// reads or writes two node values with one access; an odd last node of the
// block keeps its 64 halves (one per lane). The buffers have the state's
// size and block offsets. off = f_offset of an even node a of a block at the
// lane; the words of nodes a + 2m, a + 2m + 1 follow at m * 64.
__device__ __forceinline__ const uint32_t* inc_pairs(const uint16_t* d, int64_t off) {
  return (const uint32_t*)(d + (off & ~(int64_t)(kVB - 1))) + (off & (kVB - 1));
}
__device__ __forceinline__ uint32_t* inc_pairs(uint16_t* d, int64_t off) {
  return (uint32_t*)(d + (off & ~(int64_t)(kVB - 1))) + (off & (kVB - 1));
}
__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }
// v[i] += increment of node a + i, i < N (N odd: the block's last nodes)
template <int N, typename CT>
__device__ __forceinline__ void add_increments(CT (&v)[N], const uint16_t* d, int64_t off) {
  const uint32_t* w = inc_pairs(d, off);
#pragma unroll
  for (int m = 0; m < N / 2; ++m) {
    const uint32_t x = w[m * kVB];
    v[2 * m] += bf16_lo(x);
    v[2 * m + 1] += bf16_hi(x);
  }
  if constexpr (N % 2 != 0) v[N - 1] += bf16_f32(d[off + (N - 1) * kVB]);
}
// increment of node a + i alone (i < N, as above)
template <int N>
__device__ __forceinline__ float increment_of(const uint16_t* d, int64_t off, int i) {
  if (N % 2 != 0 && i == N - 1) return bf16_f32(d[off + i * kVB]);
  const uint32_t x = inc_pairs(d, off)[(i >> 1) * kVB];
  return (i & 1) ? bf16_hi(x) : bf16_lo(x);
}
__device__ __forceinline__ uint16_t f32_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Diffuse walls: outgoing mass flux per wall flux point and velocity chunk
// (k_wall_flux), then the re-emitted density per flux point (k_wall_rho).
// Sides are listed in order; side q covers nface[q] elements of the wall,
// each with (p+1)^(d-1) flux points starting at off[q] in wall_rho.
struct WallArgs {
  DevGeom g;
  double lamL[kMaxN1], lamR[kMaxN1];
  const void* fin;       // stage input (storage precision)
  const double* wallp;   // [k][s][8], see StageArgs
  double* part;          // [flux point][chunk] partial sums
  double* rho;           // [flux point] re-emitted density
  int32_t nside;
  int32_t side_k[4], side_s[4], off[4], nface[4];
  int32_t blk0[5];       // first block of every side (k_wall_flux)
  int32_t npoints;       // flux points over all sides
};

struct NewtonArgs {
  DevGeom g;
  const double* partials;
  double* params;
  double* etab;  // equilibrium factor rows (FP64)
  double* Q;   // optional [nx][5] output of the reduced moments
  unsigned long long* diag;
  double gamma, mu_ref, theta_ref, omega, tol;
  double sutherland;  // > 0: Sutherland constant (power law otherwise)
  int32_t maxit, collide;
  int32_t continuous;  // 1: continuous Maxwellian of (rho, U, theta), no Newton solve
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

// Linear block id -> work id with groups of `part` XCDs (8, 4 or 2) sharing
// one velocity chunk at a time: XCD x of group x / part takes the
// (x % part)-th share of every chunk the group walks, so that the XCDs of a
// group hold neighbouring work items of one chunk together and a neighbour
// read that misses one XCD's L2 finds nodes that another XCD has just
// fetched into the memory-side cache. per_chunk work items per chunk,
// nb = chunks x per_chunk; other part values or sizes: contiguous ranges.
__device__ __forceinline__ int64_t xcd_chunk_remap(int64_t bid, int64_t nb, int64_t per_chunk,
                                                   int32_t part) {
  if (part != 2 && part != 4 && part != 8) return xcd_remap(bid, nb);
  const int ng = kNumXCD / part;
  if (per_chunk % part != 0 || (nb / per_chunk) % ng != 0) return xcd_remap(bid, nb);
  const int64_t x = bid % kNumXCD, k = bid / kNumXCD;
  const int64_t s = per_chunk / part, r = k / s;
  const int64_t c = r * ng + x / part;
  return c * per_chunk + (x % part) * s + (k - r * s);
}

// Element of work item w (velocity-chunk major): the k-th element of the
// traversal order, which visits hexahedra brick by brick so that the
// upwind neighbours of an element were visited a few work items earlier.
__device__ __forceinline__ int64_t work_element(const int32_t* order, int64_t e0, int64_t w,
                                                int64_t ecount) {
  const int64_t k = w % ecount;
  return order ? (int64_t)order[k] : e0 + k;
}

// DPP moves whose source lanes are all valid (permutations inside a row), so
// no previous value is needed (bound_ctrl set); the compiler can then fold
// the move into the consuming add or multiply.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}

// Partner value across lane bit O (O <= 8) by a DPP move.
template <int O, typename T>
__device__ __forceinline__ T dpp_partner(T x) {
  return dpp_mov<O == 8 ? 0x128 : O == 4 ? 0x141 : O == 2 ? 0x4E : 0xB1>(x);
}

// Value of lane (lane ^ R) inside the quad, R < 4.
template <int R, typename T>
__device__ __forceinline__ T quad_xor(T x) {
  return dpp_mov<R == 1 ? 0xB1 : R == 2 ? 0x4E : 0x1B>(x);
}

// ---------------------------------------------------------------------------
// Per-lane velocity of velocity slot j (32-bit index arithmetic).
// ---------------------------------------------------------------------------
struct Vel {
  int b[3];
  double u[3];
  double w;  // trapezoid weight
};

// Slot order of a velocity grid (g.dim, nv1, vlo, du set): with octants, the
// split of transported axis k is the number of nodes with u_k <= 0, by the
// same u_k = vlo_k + b du_k > 0 test the stage kernels make; without, every
// split is 0 and the slots are the lexicographic indices.
inline void set_velocity_slots(DevGeom& g, bool octants) {
  for (int k = 0; k < 3; ++k) {
    int m = 0;
    if (octants && k < g.dim)
      while (m < g.nv1[k] && !(g.vlo[k] + m * g.du[k] > 0.0)) ++m;
    g.vsplit[k] = m;
  }
  int off = 0;
  for (int o = 0; o < 8; ++o) {
    g.voct[o] = off;
    int sz = 1;
    for (int k = 0; k < 3; ++k) sz *= (o >> k) & 1 ? g.nv1[k] - g.vsplit[k] : g.vsplit[k];
    off += sz;
  }
  g.voct[8] = off;  // nv
}

// Slot of the velocity with node indices b (the order described at DevGeom).
__host__ __device__ __forceinline__ int vel_slot(const DevGeom& g, const int (&b)[3]) {
  int o = 0, l[3], n[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int hi = b[k] >= g.vsplit[k] ? 1 : 0;
    o |= hi << k;
    l[k] = b[k] - (hi ? g.vsplit[k] : 0);
    n[k] = hi ? g.nv1[k] - g.vsplit[k] : g.vsplit[k];
  }
  return g.voct[o] + l[0] + n[0] * (l[1] + n[1] * l[2]);
}

// Slot of canonical velocity index jc = b0 + N0 (b1 + N1 b2).
__host__ __device__ __forceinline__ int vel_slot_of_canonical(const DevGeom& g, int jc) {
  const int r = jc / g.nv1[0];
  const int b[3] = {jc - r * g.nv1[0], r % g.nv1[1], r / g.nv1[1]};
  return vel_slot(g, b);
}

// Node indices b of slot j (the inverse of vel_slot).
__host__ __device__ __forceinline__ void slot_nodes(const DevGeom& g, int j, int (&b)[3]) {
  // octant: the last one starting at or before j (empty octants start where
  // the next one does, so they are never picked)
  int o = 0;
#pragma unroll
  for (int q = 1; q < 8; ++q) o = j >= g.voct[q] ? q : o;
  int n[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) n[k] = (o >> k) & 1 ? g.nv1[k] - g.vsplit[k] : g.vsplit[k];
  const int loc = j - g.voct[o], r = loc / n[0], l2 = r / n[1];
  const int l[3] = {loc - r * n[0], r - l2 * n[1], l2};
#pragma unroll
  for (int k = 0; k < 3; ++k) b[k] = l[k] + ((o >> k) & 1 ? g.vsplit[k] : 0);
}

// LEX: the grid has a single octant (slots are the lexicographic indices),
// decoded with the grid's own, uniform divisors.
template <bool LEX = false>
__device__ __forceinline__ Vel velocity_of(const DevGeom& g, int j) {
  Vel v;
  if constexpr (LEX) {
    const int r = j / g.nv1[0];
    v.b[0] = j - r * g.nv1[0];
    v.b[2] = r / g.nv1[1];
    v.b[1] = r - v.b[2] * g.nv1[1];
  } else {
    slot_nodes(g, j, v.b);
  }
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

// Uniform kernel-argument value as an opaque scalar register value: a
// per-lane select between two of them then stays a register select (the
// compiler would otherwise turn it into a load through a selected address).
// Work-group barrier that orders LDS only. A plain __syncthreads() also
// orders global memory, so it waits for every load and store in flight (the
// bulk loads issued ahead of the table stores, the output stores ahead of the
// reduction); this one waits for LDS operations alone.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Face coefficients for the upwind selection, one copy per wave in LDS:
// row 1 holds (lamL, GL), used where u_k > 0 (inflow through the left face),
// row 0 holds (lamR, GR); then the derivative matrix, for kernels that need
// a per-lane row of it. A lane reads its row through a per-lane address;
// picking between two uniform values per lane in registers would take two
// moves and a select per 32-bit half (one scalar operand per VALU op).
template <typename CT>
struct alignas(16) FaceRows {
  CT r[2][2 * kMaxN1];
  CT D[kMaxN1 * kMaxN1];  // D[a][b] at a kMaxN1 + b, zero outside the element
};

template <typename CT, int N1, bool WITH_D = false>
__device__ __forceinline__ void face_rows_store(FaceRows<CT>& fr, const DevOpsT<CT>& OP,
                                                const int tid) {
  if ((tid & 63) == 0) {
#pragma unroll
    for (int b = 0; b < N1; ++b) {
      fr.r[0][b] = OP.lamR[b];
      fr.r[0][kMaxN1 + b] = OP.GR[b];
      fr.r[1][b] = OP.lamL[b];
      fr.r[1][kMaxN1 + b] = OP.GL[b];
    }
    if constexpr (WITH_D) {
#pragma unroll
      for (int a = 0; a < kMaxN1; ++a)
#pragma unroll
        for (int b = 0; b < kMaxN1; ++b) fr.D[a * kMaxN1 + b] = a < N1 && b < N1 ? OP.D[a][b] : CT(0);
    }
  }
  // the other lanes of this wave read what lane 0 wrote (LDS is ordered
  // within a wave; the fences keep the compiler from moving the reads up)
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

__device__ __forceinline__ double sreg(double x) {
  const int lo = __builtin_amdgcn_readfirstlane(__double2loint(x));
  const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(x));
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float sreg(float x) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
__device__ __forceinline__ int sreg(int x) { return __builtin_amdgcn_readfirstlane(x); }

template <typename ST> struct Compute;
template <> struct Compute<double> { using T = double; };
template <> struct Compute<float> { using T = float; };

// sum_i W_i v_i over the (p+1)^D nodes of a D-dimensional tensor block
// (D = 1, 2), W_i the product of the 1-D Gauss weights of node i, summed one
// dimension at a time.
template <int D, int N1, typename CT>
__device__ __forceinline__ CT tensor_wsum(const CT* v, const CT* w) {
  if constexpr (D == 1) {
    CT s = (CT)0;
#pragma unroll
    for (int a = 0; a < N1; ++a) s += sreg(w[a]) * v[a];
    return s;
  } else {
    CT s = (CT)0;
#pragma unroll
    for (int b = 0; b < N1; ++b) s += sreg(w[b]) * tensor_wsum<D - 1, N1>(v + b * N1, w);
    return s;
  }
}

// Operators in the arithmetic type (kernel arguments, uniform over the grid).
template <typename CT>
__device__ __forceinline__ const DevOpsT<CT>& ops_of(const StageArgs& A) {
  if constexpr (sizeof(CT) == 8) return A.op;
  else return A.opf;
}

// The row entries a work-group loads, numbered compactly: entry t is node
// a = t / ncols, column c = t - a ncols of the needed ones (x factors, y
// factors, z factors, 1/tau). It is read from offset(t) = a S + column of the
// element's rows and kept at LDS index t, so a node's entries in LDS are a
// row of ncols values: x factor of velocity node bx at bx - x0, y factor at
// nx + by - y0, z factor at nx + ny + bz - z0, 1/tau last. t / ncols is the
// high word of t magic, exact while t ncols < 2^32 (t < 8192 entries of 8 B
// fit LDS).
struct RowPick {
  int S, x0, y0, z0, oy, oz, nx, nxy, nxyz, ncols, count;
  uint32_t magic;
  __device__ __forceinline__ int offset(int t) const {
    const int a = (int)__umulhi((unsigned)t, magic);
    const int c = t - a * ncols;
    const int col = c < nx ? x0 + c : c < nxy ? oy + (c - nx) : c < nxyz ? oz + (c - nxy) : S - 1;
    return a * S + col;
  }
};

__device__ __forceinline__ RowPick row_pick(const StageArgs& A, int chunk, int ns) {
  const RowCols rc = A.rcols[chunk & A.rc_mask];  // global memory: scalar loads
  RowPick r;
  r.S = A.g.tabw;
  r.x0 = rc.x0;
  r.y0 = rc.y0;
  r.z0 = rc.z0;
  r.oy = A.g.nv1[0] + rc.y0;
  r.oz = A.g.nv1[0] + A.g.nv1[1] + rc.z0;
  r.nx = rc.nx;
  r.nxy = rc.nx + rc.ny;
  r.nxyz = rc.nx + rc.ny + rc.nz;
  r.ncols = rc.ncols;
  r.magic = (uint32_t)rc.magic;
  r.count = ns * rc.ncols;
  return r;
}

// Row entries from compact index kU * kBlock on (the first kU * kBlock are
// loaded with the bulk loads) -> LDS index t.
template <int kU>
__device__ __forceinline__ void table_rest(double* tab, const double* et, const RowPick& rp,
                                           const int tid) {
  for (int t0 = kU * kBlock; t0 < rp.count; t0 += kU * kBlock) {
    double v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int t = t0 + u * kBlock + tid;
      v[u] = et[rp.offset(t < rp.count ? t : rp.count - 1)];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int t = t0 + u * kBlock + tid;
      if (t < rp.count) tab[t] = v[u];
    }
  }
}

// Moment partials of one element as an FP64 matrix product on the matrix
// cores: per wave, P[node][m] = sum over the wave's 64 velocities v of
// f[node][v] * (w psi_m)(v), a 16 x 64 by 64 x 5 contraction. The operands
// need velocity across the K index, so each lane first writes its column (its
// velocity's node values, and w psi of its velocity) to LDS; wave_moments_4x4
// reads the operands back and runs the products. The four waves' tiles are
// then added in a fixed order. `stage` is the work-group's MFMA staging area
// (mfma_lds_bytes<ST>() bytes: 16 rows per wave, one tile of 16 nodes at a
// time), `red` 4 x part_rows<NS>() x 5 doubles.
constexpr int kGst = 66;  // LDS row stride (elements) of the staged node values
template <typename ST>
constexpr int mfma_lds_bytes() {
  return (kBlock / 64) * (64 * 5 * (int)sizeof(double) + 16 * kGst * (int)sizeof(ST));
}
typedef double mfma_d4 __attribute__((ext_vector_type(4)));

// Moment sums of the values one wave staged in LDS:
//   redw[n][m] = sum_{v < K} F[n][v] W[v][m],  m < 5,
// with F in rows of `gw` (row stride rs; NT tiles of 16 rows of which the
// first NV are used, node n = t NV + r for row 16 t + r) and W in `ps`
// ([v][5], FP64). On v_mfma_f64_4x4x4_4b, block b of one instruction takes
// four rows (nodes) and four moments for four velocities; the energy moment
// takes a second instruction with the same A operand. Operand layout of
// block b: A[i][k] in lane 16k + 4b + i, B[k][j] in lane 16k + 4b + j; the
// result D[i][j] lands in lane 16i + 4b + j. (FP64 MFMA has the FP64 vector
// rate here, so the 16x16x4 shape, with 11 of its 16 columns idle for five
// moments, would take twice the matrix-core cycles.)
template <int NT, int NV, int K, typename ST>
__device__ __forceinline__ void wave_moments_4x4(const ST* gw, int rs, const double* ps,
                                                 double* redw, const int tid) {
  static_assert(NV <= 16 && K % 4 == 0, "tiles of 16 rows, velocities in fours");
  const int lane = tid & 63;
  const int k = lane >> 4, blk = (lane >> 2) & 3, j = lane & 3;
  const int ra = 4 * blk + j;  // A row of this lane inside a tile
  double d0[NT], d1[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) d0[t] = d1[t] = 0.0;
  // operands of up to 8 steps are read before the first of them is used
  // (B once per batch, A one tile at a time)
  constexpr int kB = K / 4 < 8 ? K / 4 : 8;
#pragma unroll
  for (int s0 = 0; s0 < K / 4; s0 += kB) {
    double b0[kB], b1[kB];
#pragma unroll
    for (int st = 0; st < kB; ++st) {
      const int v = 4 * (s0 + st) + k;
      b0[st] = ps[v * 5 + j];
      b1[st] = j == 0 ? ps[v * 5 + 4] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      double a[kB];
#pragma unroll
      for (int st = 0; st < kB; ++st) {
        const int v = 4 * (s0 + st) + k;
        a[st] = ra < NV ? (double)gw[(16 * t + ra) * rs + v] : 0.0;
      }
#pragma unroll
      for (int st = 0; st < kB; ++st) {
        d0[t] = __builtin_amdgcn_mfma_f64_4x4x4f64(a[st], b0[st], d0[t], 0, 0, 0);
        d1[t] = __builtin_amdgcn_mfma_f64_4x4x4f64(a[st], b1[st], d1[t], 0, 0, 0);
      }
    }
  }
  const int rd = 4 * blk + k;  // result row of this lane inside a tile
  if (rd < NV) {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      double* o = redw + (t * NV + rd) * 5;
      o[j] = d0[t];
      if (j == 0) o[4] = d1[t];
    }
  }
}

// Rows of the per-wave partial sums of an element of NS nodes (tiles of 16).
template <int NS>
constexpr int part_rows() {
  return (NS + 15) / 16 * 16;
}

// Tile T of 16 nodes: stage the values, then the products (the staging rows
// are reused by the next tile once this wave has read them).
template <int T, int NS, typename ST, typename CT>
__device__ __forceinline__ void element_tiles(const CT (&fv)[NS], ST* gw, const double* ps,
                                              double* redw, const int tid) {
  if constexpr (16 * T < NS) {
    constexpr int NV = NS - 16 * T < 16 ? NS - 16 * T : 16;
    const int lane = tid & 63;
#pragma unroll
    for (int i = 0; i < NV; ++i) gw[i * kGst + lane] = (ST)fv[16 * T + i];
    // the lanes of this wave read what the others wrote (LDS is ordered
    // within a wave; the fences keep the compiler from moving accesses across)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
    wave_moments_4x4<1, NV, 64, ST>(gw, kGst, ps, redw + 16 * T * 5, tid);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
    element_tiles<T + 1, NS, ST, CT>(fv, gw, ps, redw, tid);
  }
}

template <int NS, typename ST, typename CT>
__device__ __forceinline__ void element_partials_mfma(const CT (&fv)[NS], const Vel& vel,
                                                      double* __restrict__ partials,
                                                      int64_t node0, int64_t nx, int chunk,
                                                      unsigned char* stage, double* red,
                                                      const int tid) {
  constexpr int NR = part_rows<NS>();
  const int lane = tid & 63, wave = tid >> 6;
  double* ps = reinterpret_cast<double*>(stage) + wave * 64 * 5;
  ST* gw = reinterpret_cast<ST*>(stage + (kBlock / 64) * 64 * 5 * sizeof(double)) + wave * 16 * kGst;
  const double psi4 = 0.5 * (vel.u[0] * vel.u[0] + vel.u[1] * vel.u[1] + vel.u[2] * vel.u[2]);
  ps[lane * 5 + 0] = vel.w;
  ps[lane * 5 + 1] = vel.w * vel.u[0];
  ps[lane * 5 + 2] = vel.w * vel.u[1];
  ps[lane * 5 + 3] = vel.w * vel.u[2];
  ps[lane * 5 + 4] = vel.w * psi4;
  element_tiles<0, NS, ST, CT>(fv, gw, ps, red + wave * NR * 5, tid);
  lds_barrier();
  for (int t = tid; t < 5 * NS; t += kBlock) {
    const int node = t / 5, m = t - node * 5;
    double sum = red[node * 5 + m];
#pragma unroll
    for (int w = 1; w < kBlock / 64; ++w) sum += red[(w * NR + node) * 5 + m];
    partials[((int64_t)chunk * nx + node0 + node) * 5 + m] = sum;
  }
}

// BGK collision term at one (node, velocity) in FP64 (Sec. 2, C = (g - f)/tau;
// Sec. 2.1, g the discretely conservative equilibrium): from the node's FP64
// equilibrium row ti (Ex with exp(alpha_0) and 1/tau folded in, Ey, Ez, then
// 1/tau at ti[S - 1]) and the velocity's row offsets. Every stage kernel, in
// every storage precision, forms the collision term with this function, so
// its discrete moments vanish to FP64 rounding (the conservation the Newton
// solve of the equilibrium reaches); bgk_collision_moments measures them with
// the same function.
__device__ __forceinline__ double collision_term(const double* ti, int bx, int oy, int oz, int S,
                                                 double f) {
  return fma(-f, ti[S - 1], ti[bx] * ti[oy] * ti[oz]);
}

// Stored BF16 increment of a stage value o over the FP32 base F, and the
// value F + increment that the next stage reads. A non-negative increment is
// rounded to nearest (ties to even); a negative one is truncated towards zero,
// so that F + increment >= o up to the FP32 rounding of o - F: where o >= 0
// and F >= 0 the stored stage is exactly >= 0, since o - F >= -F rounds to a
// value >= -F and truncation only shrinks it. The stored stages thus keep the
// positivity the limiter of Sec. 2.1 establishes (rounding to nearest could
// put F + increment below zero by up to 2^-9 F where the limiter has just
// lifted a node to zero). Returns the bits.
__device__ __forceinline__ uint16_t bf16_increment(float o, float base, float& stored) {
  const float d = o - base;
  const uint32_t u = __float_as_uint(d);
  const uint16_t h = (u & 0x80000000u) ? (uint16_t)(u >> 16) : f32_bf16(d);
  stored = base + bf16_f32(h);
  return h;
}


typedef float mfma_f4 __attribute__((ext_vector_type(4)));

// One line on v_mfma_f32_4x4x1_16b_f32: block b of the instruction takes lanes
// 4b..4b+3 (four velocities); its A operand (4 x 1) comes from those lanes'
// registers (row i from lane 4b + i), its B operand (1 x 4) and its result
// column j from lane 4b + j. With A = column k of the operator (row lane & 3,
// read by every lane from the same table) and B = the lane's own value of node
// k of the line, the result column of a lane is the operator applied to its
// own line: a lane-local (p+1)-point contraction, with the blocks of four
// velocities sharing the operator (the layout was checked on the device with
// distinct operands in every lane).
template <int N1>
__device__ __forceinline__ mfma_f4 line_mfma(const float (&dp)[4], const float (&ev)[4],
                                             const float (&fl)[N1], const float (&nl)[N1]) {
  mfma_f4 c = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int k = 0; k < N1; ++k) c = __builtin_amdgcn_mfma_f32_4x4x1f32(dp[k], fl[k], c, 0, 0, 0);
#pragma unroll
  for (int k = 0; k < N1; ++k) c = __builtin_amdgcn_mfma_f32_4x4x1f32(ev[k], nl[k], c, 0, 0, 0);
  return c;
}

// The own part Dp f_own of one line (see line_mfma).
template <int N1>
__device__ __forceinline__ mfma_f4 line_mfma_own(const float (&dp)[4], const float (&fl)[N1]) {
  mfma_f4 c = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int k = 0; k < N1; ++k) c = __builtin_amdgcn_mfma_f32_4x4x1f32(dp[k], fl[k], c, 0, 0, 0);
  return c;
}

// Column sweep: the outflow traces of the element's lines along the last
// axis (stride NT between the nodes of a line), sum_b lout[b] f(line node b),
// lout = lamR where the sweep runs towards +x_k (the downwind element's
// exterior trace is this element's right trace) and lamL otherwise; kept in
// registers (tr) or in this lane's column of trl.
template <int N1, int NT, bool LDS, typename CT, int NS, int R>
__device__ __forceinline__ void sweep_store(const CT* lout, const CT (&f)[NS], CT* trl,
                                            CT (&tr)[R], const int tid) {
  CT lo[N1];
#pragma unroll
  for (int bb = 0; bb < N1; ++bb) lo[bb] = lout[bb];
#pragma unroll
  for (int base = 0; base < NT; ++base) {
    CT t = (CT)0;
#pragma unroll
    for (int bb = 0; bb < N1; ++bb) t += lo[bb] * f[base + bb * NT];
    if constexpr (LDS) trl[base * kBlock + tid] = t;
    else tr[base] = t;
  }
}

// Copy the line operators to this wave's LDS copy (read back through per-lane
// addresses).
__device__ __forceinline__ void line_ops_store(LineOps& lo, const LineOps& src, const int tid) {
  const int lane = tid & 63;
  const float* s = reinterpret_cast<const float*>(&src);
  float* d = reinterpret_cast<float*>(&lo);
  for (int t = lane; t < kLineOpsFloats; t += 64) d[t] = s[t];
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// Operator columns of this lane's row for table sign sg and trace side ur.
__device__ __forceinline__ void line_ops_row(const LineOps& lo, int sg, int ur, const int tid,
                                             float (&dp)[4],
                                             float (&ev)[4]) {
  const int i = tid & 3;
  const float4 d = *reinterpret_cast<const float4*>(&lo.Dp[sg][i][0]);
  const float4 e = *reinterpret_cast<const float4*>(&lo.E[sg][ur][i][0]);
  dp[0] = d.x, dp[1] = d.y, dp[2] = d.z, dp[3] = d.w;
  ev[0] = e.x, ev[1] = e.y, ev[2] = e.z, ev[3] = e.w;
}

// True when every aligned group of four lanes of the wave agrees on pos, so
// that one operator per block serves all its velocities (always the case in
// the slot order of the grids whose sign octants hold multiples of four
// velocities).
__device__ __forceinline__ bool quads_agree(bool pos) {
  const int v = pos ? 1 : 0;
  const int a = __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true);
  const int b = __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true);
  return __ballot(a != v || b != v) == 0;
}

// Waves per SIMD the stage kernel is built for: segments and quadrilaterals 5
// with FP32 storage (6-7 % faster than 4 on the 32^2 p = 3 box) and with BF16
// increments (one 32-bit load per two node increments; 3 spilled registers
// in stages 2-3 at p = 3, 2.5 % faster than 4 on that box, where one 16-bit
// load per increment spilled enough to double the time), 3 in FP64; hexahedra (one lane per velocity with all
// (p+1)^3 nodes) 4 at p = 2 in FP32 arithmetic (128 registers without
// spills since the relaxation is formed before f^n is loaded; Mach-2 box
// 19.8 against 21.2 ms at three) and 2 in FP64 (three spill and took 2.5x as
// long), 2 at p = 3 (measured: a few spilled registers at p = 3 cost less
// than halving the waves).
template <int DIM, int P, typename CT, bool INC>
constexpr int stage_waves() {
  return DIM == 3 && P == 3 ? 2
         : DIM == 3 && P == 2 ? (sizeof(CT) == 8 ? 2 : 4)
         : sizeof(CT) == 8 ? 3 : 5;
}

// ---------------------------------------------------------------------------
// Stage kernel: FR transport (volume + upwind inflow-face lift) + BGK
// relaxation + SSP-RK combine + positivity limiter + next-stage moment
// partials (MODE 0: a stage that combines with f^n; MODE 3: the first stage,
// a = 0, which does not read f^n), or the plain residual L(f) in FP64
// (MODE 1). Dynamic LDS: NS * S FP64 values (equilibrium rows).
//
// FP64 arithmetic runs the line contractions on the VALU. FP32 arithmetic
// (FP32 storage and BF16 increments) runs them on the matrix cores
// (line_mfma), with the relaxation term formed in FP64 and added to the FP32
// stage combination in FP64 before the stored value is rounded.
// ---------------------------------------------------------------------------
// One work item (element e x velocity chunk) of one stage launch; k_stage runs
// one item per work-group, k_stage_batch one member's item from a descriptor
// table, k_stage_sweep a column of items along the last axis.
//
// Column sweep (SW): the work-group visits the elements of a column in the
// upwind direction `up` of the last axis (KS = DIM - 1) of its velocity chunk
// and hands each element's outflow traces on that axis to the next one, so
// that lanes with sign(u_KS) = up read no neighbour nodes on that axis: the
// exterior trace of a line is the carried value (`carry`: not the first
// element of the column). tr holds the carried traces in registers (1-D lines
// of quadrilaterals, NTR = p + 1 values); hexahedra keep them in LDS (NTR = 1).
// The carried trace is the same sum, in the same order, as the exterior trace
// formed from the neighbour's nodes, so the VALU paths give the same bits with
// and without the sweep.
template <int DIM, int P>
constexpr int sweep_tr_regs() {
  return DIM == 2 ? P + 1 : 1;
}
template <int DIM, int P, typename ST, int MODE, bool INC = false, bool SW = false>
__device__ __forceinline__ void stage_item(const StageArgs& A, const int chunk, const int64_t e,
                                           const bool count, const bool carry, const bool up,
                                           typename Compute<ST>::T (&tr)[sweep_tr_regs<DIM, P>()]) {
  static_assert(!INC || (MODE != 1 && sizeof(ST) == 4), "increment stages: FP32 state, RK modes");
  static_assert(!SW || (DIM >= 2 && MODE != 1), "column sweeps: quadrilaterals and hexahedra, RK modes");
  using CT = typename Compute<ST>::T;
  // FR line contractions on the matrix cores for FP32 arithmetic on p = 3
  // hexahedra (measured 2-4 % faster there); segments, quadrilaterals and
  // p < 3 hexahedra keep them on the VALU, which measured faster (2-D box:
  // 0.60 against 0.76 ms per stage; Mach-2 box, p = 2: 20.6 against 21.8 ms)
  constexpr bool kMfma = sizeof(CT) == 4 && DIM == 3 && P == 3;
  constexpr int N1 = P + 1;
  constexpr int NS = ipow(N1, DIM);
  // the upwind neighbours' nodes are held in registers, one axis at a time,
  // when they fit the register budget (1-D and 2-D elements); otherwise each
  // value is read where it is used
  constexpr bool kPreload = NS * DIM <= 48;
  constexpr int KS = DIM - 1;                 // sweep axis
  constexpr int NT = ipow(N1, DIM - 1);       // lines along it
  constexpr bool kTrLds = SW && sweep_tr_regs<DIM, P>() < NT;
  __shared__ double red[(kBlock / 64) * part_rows<NS>() * 5];
  __shared__ FaceRows<CT> frows[kBlock / 64];
  __shared__ LineOps lops[kMfma ? kBlock / 64 : 1];
  __shared__ CT trl[kTrLds ? NT * kBlock : 1];  // carried traces, [line][lane]
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  double* tab = reinterpret_cast<double*>(dyn_lds);

  // thread index; in a sweep it is opaque to the compiler for every element
  // of the column, so that what derives from it (the lane's velocity, LDS
  // addresses) is recomputed per element instead of being held in registers
  // across the column (which spilled)
  int tid = (int)threadIdx.x;
  if constexpr (SW) asm volatile("" : "+v"(tid));
  const DevGeom& g = A.g;
  const DevOpsT<CT>& OP = ops_of<CT>(A);
  FaceRows<CT>& fr = frows[tid >> 6];
  face_rows_store<CT, N1>(fr, OP, tid);
  LineOps& lo = lops[kMfma ? tid >> 6 : 0];
  if constexpr (kMfma) line_ops_store(lo, A.lops, tid);
  const int64_t nv = g.nv;
  const int S = g.tabw;
  const int64_t node0 = e * NS;

  const int j = chunk * kBlock + tid;
  const bool valid = j < nv;
  const int jj = valid ? j : (int)nv - 1;
  Vel vel = velocity_of(g, jj);
  if (!valid) vel.w = 0.0;

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

  // Per axis: the upwind neighbour (left one when u_k > 0, right one
  // otherwise) or, at a specular wall, the own element at the velocity with
  // component k mirrored; the exterior trace is the neighbour's right trace
  // (u_k > 0), its left trace (u_k < 0), or the own trace on the wall side.
  // At a diffuse wall the exterior state is the re-emitted wall Maxwellian
  // (dif[k]; the loads then read the own element and go unused).
  const ST* __restrict__ fin = (const ST*)A.fin;
  const ST* src[DIM];
  bool pos[DIM], use_right[DIM], dif[DIM], wall_in[DIM][2];
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    pos[k] = vel.u[k] * g.scale[k] > 0.0;
    const int nek = sreg(g.nelem[k]);
    const bool wall_lo = sreg(g.bc[k][0]) != 0, wall_hi = sreg(g.bc[k][1]) != 0;
    // a wall on the inflow side of the element, for either sign of u_k
    wall_in[k][1] = ek[k] == 0 && wall_lo;
    wall_in[k][0] = ek[k] == nek - 1 && wall_hi;
    int nk = ek[k] + (pos[k] ? -1 : 1);
    bool wall = false;
    if (nk < 0 || nk >= nek) {
      wall = pos[k] ? wall_lo : wall_hi;
      nk = (nk + nek) % nek;
    }
    dif[k] = wall && (pos[k] ? sreg(g.bc[k][0]) : sreg(g.bc[k][1])) == 2;
    int64_t src_e = e;
    int src_j = jj;
    if (dif[k]) {
      // own element, own velocity (unused values)
    } else if (wall) {
      int bm[3] = {vel.b[0], vel.b[1], vel.b[2]};
      bm[k] = g.nv1[k] - 1 - bm[k];
      src_j = vel_slot(g, bm);
    } else {
      int64_t stride = 1;
      for (int m = 0; m < k; ++m) stride *= g.nelem[m];
      src_e = e + (int64_t)(nk - ek[k]) * stride;
    }
    use_right[k] = (pos[k] != wall);
    src[k] = fin + f_offset(g, src_e, 0, src_j);
  }
  // sweep: lanes whose upwind neighbour on axis KS is the previous element of
  // the column take its carried traces; a wave loads that neighbour's nodes
  // only when one of its lanes does not (uniform)
  bool lane_carry = false, wave_load = true;
  if constexpr (SW) {
    lane_carry = carry && pos[KS] == up;
    // every wave loads at the column's entry element, also one whose lanes
    // are all beyond the velocity count: their carried values must be finite
    // (they enter the moment partials with weight 0)
    wave_load = !carry || __ballot(valid && !lane_carry) != 0;
  }

  // Global loads in three batches, each issued before any of its values is
  // used: (1) the element's equilibrium rows (factors and 1/tau, first
  // batch), own nodes and the axis-0 upwind neighbour's nodes; (2) the next
  // axis' neighbour after the axis-0 transport (its registers are then free:
  // 142 instead of 213 VGPRs at p = 3 in FP64, three waves per SIMD); (3) f^n
  // after the transport. Every lane loads (clamped index, no branch): a
  // conditional load makes the compiler wait for it right there.
  constexpr int kU = 2;  // covers the row entries of a 1-D or 2-D chunk (ns x ncols <= 512)
  const RowPick rp = row_pick(A, chunk, NS);
  const double* et = A.etab + node0 * S;
  double tv[kU];
  if (A.collide) {
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int t = u * kBlock + tid;
      tv[u] = et[rp.offset(t < rp.count ? t : rp.count - 1)];
    }
  }
  // BF16-increment stages: the input of stages 2-3 is F + increment (same
  // offsets). F of the own nodes (the base of the stored increment, and the
  // f^n of the combine) stays in registers for small elements and is read
  // again (a cache hit) for hexahedra.
  constexpr bool kDin = INC && MODE == 0;
  constexpr bool kKeepF = INC && NS <= 16;
  const uint16_t* __restrict__ din = A.din;
  const ST* fe = fin + f_offset(g, e, 0, jj);
  CT f[NS];
  CT fb[kKeepF ? NS : 1];
#pragma unroll
  for (int i = 0; i < NS; ++i) f[i] = (CT)fe[i * kVB];
  if constexpr (kKeepF) {
#pragma unroll
    for (int i = 0; i < NS; ++i) fb[i] = f[i];
  }
  if constexpr (kDin) add_increments(f, din, fe - fin);
  CT nbv[kPreload ? DIM : 1][kPreload ? NS : 1];
  if constexpr (kPreload) {
#pragma unroll
    for (int i = 0; i < NS; ++i) nbv[0][i] = (CT)src[0][i * kVB];
    if constexpr (kDin) add_increments(nbv[0], din, src[0] - fin);
  }
  // the needed entries of this element's equilibrium rows -> LDS
  if (A.collide) {
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int t = u * kBlock + tid;
      if (t < rp.count) tab[t] = tv[u];
    }
  }

  CT acc[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) acc[i] = (CT)0;

#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    int S1 = 1;
#pragma unroll
    for (int m = 0; m < k; ++m) S1 *= N1;
    // the neighbour's nodes on this axis are needed (uniform)
    const bool ld = !SW || k != KS || wave_load;
    if constexpr (kPreload) {
      if (k > 0) {  // batch (2): keep the scheduler from hoisting these loads
        __builtin_amdgcn_sched_barrier(0);
        if (ld) {
#pragma unroll
          for (int i = 0; i < NS; ++i) nbv[k][i] = (CT)src[k][i * kVB];
          if constexpr (kDin) add_increments(nbv[k], din, src[k] - fin);
        }
      }
    }
    // value of node i of the upwind (or wall) neighbour on axis k
    auto nbval = [&](int i) -> CT {
      if constexpr (kPreload) {
        return nbv[k][i];
      } else {
        CT xv = (CT)src[k][i * kVB];
        if constexpr (kDin) xv += increment_of<NS>(din, src[k] - fin, i);
        return xv;
      }
    };
    // sweep axis: every lane takes the exterior traces of its lines from the
    // carried store (tr or trl); where a wave has lanes that do not carry,
    // those lanes first put there the traces formed from the neighbour's
    // nodes (the same sums as below without the sweep)
    if constexpr (SW) {
      if (k == KS && wave_load) {
        const CT* re = fr.r[use_right[k] ? 0 : 1];
        CT lx[N1];
#pragma unroll
        for (int bb = 0; bb < N1; ++bb) lx[bb] = re[bb];
#pragma unroll
        for (int base = 0; base < NT; ++base) {
          CT t = (CT)0;
#pragma unroll
          for (int bb = 0; bb < N1; ++bb) t += lx[bb] * nbval(base + bb * NT);
          if constexpr (kTrLds) {
            if (!lane_carry) trl[base * kBlock + tid] = t;
          } else {
            tr[base] = lane_carry ? tr[base] : t;
          }
        }
      }
    }
    auto ext_sweep = [&](int base) -> CT {
      if constexpr (kTrLds) return trl[base * kBlock + tid];
      else return tr[base];
    };
    const CT a = (CT)(vel.u[k] * g.scale[k]);
    // diffuse walls of this axis touching the element (uniform)
    const double* rho_lo = nullptr;
    const double* rho_hi = nullptr;
    bool dwall = false;
    CT mw = (CT)0;
    if constexpr (DIM <= 2 && !SW) {  // sweeps run meshes without diffuse walls
      const int off_lo = sreg(A.wall_off[k][0]), off_hi = sreg(A.wall_off[k][1]);
      const bool dlo = off_lo >= 0 && ek[k] == 0;
      const bool dhi = off_hi >= 0 && ek[k] == sreg(g.nelem[k]) - 1;
      dwall = dlo || dhi;
      if (dwall) {
        constexpr int NF = ipow(N1, DIM - 1);
        const int fe = DIM == 1 ? 0 : ek[1 - k];  // element index on the wall face
        rho_lo = A.wall_rho + (dlo ? off_lo : 0) + fe * NF;
        rho_hi = A.wall_rho + (dhi ? off_hi : 0) + fe * NF;
        // unit-density wall Maxwellian at this lane's velocity, inflow side
        const double* wp = A.wallp + (k * 2 + (pos[k] ? 0 : 1)) * 8;
        const double d0 = vel.u[0] - wp[2], d1 = vel.u[1] - wp[3], d2 = vel.u[2] - wp[4];
        mw = (CT)(wp[0] * exp(-(d0 * d0 + d1 * d1 + d2 * d2) * wp[1]));
      }
    }
    if constexpr (kMfma) {
      if (!dwall) {  // uniform
        // one pass with each lane's own operators when every block of four
        // lanes shares the sign of u_k; otherwise one pass per sign, each
        // applied to the lanes of that sign only
        const bool uni = quads_agree(pos[k]);
        const int npass = uni ? 1 : 2;
        // sweep axis: the exterior trace t of each line enters as G_in t (one
        // more 4x4x1 product) instead of E applied to the neighbour's line
        for (int ps = 0; ps < npass; ++ps) {
          const int sg = uni ? (pos[k] ? 1 : 0) : ps;
          const int ur = sg ? (wall_in[k][1] ? 0 : 1) : (wall_in[k][0] ? 1 : 0);
          float dp[4], ev[4];
          line_ops_row(lo, sg, ur, tid, dp, ev);
          const float gin = lo.G[sg][tid & 3];
          const CT as = (uni || (pos[k] ? 1 : 0) == sg) ? a : (CT)0;
#pragma unroll
          for (int base = 0; base < NS; ++base) {
            if ((base / S1) % N1 != 0) continue;
            float fl[N1];
#pragma unroll
            for (int bb = 0; bb < N1; ++bb) fl[bb] = f[base + bb * S1];
            mfma_f4 c;
            if (SW && k == KS) {
              c = line_mfma_own<N1>(dp, fl);
              c = __builtin_amdgcn_mfma_f32_4x4x1f32(gin, ext_sweep(base), c, 0, 0, 0);
            } else {
              float nl[N1];
#pragma unroll
              for (int bb = 0; bb < N1; ++bb) nl[bb] = nbval(base + bb * S1);
              c = line_mfma<N1>(dp, ev, fl, nl);
            }
#pragma unroll
            for (int ia = 0; ia < N1; ++ia) acc[base + ia * S1] = fmaf(as, c[ia], acc[base + ia * S1]);
          }
          // sweep: the last axis loads nothing; keeping its products apart
          // from the previous axis' (whose loads may still be issued during
          // the axis before it) leaves the element without spills (80-116
          // bytes per lane otherwise). A barrier after every axis also
          // removed them, but then no neighbour load was issued early and
          // the launch took 40 % longer.
          if constexpr (SW) {
            if (k == KS - 1) __builtin_amdgcn_sched_barrier(0);
          }
        }
        if constexpr (SW) {
          if (k == KS) sweep_store<N1, NT, kTrLds>(fr.r[up ? 0 : 1], f, trl, tr, tid);
        }
        continue;
      }
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
    for (int base = 0; base < NS; ++base) {
      if ((base / S1) % N1 != 0) continue;
      CT line[N1];
#pragma unroll
      for (int bb = 0; bb < N1; ++bb) line[bb] = f[base + bb * S1];
      CT own = (CT)0, ext = (CT)0;
#pragma unroll
      for (int bb = 0; bb < N1; ++bb) own += lown[bb] * line[bb];
      if (SW && k == KS) {
        ext = ext_sweep(base);
      } else {
#pragma unroll
        for (int bb = 0; bb < N1; ++bb) ext += lext[bb] * nbval(base + bb * S1);
      }
      if (dwall) {  // uniform: the element touches a diffuse wall of axis k
        // flux point of this line on the wall face
        const int fp = (base % S1) + (base / (S1 * N1)) * S1;
        const CT rw = (CT)(pos[k] ? sreg(rho_lo[fp]) : sreg(rho_hi[fp]));
        ext = dif[k] ? rw * mw : ext;
      }
      const CT jump = a * (ext - own);
#pragma unroll
      for (int ia = 0; ia < N1; ++ia) {
        CT df = (CT)0;
#pragma unroll
        for (int bb = 0; bb < N1; ++bb) df += OP.D[ia][bb] * line[bb];
        acc[base + ia * S1] += a * df + jump * Gin[ia];
      }
    }
    if constexpr (SW) {
      if (k == KS) sweep_store<N1, NT, kTrLds>(fr.r[up ? 0 : 1], f, trl, tr, tid);
    }
  }

  // BGK relaxation towards the discretely conservative equilibrium (FP64
  // rows from LDS), combined with the transport and the SSP-RK weights: the
  // stage value is a f^n + h with
  //   h = b (f - dt T) + b dt C,   C = (g - f)/tau in FP64, added in FP64
  // (FP32 arithmetic: b (f - dt T) in FP32, the sum rounded once). Where it
  // lowers the register peak (kFold) h is formed before f^n is loaded, so f
  // and T are dead by then; the matrix-core path of p = 3 hexahedra (whose
  // peak is in the transport) loads f^n first and rounds a f^n + h once.
  // The whole relaxation sits in the one branch that loads the rows (keeping
  // it there lets the compiler overlap the LDS reads of all nodes without
  // holding them across the branch).
  constexpr bool kFold = true;
  // f^n (MODE 0), or the FP32 state F that BF16 increments are taken against
  // (increment stages). f^n and the stage output are streams that no other
  // work-group of the launch reads again: they are loaded and stored with
  // the non-temporal hint, so they do not displace from L2 the nodes that the
  // neighbouring work-groups re-read (3-5 % per launch on the 2-D box and the
  // Taylor-Green box). F of the own nodes is kept in registers for small
  // elements and read again (a cache hit) otherwise.
  CT fnv[NS];
  if constexpr (!kFold) {
    if constexpr (MODE == 0) {
      const ST* fn = (const ST*)A.fn + f_offset(g, e, 0, jj);
#pragma unroll
      for (int i = 0; i < NS; ++i) fnv[i] = (CT)__builtin_nontemporal_load(&fn[i * kVB]);
    }
  }
  // positions of this velocity's factors in a node's LDS row (compact)
  const int cx = vel.b[0] - rp.x0, oy = rp.nx + vel.b[1] - rp.y0,
            oz = rp.nxy + vel.b[2] - rp.z0;
  double* oe1 = nullptr;  // residual output (canonical layout, MODE 1)
  if constexpr (MODE == 1) {
    const int jc = vel.b[0] + g.nv1[0] * (vel.b[1] + g.nv1[1] * vel.b[2]);
    oe1 = (double*)A.out + (e - A.out_e0) * NS * nv + jc;
  }
  const CT dt = (CT)A.dt, ca = (CT)A.a, cb = (CT)A.b;
  const double wc = A.b * A.dt;
  CT o[NS];
  if (A.collide) {  // uniform; one branch, so the LDS reads of all nodes overlap
    // rows beyond the first batch (large velocity grids), loaded only now so
    // that their loop does not hold back the waits of the bulk loads
    table_rest<kU>(tab, et, rp, tid);
    lds_barrier();
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      const double c = collision_term(tab + i * rp.ncols, cx, oy, oz, rp.ncols, (double)f[i]);
      if constexpr (MODE == 1) {
        if (valid) oe1[(int64_t)i * nv] = c - (double)acc[i];
      } else if constexpr (!kFold) {
        const CT r = fmaf(-dt, acc[i], f[i]);
        const CT b32 = MODE == 0 ? fmaf(ca, fnv[i], cb * r) : cb * r;
        o[i] = (CT)fma(wc, c, (double)b32);
      } else if constexpr (sizeof(CT) == 8) {
        acc[i] = fma(wc, c, cb * (f[i] - dt * acc[i]));
      } else {
        acc[i] = (CT)fma(wc, c, (double)(cb * (f[i] - dt * acc[i])));
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      if constexpr (MODE == 1) {
        if (valid) oe1[(int64_t)i * nv] = -(double)acc[i];
      } else if constexpr (!kFold) {
        const CT r = fmaf(-dt, acc[i], f[i]);
        o[i] = MODE == 0 ? fmaf(ca, fnv[i], cb * r) : cb * r;
      } else {
        acc[i] = cb * (f[i] - dt * acc[i]);
      }
    }
  }
  if constexpr (kFold && MODE != 1) {
    // keep the scheduler from hoisting these loads above the relaxation
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (kKeepF) {
#pragma unroll
      for (int i = 0; i < NS; ++i) fnv[i] = fb[i];
    } else if constexpr (INC) {
#pragma unroll
      for (int i = 0; i < NS; ++i) fnv[i] = (CT)fe[i * kVB];
    } else if constexpr (MODE == 0) {
      const ST* fn = (const ST*)A.fn + f_offset(g, e, 0, jj);
#pragma unroll
      for (int i = 0; i < NS; ++i) fnv[i] = (CT)__builtin_nontemporal_load(&fn[i * kVB]);
    }
#pragma unroll
    for (int i = 0; i < NS; ++i) o[i] = MODE == 0 ? ca * fnv[i] + acc[i] : acc[i];
  }

  if constexpr (MODE == 1) {
    if (tid == 0 && count) atomicAdd(&A.diag[4], 1ull);
  } else {
    if (A.limiter) {
      CT fmin = o[0];
#pragma unroll
      for (int i = 0; i < NS; ++i) fmin = o[i] < fmin ? o[i] : fmin;
      const CT mean = tensor_wsum<DIM, N1>(o, OP.w) / OP.Wsum;
      const bool hit = valid && (fmin < (CT)0);
      if (hit && mean != fmin) {
        CT beta = fabs(mean / (mean - fmin));
        beta = beta > (CT)1 ? (CT)1 : beta;
#pragma unroll
        for (int i = 0; i < NS; ++i) o[i] = mean + beta * (o[i] - mean);
      }
      const unsigned long long nh = __popcll(__ballot(hit));
      const unsigned long long nb = __popcll(__ballot(hit && !(mean > (CT)0)));
      if ((tid & 63) == 0 && nh) {
        atomicAdd(&A.diag[2], nh);
        if (nb) atomicAdd(&A.diag[3], nb);
      }
    }
    if constexpr (INC) {
      // the increment o - F in BF16, and the stored state F + increment for
      // the partials; the last stage stores o itself in FP32
      if (A.out_full) {
        if (valid) {
          ST* oe = (ST*)A.out + f_offset(g, e, 0, j);
#pragma unroll
          for (int i = 0; i < NS; ++i) __builtin_nontemporal_store((ST)o[i], &oe[i * kVB]);
        }
      } else {
        const int64_t ooff = f_offset(g, e, 0, jj);
        uint32_t* ow = inc_pairs((uint16_t*)A.out, ooff);
        float omin = INFINITY, smin = INFINITY;  // stage values / stored values
        uint32_t hp = 0;
#pragma unroll
        for (int i = 0; i < NS; ++i) {
          float stored;
          const uint16_t h = bf16_increment(o[i], fnv[i], stored);
          if (i % 2 == 0 && i == NS - 1) {
            if (valid) __builtin_nontemporal_store(h, (uint16_t*)A.out + ooff + i * kVB);
          } else if (i % 2 == 0) {
            hp = h;
          } else if (valid) {
            __builtin_nontemporal_store(hp | ((uint32_t)h << 16), &ow[(i >> 1) * kVB]);
          }
          omin = fminf(omin, o[i]);
          smin = fminf(smin, stored);
          o[i] = stored;
        }
        // slices whose stored stage is negative where the stage itself is not
        const unsigned long long nviol = __popcll(__ballot(valid && smin < 0.0f && !(omin < 0.0f)));
        if ((tid & 63) == 0 && nviol) atomicAdd(&A.diag[5], nviol);
      }
    } else {
      ST* out = (ST*)A.out;
      if (valid) {
        ST* oe = out + f_offset(g, e, 0, j);
#pragma unroll
        for (int i = 0; i < NS; ++i) __builtin_nontemporal_store((ST)o[i], &oe[i * kVB]);
      }
    }
    // moment partials of what was stored (FP64 sums on the matrix cores); the
    // staging area reuses the equilibrium rows' LDS once every wave is done
    // with them
    if (A.collide) lds_barrier();
    element_partials_mfma<NS, ST, CT>(o, vel, A.partials, node0, g.nx, chunk, dyn_lds, red, tid);
    if (tid == 0 && count) atomicAdd(&A.diag[4], 1ull);
  }
}

template <int DIM, int P, typename ST, int MODE, bool INC = false>
__global__ void __launch_bounds__(kBlock)
    __attribute__((amdgpu_waves_per_eu(stage_waves<DIM, P, typename Compute<ST>::T, INC>())))
    k_stage(const StageArgs A) {
  const int64_t w = xcd_chunk_remap(blockIdx.x, gridDim.x, A.ecount, A.xcd_part);
  typename Compute<ST>::T tr[sweep_tr_regs<DIM, P>()];
  stage_item<DIM, P, ST, MODE, INC>(A, (int)(w / A.ecount), work_element(A.order, A.e0, w, A.ecount),
                                    w == 0, false, false, tr);
}

// Pointer into argument memory that is read-only while kernels run (kernel
// arguments, descriptor tables): loads through the constant address space
// become scalar loads that the compiler may repeat where a value is used,
// instead of vector loads (or scalar registers) held across a loop.
template <typename T>
using table_ptr = const __attribute__((address_space(4))) T*;
template <typename T>
__device__ __forceinline__ const T& table_entry(table_ptr<T> p, int64_t i) {
  return *(const T*)&p[i];
}

// Direction of the column sweep of velocity chunk `chunk` (slots from v0 on):
// true when the last transported component of its first velocity slot is
// positive (the test the stage kernels make per lane), i.e. when the sweep
// runs towards increasing element index on the last axis. Lanes of the chunk
// with the other sign read their neighbours as in k_stage.
__device__ __forceinline__ bool sweep_up(const DevGeom& g, int v0) {
  int b[3];
  slot_nodes(g, v0 < g.nv ? v0 : (int)g.nv - 1, b);
  const int k = g.dim - 1;
  return (g.vlo[k] + b[k] * g.du[k]) * g.scale[k] > 0.0;
}

// Stage launch as column sweeps (RK stages over the whole mesh; no diffuse
// wall on the last axis). Work item w = (velocity chunk, segment of sweep_seg
// elements of one column along the last axis); columns vary fastest, so the
// work-groups in flight on an XCD hold neighbouring columns at about the same
// position along the sweep, and their x (and y) neighbours' nodes are read
// while still in L2. Each work-group walks its segment in the upwind
// direction of its chunk, carrying the outflow traces (stage_item).
template <int DIM, int P, typename ST, int MODE, bool INC = false>
__global__ void __launch_bounds__(kBlock)
    __attribute__((amdgpu_waves_per_eu(stage_waves<DIM, P, typename Compute<ST>::T, INC>())))
    k_stage_sweep(const StageArgs A) {
  const DevGeom& g = A.g;
  const int nl = sreg(g.nelem[DIM - 1]), seg = sreg(A.sweep_seg);
  const int64_t ncol = g.ne / nl, nseg = nl / seg, per_chunk = ncol * nseg;
  const int64_t w = xcd_chunk_remap(blockIdx.x, gridDim.x, per_chunk, A.xcd_part);
  const int chunk = (int)(w / per_chunk);
  const int64_t r = w - (int64_t)chunk * per_chunk;
  const int64_t sg = r / ncol, col = r - sg * ncol;
  const bool up = sweep_up(g, chunk * kBlock);
  typename Compute<ST>::T tr[sweep_tr_regs<DIM, P>()];
  // the arguments are read through a pointer the compiler cannot follow
  // across iterations, so that they are fetched again (scalar loads) where an
  // element needs them instead of being held in scalar registers across the
  // column (which spilled)
  table_ptr<StageArgs> ap = (table_ptr<StageArgs>)__builtin_amdgcn_kernarg_segment_ptr();
  for (int s = 0; s < seg; ++s) {
    const int el = (int)(sg * seg) + s;
    const int64_t e = col + (int64_t)(up ? el : nl - 1 - el) * ncol;
    // the previous item's last LDS reads (partial sums) are ordered before
    // this item's writes by the barrier of the relaxation; without collisions
    // by this one
    if (s > 0 && !A.collide) lds_barrier();
    asm volatile("" : "+s"(ap));
    stage_item<DIM, P, ST, MODE, INC, true>(table_entry(ap, 0), chunk, e, w == 0 && s == 0, s > 0,
                                            up, tr);
  }
}

// ---------------------------------------------------------------------------
// Descriptor tables of a batch (serving): the arguments of every member slot
// live in device memory (StageArgs for each of the three RK stages, the
// NewtonArgs, the WallArgs for each stage), and one BatchList per launch names
// the members it covers and the prefix sums of their work units, so that one
// launch covers every member of a kernel family and a change of membership
// rewrites tables instead of rebuilding launch arguments.
// ---------------------------------------------------------------------------
constexpr int kMaxBatchMembers = 64;

// The tables are rewritten by copies between launches and never during one,
// so kernels read them through table_ptr (constant address space).
struct BatchList {
  int32_t n;     // members covered
  int32_t pad;
  int32_t slot[kMaxBatchMembers];              // member slots
  // prefix sums of the members' work units (the host keeps every total
  // below 2^31): stage work items (element x chunk), equilibrium
  // work-groups of 256 lanes, wall-flux work-groups, wall-density
  // work-groups of 256 lanes
  int32_t stage_off[kMaxBatchMembers + 1];
  int32_t newton_off[kMaxBatchMembers + 1];
  int32_t wflux_off[kMaxBatchMembers + 1];
  int32_t wrho_off[kMaxBatchMembers + 1];
};

// Member of the list whose range of work units holds unit t (off[m] <= t <
// off[m + 1]), by bisection; uniform over a work-group. Members with no
// units share their offset with the next member, and the largest such m is
// the one whose range is not empty.
__device__ __forceinline__ int batch_member(const __attribute__((address_space(4))) int32_t* off,
                                           int n, int32_t t) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Stage launch over the members of one kernel family (dimension, order,
// storage precision) at RK stage `stage`: one work-group per item of every
// member in the list (the host sizes the grid to the list's item count), the
// items dealt to the XCDs in contiguous ranges as in k_stage.
template <int DIM, int P, typename ST, int MODE>
__global__ void __launch_bounds__(kBlock)
    __attribute__((amdgpu_waves_per_eu(stage_waves<DIM, P, typename Compute<ST>::T, false>())))
    k_stage_batch(table_ptr<StageArgs> args, table_ptr<BatchList> list, int stage) {
  // one item per work-group; the grid is the list's item count
  const int32_t u = (int32_t)xcd_remap(blockIdx.x, gridDim.x);
  const int m = batch_member(list->stage_off, list->n, u);
  const StageArgs& A = table_entry(args, list->slot[m] * 3 + stage);
  const int64_t w = u - list->stage_off[m];
  typename Compute<ST>::T tr[sweep_tr_regs<DIM, P>()];
  stage_item<DIM, P, ST, MODE>(A, (int)(w / A.ecount), work_element(A.order, A.e0, w, A.ecount),
                               w == 0, false, false, tr);
}

// Moment partials of a stored state (first stage after installation).
template <int DIM, int P, typename ST>
__global__ void __launch_bounds__(kBlock) k_moments(const StageArgs A) {
  using CT = typename Compute<ST>::T;
  constexpr int N1 = P + 1;
  constexpr int NS = ipow(N1, DIM);
  __shared__ double red[(kBlock / 64) * part_rows<NS>() * 5];
  extern __shared__ __align__(16) unsigned char dyn_lds[];  // MFMA staging
  const DevGeom& g = A.g;
  const int64_t w = xcd_remap(blockIdx.x, gridDim.x);
  const int chunk = (int)(w / A.ecount);
  const int64_t e = work_element(A.order, A.e0, w, A.ecount);
  const int64_t nv = g.nv;
  const int j = chunk * kBlock + (int)threadIdx.x;
  const bool valid = j < nv;
  const int jj = valid ? j : (int)nv - 1;
  Vel vel = velocity_of(g, jj);
  if (!valid) vel.w = 0.0;
  const ST* fe = (const ST*)A.fin + f_offset(g, e, 0, jj);
  CT f[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) f[i] = (CT)fe[i * kVB];
  element_partials_mfma<NS, ST, CT>(f, vel, A.partials, e * NS, g.nx, chunk, dyn_lds, red,
                                    (int)threadIdx.x);
}

}  // namespace bgk
