// bgk_runtime.hip -- C-ABI runtime of libbgk (declared in include/bgk.h).
//
// Host responsibilities: validate the problem, lay out the caller's device
// workspace, build the FP64 operator tables, sequence the kernels of a
// residual evaluation or of SSP-RK3 steps on the caller's stream, and move
// canonical FP64 data in and out. No device memory is allocated here.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/bgk.h"
#include "bgk_launch.hpp"

using namespace bgk;

namespace {

thread_local std::string g_last_error;

bgk_status fail(bgk_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
bgk_status fail(bgk_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t _e = (expr);                                                              \
    if (_e != hipSuccess)                                                                \
      return fail(BGK_ERR_DEVICE, "%s: %s (%s:%d)", #expr, hipGetErrorString(_e), __FILE__, \
                  __LINE__);                                                             \
  } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// ---------------------------------------------------------------------------
// One-dimensional operators, built on the host in FP64.
//
// Gauss-Legendre rule by the Golub-Welsch construction: the nodes are the
// eigenvalues of the symmetric tridiagonal Jacobi matrix of the Legendre
// recurrence (off-diagonal k / sqrt(4k^2 - 1)), the weights are twice the
// squared first components of the normalised eigenvectors. The small
// symmetric eigenproblem is solved by cyclic Jacobi rotations.
// ---------------------------------------------------------------------------
void gauss_golub_welsch(int n, double* x, double* w) {
  double A[kMaxN1][kMaxN1] = {}, V[kMaxN1][kMaxN1] = {};
  for (int i = 0; i < n; ++i) V[i][i] = 1.0;
  for (int k = 1; k < n; ++k) A[k - 1][k] = A[k][k - 1] = k / sqrt(4.0 * k * k - 1.0);
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += A[p][q] * A[p][q];
    if (off < 1e-34) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        if (A[p][q] == 0.0) continue;
        const double th = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
        const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // A <- A R
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - s * akq;
          A[k][q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // A <- R^T A
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - s * aqk;
          A[q][k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {  // V <- V R
          const double vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - s * vkq;
          V[k][q] = s * vkp + c * vkq;
        }
      }
  }
  int idx[kMaxN1];
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx, idx + n, [&](int a, int b) { return A[a][a] < A[b][b]; });
  for (int i = 0; i < n; ++i) {
    const int k = idx[i];
    double nrm = 0.0;
    for (int r = 0; r < n; ++r) nrm += V[r][k] * V[r][k];
    x[i] = A[k][k];
    w[i] = 2.0 * V[0][k] * V[0][k] / nrm;
  }
  // symmetrise (the rule is exactly symmetric about 0)
  for (int i = 0; i < n / 2; ++i) {
    const double xm = 0.5 * (x[n - 1 - i] - x[i]), wm = 0.5 * (w[i] + w[n - 1 - i]);
    x[i] = -xm;
    x[n - 1 - i] = xm;
    w[i] = w[n - 1 - i] = wm;
  }
  if (n % 2 == 1) x[n / 2] = 0.0;
}

// Barycentric Lagrange tools: weights c_b = 1 / prod_{m != b}(xi_b - xi_m);
// D_ab = (c_b / c_a) / (xi_a - xi_b) (a != b), D_aa = -sum_{b != a} D_ab;
// l_b(x) = (c_b / (x - xi_b)) / sum_m (c_m / (x - xi_m)) off the nodes.
void build_ops(int n1, int dim, DevOps& op) {
  double xi[kMaxN1], wq[kMaxN1], c[kMaxN1];
  gauss_golub_welsch(n1, xi, wq);
  for (int b = 0; b < n1; ++b) {
    double pr = 1.0;
    for (int m = 0; m < n1; ++m)
      if (m != b) pr *= xi[b] - xi[m];
    c[b] = 1.0 / pr;
  }
  memset(&op, 0, sizeof(op));
  for (int a = 0; a < n1; ++a) {
    double diag = 0.0;
    for (int b = 0; b < n1; ++b) {
      if (a == b) continue;
      op.D[a][b] = (c[b] / c[a]) / (xi[a] - xi[b]);
      diag -= op.D[a][b];
    }
    op.D[a][a] = diag;
  }
  for (int side = 0; side < 2; ++side) {
    const double x0 = side == 0 ? -1.0 : 1.0;
    double den = 0.0;
    for (int m = 0; m < n1; ++m) den += c[m] / (x0 - xi[m]);
    for (int b = 0; b < n1; ++b) (side == 0 ? op.lamL : op.lamR)[b] = (c[b] / (x0 - xi[b])) / den;
  }
  // Correction functions recovering nodal DG: at Gauss points their slopes are
  // g_L'(xi_a) = -l_a(-1) / w_a and g_R'(xi_a) = l_a(+1) / w_a.
  for (int a = 0; a < n1; ++a) {
    op.GL[a] = -op.lamL[a] / wq[a];
    op.GR[a] = op.lamR[a] / wq[a];
  }
  // node weights are the tensor products w[a_1] ... w[a_d]; their sum is
  // (sum_a w_a)^d
  double w1 = 0.0;
  for (int a = 0; a < n1; ++a) {
    op.w[a] = wq[a];
    w1 += wq[a];
  }
  double ws = 1.0;
  for (int k = 0; k < dim; ++k) ws *= w1;
  op.Wsum = ws;
}

void gauss_nodes(int n1, double* xi) {
  double w[kMaxN1];
  gauss_golub_welsch(n1, xi, w);
}

struct Layout {
  size_t f[3], partials, params, etab, order, rcols, Q, prim, diag, wallp, wall_part, wall_rho,
      total;
  int64_t nx, nv, ne, nvb;
  int ns, nchunk;
  int64_t wall_points;  // flux points on diffuse walls
  size_t fbytes;   // one FP64/FP32 state buffer
  size_t fsz[3];   // bytes of f(0), f(1), f(2)
};

// Flux points of the diffuse walls: side (k, s) holds ne / nelem[k] faces of
// (p+1)^(d-1) points each.
int64_t diffuse_wall_points(const bgk_problem* pb) {
  int64_t ne = 1, nf = 1, n = 0;
  for (int k = 0; k < pb->dim; ++k) ne *= pb->nelem[k];
  for (int k = 0; k + 1 < pb->dim; ++k) nf *= pb->order + 1;
  for (int k = 0; k < pb->dim; ++k)
    for (int s = 0; s < 2; ++s)
      if (pb->bc[k][s] == BGK_BC_DIFFUSE) n += ne / pb->nelem[k] * nf;
  return n;
}

bgk_status validate(const bgk_problem* pb) {
  if (!pb) return fail(BGK_ERR_INVALID_ARG, "problem is NULL");
  if (pb->dim < 1 || pb->dim > 3) return fail(BGK_ERR_INVALID_ARG, "dim must be 1, 2 or 3");
  if (pb->order < 1 || pb->order > 3)
    return fail(BGK_ERR_UNSUPPORTED, "order %d not built (1..3)", pb->order);
  if (pb->precision != BGK_FP64 && pb->precision != BGK_FP32 && pb->precision != BGK_BF16)
    return fail(BGK_ERR_INVALID_ARG, "precision must be BGK_FP64, BGK_FP32 or BGK_BF16");
  if (pb->limiter != 0 && pb->limiter != 1)
    return fail(BGK_ERR_INVALID_ARG, "limiter must be 0 or 1");
  if (pb->equilibrium != BGK_EQ_CONSERVATIVE && pb->equilibrium != BGK_EQ_CONTINUOUS)
    return fail(BGK_ERR_INVALID_ARG, "equilibrium must be BGK_EQ_CONSERVATIVE or BGK_EQ_CONTINUOUS");
  for (int k = 0; k < pb->dim; ++k) {
    if (pb->nelem[k] < 1) return fail(BGK_ERR_INVALID_ARG, "nelem[%d] < 1", k);
    if (!(pb->xhi[k] > pb->xlo[k])) return fail(BGK_ERR_INVALID_ARG, "xhi[%d] <= xlo[%d]", k, k);
    for (int s = 0; s < 2; ++s) {
      if (pb->bc[k][s] != BGK_BC_PERIODIC && pb->bc[k][s] != BGK_BC_SPECULAR &&
          pb->bc[k][s] != BGK_BC_DIFFUSE)
        return fail(BGK_ERR_INVALID_ARG, "bc[%d][%d] unknown", k, s);
      if (pb->bc[k][s] == BGK_BC_DIFFUSE) {
        if (pb->dim == 3)
          return fail(BGK_ERR_UNSUPPORTED, "diffuse walls are built for 1-D and 2-D meshes");
        if (pb->precision == BGK_BF16)
          return fail(BGK_ERR_UNSUPPORTED, "diffuse walls are built for FP64 and FP32 storage");
        if (!(pb->wall_theta[k][s] > 0.0))
          return fail(BGK_ERR_INVALID_ARG, "wall_theta[%d][%d] must be > 0", k, s);
      }
    }
    if ((pb->bc[k][0] == BGK_BC_PERIODIC) != (pb->bc[k][1] == BGK_BC_PERIODIC))
      return fail(BGK_ERR_INVALID_ARG, "axis %d: periodic on one side only", k);
    if (pb->bc[k][0] == BGK_BC_SPECULAR && pb->vlo[k] != -pb->vhi[k])
      return fail(BGK_ERR_INVALID_ARG, "specular wall on axis %d needs vlo == -vhi", k);
  }
  for (int c = 0; c < 3; ++c) {
    if (pb->nvel[c] < 2) return fail(BGK_ERR_INVALID_ARG, "nvel[%d] < 2", c);
    if (!(pb->vhi[c] > pb->vlo[c])) return fail(BGK_ERR_INVALID_ARG, "vhi[%d] <= vlo[%d]", c, c);
  }
  {
    int ns = 1;
    for (int k = 0; k < pb->dim; ++k) ns *= pb->order + 1;
    const double nv = (double)pb->nvel[0] * pb->nvel[1] * pb->nvel[2];
    if (nv >= 2147483647.0) return fail(BGK_ERR_UNSUPPORTED, "velocity grid too large");
    // equilibrium rows are FP64 for every storage precision
    const size_t tab = (size_t)ns * (pb->nvel[0] + pb->nvel[1] + pb->nvel[2] + 1) * 8;
    if (tab > (size_t)kMaxTabBytes)
      return fail(BGK_ERR_UNSUPPORTED, "equilibrium factors of one element (%zu B) exceed LDS", tab);
  }
  if (!(pb->theta_ref > 0.0) && pb->mu_ref > 0.0)
    return fail(BGK_ERR_INVALID_ARG, "theta_ref must be > 0");
  if (!(pb->sutherland >= 0.0) || !isfinite(pb->sutherland))
    return fail(BGK_ERR_INVALID_ARG, "sutherland must be finite and >= 0");
  return BGK_OK;
}

Layout layout_of(const bgk_problem* pb) {
  Layout L;
  L.ne = 1;
  for (int k = 0; k < pb->dim; ++k) L.ne *= pb->nelem[k];
  L.ns = 1;
  for (int k = 0; k < pb->dim; ++k) L.ns *= pb->order + 1;
  L.nx = L.ne * L.ns;
  L.nv = (int64_t)pb->nvel[0] * pb->nvel[1] * pb->nvel[2];
  const int vb = velocities_per_block(pb->dim, pb->order, pb->precision);
  L.nchunk = (int)((L.nv + vb - 1) / vb);
  const size_t s = pb->precision == BGK_FP64 ? 8 : 4;
  L.nvb = (L.nv + kVB - 1) / kVB;
  L.fbytes = (size_t)L.nx * (size_t)(L.nvb * kVB) * s;  // internal layout, padded blocks
  // FP64/FP32: three state-precision buffers (f^n, f^(1), f^(2)). BF16: two
  // FP32 buffers that alternate as f^n and f^(n+1) (the first increment lives
  // in the second one) and one BF16 buffer for the second increment.
  L.fsz[0] = L.fsz[1] = L.fbytes;
  L.fsz[2] = pb->precision == BGK_BF16 ? L.fbytes / 2 : L.fbytes;
  size_t off = 0;
  for (int b = 0; b < 3; ++b) {
    L.f[b] = off;
    off = align_up(off + L.fsz[b]);
  }
  L.partials = off;
  off = align_up(off + (size_t)L.nx * L.nchunk * 5 * sizeof(double));
  L.params = off;
  off = align_up(off + (size_t)L.nx * 8 * sizeof(double));
  L.etab = off;
  off = align_up(off + (size_t)L.nx * (pb->nvel[0] + pb->nvel[1] + pb->nvel[2] + 1) *
                             sizeof(double));
  L.order = off;
  off = align_up(off + (size_t)L.ne * sizeof(int32_t));
  L.rcols = off;
  off = align_up(off + (size_t)L.nchunk * sizeof(RowCols));
  L.Q = off;
  off = align_up(off + (size_t)L.nx * 5 * sizeof(double));
  L.prim = off;
  off = align_up(off + (size_t)L.nx * 5 * sizeof(double));
  L.diag = off;
  off = align_up(off + 8 * sizeof(unsigned long long));
  L.wall_points = diffuse_wall_points(pb);
  L.wallp = off;
  off = align_up(off + (L.wall_points ? 32 * sizeof(double) : 0));
  L.wall_part = off;
  off = align_up(off + (size_t)L.wall_points * L.nchunk * sizeof(double));
  L.wall_rho = off;
  off = align_up(off + (size_t)L.wall_points * sizeof(double));
  L.total = off;
  return L;
}

}  // namespace

struct bgk_solver {
  bgk_problem pb;
  Layout L;
  DevGeom g;
  DevOps op;
  char* ws;
  hipStream_t stream;
  int precision;
  bool has_state = false;
  bool partials_valid = false;
  bool failed = false;
  bool counters_ready = false;  // device counters cleared since create
  bool in_batch = false;
  double gamma;
  // event timing of rk3_step launches: events[i] .. events[i+1] brackets
  // interval i of kind kinds[i] (0 newton, 1 stage, 2 host gap)
  bool timing = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<int> kinds;
  int cur = 0;  // state buffer (BF16 storage alternates between f(0) and f(1))
  int sweep_seg = 0;  // column sweeps of the RK stages: elements per work item (0: none)
  int xcd_part = 0;   // stage work items dealt to the XCDs chunk by chunk (xcd_chunk_remap)
  void* f(int b) const { return ws + L.f[b]; }
  void* state() const { return f(cur); }
  double* partials() const { return (double*)(ws + L.partials); }
  double* params() const { return (double*)(ws + L.params); }
  double* etab() const { return (double*)(ws + L.etab); }
  int32_t* order() const { return (int32_t*)(ws + L.order); }
  RowCols* rcols() const { return (RowCols*)(ws + L.rcols); }
  bool order_ready = false;
  std::vector<int32_t> order_host;  // traversal order (empty: lexicographic)
  std::vector<RowCols> rcols_host;  // row entries per velocity chunk (empty: all)
  std::vector<double> wallp_host;   // [k][s][8] diffuse-wall constants (empty: none)
  WallArgs wall;                    // sides of the diffuse walls (fin set per stage)
  double* wallp() const { return (double*)(ws + L.wallp); }
  double* wall_part() const { return (double*)(ws + L.wall_part); }
  double* wall_rho() const { return (double*)(ws + L.wall_rho); }
  double* Q() const { return (double*)(ws + L.Q); }
  double* prim() const { return (double*)(ws + L.prim); }
  unsigned long long* diag() const { return (unsigned long long*)(ws + L.diag); }
  size_t s_bytes() const { return precision == BGK_FP64 ? 8 : 4; }
};

namespace {

// Row entries read by the velocity slots [j0, j1): per axis the range of
// velocity nodes they use, and 1/tau.
RowCols row_cols(const DevGeom& g, int j0, int j1) {
  int lo[3] = {g.nv1[0], g.nv1[1], g.nv1[2]}, hi[3] = {-1, -1, -1};
  for (int j = j0; j < j1; ++j) {
    int b[3];
    slot_nodes(g, j, b);
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::min(lo[k], b[k]);
      hi[k] = std::max(hi[k], b[k]);
    }
  }
  RowCols r;
  r.x0 = lo[0];
  r.nx = hi[0] - lo[0] + 1;
  r.y0 = lo[1];
  r.ny = hi[1] - lo[1] + 1;
  r.z0 = lo[2];
  r.nz = hi[2] - lo[2] + 1;
  r.ncols = r.nx + r.ny + r.nz + 1;
  r.magic = (int32_t)(uint32_t)(((1ull << 32) + r.ncols - 1) / r.ncols);
  return r;
}

// Every row entry (all velocity nodes of every axis, and 1/tau).
RowCols row_cols_all(const DevGeom& g) {
  RowCols r;
  r.x0 = r.y0 = r.z0 = 0;
  r.nx = g.nv1[0];
  r.ny = g.nv1[1];
  r.nz = g.nv1[2];
  r.ncols = g.tabw;
  r.magic = (int32_t)(uint32_t)(((1ull << 32) + r.ncols - 1) / r.ncols);
  return r;
}

StageArgs stage_args(const bgk_solver* s) {
  StageArgs A;
  memset(&A, 0, sizeof(A));
  A.g = s->g;
  A.op = s->op;
  {
    const DevOps& o = s->op;
    DevOpsT<float>& q = A.opf;
    for (int a = 0; a < kMaxN1; ++a) {
      for (int b = 0; b < kMaxN1; ++b) q.D[a][b] = (float)o.D[a][b];
      q.lamL[a] = (float)o.lamL[a];
      q.lamR[a] = (float)o.lamR[a];
      q.GL[a] = (float)o.GL[a];
      q.GR[a] = (float)o.GR[a];
    }
    for (int a = 0; a < kMaxN1; ++a) q.w[a] = (float)o.w[a];
    q.Wsum = (float)o.Wsum;
    // line operators with the inflow-face correction folded in (FP64, then
    // rounded): Dp = D - G_in lam_own^T, E = G_in lam_ext^T
    LineOps& lo = A.lops;
    memset(&lo, 0, sizeof(lo));
    const int n1 = s->g.n1;
    for (int pos = 0; pos < 2; ++pos) {
      const double* lown = pos ? o.lamL : o.lamR;
      const double* gin = pos ? o.GL : o.GR;
      for (int i = 0; i < n1; ++i) lo.G[pos][i] = (float)gin[i];
      for (int i = 0; i < n1; ++i)
        for (int k = 0; k < n1; ++k) {
          lo.Dp[pos][i][k] = (float)(o.D[i][k] - gin[i] * lown[k]);
          for (int ur = 0; ur < 2; ++ur)
            lo.E[pos][ur][i][k] = (float)(gin[i] * (ur ? o.lamR[k] : o.lamL[k]));
        }
    }
  }
  A.params = s->params();
  A.etab = s->etab();
  A.order = s->order_host.empty() ? nullptr : s->order();
  A.rcols = s->rcols();
  A.rc_mask = s->rcols_host.empty() ? 0 : -1;
  A.partials = s->partials();
  A.diag = s->diag();
  A.e0 = 0;
  A.ecount = s->L.ne;
  A.out_e0 = 0;
  A.limiter = s->pb.limiter;
  A.collide = s->pb.mu_ref > 0.0 ? 1 : 0;
  A.sweep_seg = s->sweep_seg;
  A.xcd_part = s->xcd_part;
  for (int k = 0; k < 2; ++k)
    for (int sd = 0; sd < 2; ++sd) A.wall_off[k][sd] = -1;
  if (s->wall.nside) {
    A.wallp = s->wallp();
    A.wall_rho = s->wall_rho();
    for (int q = 0; q < s->wall.nside; ++q)
      A.wall_off[s->wall.side_k[q]][s->wall.side_s[q]] = s->wall.off[q];
  }
  return A;
}

NewtonArgs newton_args(const bgk_solver* s) {
  NewtonArgs N;
  memset(&N, 0, sizeof(N));
  N.g = s->g;
  N.partials = s->partials();
  N.params = s->params();
  N.etab = s->etab();
  N.Q = s->Q();
  N.diag = s->diag();
  N.gamma = s->gamma;
  N.mu_ref = s->pb.mu_ref;
  N.theta_ref = s->pb.theta_ref;
  N.omega = s->pb.omega;
  N.sutherland = s->pb.sutherland;
  N.tol = s->pb.newton_tol > 0.0 ? s->pb.newton_tol : 1e-14;
  N.maxit = s->pb.newton_maxit > 0 ? s->pb.newton_maxit : 20;
  N.collide = s->pb.mu_ref > 0.0 ? 1 : 0;
  N.continuous = s->pb.equilibrium == BGK_EQ_CONTINUOUS ? 1 : 0;
  return N;
}

// The device counters are cleared, and the element traversal order is
// uploaded, by the first call that queues device work (create itself never
// touches the workspace).
bgk_status ensure_counters(bgk_solver* s) {
  if (!s->counters_ready) {
    HIP_TRY(hipMemsetAsync(s->diag(), 0, 8 * sizeof(unsigned long long), s->stream));
    s->counters_ready = true;
  }
  if (!s->order_ready) {
    if (!s->order_host.empty()) {
      HIP_TRY(hipMemcpyAsync(s->order(), s->order_host.data(),
                             s->order_host.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                             s->stream));
    }
    if (!s->rcols_host.empty()) {
      HIP_TRY(hipMemcpyAsync(s->rcols(), s->rcols_host.data(),
                             s->rcols_host.size() * sizeof(RowCols), hipMemcpyHostToDevice,
                             s->stream));
    }
    if (!s->wallp_host.empty()) {
      HIP_TRY(hipMemcpyAsync(s->wallp(), s->wallp_host.data(),
                             s->wallp_host.size() * sizeof(double), hipMemcpyHostToDevice,
                             s->stream));
    }
    s->order_ready = true;
  }
  return BGK_OK;
}

// Diffuse walls of the stage input fin: re-emitted density per flux point.
bgk_status wall_densities(bgk_solver* s, const void* fin, hipStream_t st) {
  if (!s->wall.nside) return BGK_OK;
  WallArgs W = s->wall;
  W.fin = fin;
  HIP_TRY(launch_wall(s->precision, W, st));
  return BGK_OK;
}

// Sides, offsets and constants of the diffuse walls (host, at create). For
// side (k, s): (2 pi theta_w)^{-3/2}, 1/(2 theta_w), U_w and the inverse of
// the incoming flux sum_{incoming j} w_j |u_k| M_w(u_j) of the unit wall
// Maxwellian (incoming: u_k > 0 at s = 0, u_k < 0 at s = 1).
void setup_walls(bgk_solver* s) {
  const bgk_problem* pb = &s->pb;
  WallArgs& W = s->wall;
  memset(&W, 0, sizeof(W));
  if (!s->L.wall_points) return;
  W.g = s->g;
  for (int b = 0; b < kMaxN1; ++b) {
    W.lamL[b] = s->op.lamL[b];
    W.lamR[b] = s->op.lamR[b];
  }
  W.wallp = s->wallp();
  W.part = s->wall_part();
  W.rho = s->wall_rho();
  s->wallp_host.assign(32, 0.0);
  int nf = 1;
  for (int k = 0; k + 1 < pb->dim; ++k) nf *= pb->order + 1;
  int off = 0, blk = 0;
  for (int k = 0; k < pb->dim; ++k) {
    for (int sd = 0; sd < 2; ++sd) {
      if (pb->bc[k][sd] != BGK_BC_DIFFUSE) continue;
      const int q = W.nside++;
      const int nface = (int)(s->L.ne / pb->nelem[k]);
      W.side_k[q] = k;
      W.side_s[q] = sd;
      W.off[q] = off;
      W.nface[q] = nface;
      W.blk0[q] = blk;
      off += nface * nf;
      blk += nface * s->L.nchunk;
      const double th = pb->wall_theta[k][sd];
      const double* U = pb->wall_vel[k][sd];
      const double norm = 1.0 / pow(2.0 * M_PI * th, 1.5), i2t = 1.0 / (2.0 * th);
      const DevGeom& g = s->g;
      double in = 0.0;
      for (int bz = 0; bz < g.nv1[2]; ++bz)
        for (int by = 0; by < g.nv1[1]; ++by)
          for (int bx = 0; bx < g.nv1[0]; ++bx) {
            const int b[3] = {bx, by, bz};
            double u[3], w = 1.0;
            for (int c = 0; c < 3; ++c) {
              u[c] = g.vlo[c] + b[c] * g.du[c];
              double wc = g.du[c];
              if (b[c] == 0 || b[c] == g.nv1[c] - 1) wc *= 0.5;
              w *= wc;
            }
            const double a = u[k];
            if (sd == 0 ? !(a > 0.0) : !(a < 0.0)) continue;
            const double d2 = (u[0] - U[0]) * (u[0] - U[0]) + (u[1] - U[1]) * (u[1] - U[1]) +
                              (u[2] - U[2]) * (u[2] - U[2]);
            in += w * fabs(a) * norm * exp(-d2 * i2t);
          }
      double* c = s->wallp_host.data() + (k * 2 + sd) * 8;
      c[0] = norm;
      c[1] = i2t;
      c[2] = U[0];
      c[3] = U[1];
      c[4] = U[2];
      c[5] = 1.0 / in;
    }
  }
  W.blk0[W.nside] = blk;  // end of the last side's blocks
  W.npoints = off;
}

// Brick traversal of a hexahedral mesh: bricks of 4 x 4 x 4 elements
// (clipped at the mesh boundary) in lexicographic brick order, elements
// lexicographic inside a brick.
void brick_order(const int32_t* ne, std::vector<int32_t>& out) {
  const int B = 4;
  out.clear();
  out.reserve((size_t)ne[0] * ne[1] * ne[2]);
  for (int bz = 0; bz < ne[2]; bz += B)
    for (int by = 0; by < ne[1]; by += B)
      for (int bx = 0; bx < ne[0]; bx += B)
        for (int z = bz; z < std::min(bz + B, ne[2]); ++z)
          for (int y = by; y < std::min(by + B, ne[1]); ++y)
            for (int x = bx; x < std::min(bx + B, ne[0]); ++x)
              out.push_back(x + ne[0] * (y + ne[1] * z));
}

bgk_status moments_of(bgk_solver* s, const void* fstore) {
  StageArgs A = stage_args(s);
  A.fin = fstore;
  HIP_TRY(launch_stage(s->precision, 2, A, s->stream));
  return BGK_OK;
}

bgk_status ensure_partials(bgk_solver* s) {
  if (!s->partials_valid) {
    bgk_status st = moments_of(s, s->state());
    if (st) return st;
    s->partials_valid = true;
  }
  return BGK_OK;
}

bgk_status check_failed(bgk_solver* s) {
  HIP_TRY(hipStreamSynchronize(s->stream));
  if (!s->counters_ready) return BGK_OK;
  unsigned long long d[8];
  HIP_TRY(hipMemcpy(d, s->diag(), sizeof(d), hipMemcpyDeviceToHost));
  if (d[1] > 0) {
    s->failed = true;
    return fail(BGK_ERR_NEWTON, "%llu node solve(s) failed (non-realizable moments or Newton "
                "not converged)", d[1]);
  }
  return BGK_OK;
}

// Install n canonical FP64 values from host into the internal layout at dst
// (storage precision), staging windows of the canonical array through the
// device scratch region [stage, stage + cap).
bgk_status host_to_storage(bgk_solver* s, const double* h, void* dst, int64_t n, char* stage,
                           size_t cap) {
  const int64_t per = (int64_t)(cap / 8);
  for (int64_t o = 0; o < n; o += per) {
    const int64_t m = std::min(per, n - o);
    HIP_TRY(hipMemcpyAsync(stage, h + o, (size_t)m * 8, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(launch_to_storage(s->precision, s->g, (const double*)stage, dst, o, m, s->stream));
  }
  return BGK_OK;
}

// Copy the state at src (internal layout) to n canonical FP64 values on the host.
bgk_status storage_to_host(bgk_solver* s, const void* src, double* h, int64_t n, char* stage,
                           size_t cap) {
  const int64_t per = (int64_t)(cap / 8);
  for (int64_t o = 0; o < n; o += per) {
    const int64_t m = std::min(per, n - o);
    HIP_TRY(launch_from_storage(s->precision, s->g, src, (double*)stage, o, m, s->stream));
    HIP_TRY(hipMemcpyAsync(h + o, stage, (size_t)m * 8, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
  }
  return BGK_OK;
}

// Record the next timing event on the stream (timing mode only).
bgk_status mark(bgk_solver* s) {
  if (!s->timing) return BGK_OK;
  if (s->used == s->pool.size()) {
    hipEvent_t e;
    HIP_TRY(hipEventCreate(&e));
    s->pool.push_back(e);
  }
  HIP_TRY(hipEventRecord(s->pool[s->used++], s->stream));
  return BGK_OK;
}

bgk_status reset_state_flags(bgk_solver* s) {
  HIP_TRY(hipMemsetAsync(s->diag(), 0, 8 * sizeof(unsigned long long), s->stream));
  s->counters_ready = true;
  {
    bgk_status st = ensure_counters(s);
    if (st) return st;
  }
  s->failed = false;
  s->has_state = true;
  s->partials_valid = false;
  return BGK_OK;
}

}  // namespace

namespace {

// Fill a solver object for problem *pb over the device memory ws (a validated
// problem). With brick = false the elements are visited in lexicographic
// order and every work-group loads all entries of its element's equilibrium
// rows (results are the same bit for bit; the brick order and the per-chunk
// row entries only save memory traffic) and, without diffuse walls, the host
// side allocates nothing.
void init_solver(bgk_solver* s, const bgk_problem* pb, char* ws, hipStream_t stream, bool brick) {
  s->pb = *pb;
  s->L = layout_of(pb);
  s->ws = ws;
  s->stream = stream;
  s->precision = pb->precision;
  s->gamma = pb->gamma > 0.0 ? pb->gamma : 5.0 / 3.0;
  DevGeom& g = s->g;
  memset(&g, 0, sizeof(g));
  g.dim = pb->dim;
  g.n1 = pb->order + 1;
  g.ns = s->L.ns;
  for (int k = 0; k < 3; ++k) {
    g.nelem[k] = k < pb->dim ? pb->nelem[k] : 1;
    g.bc[k][0] = k < pb->dim ? pb->bc[k][0] : 0;
    g.bc[k][1] = k < pb->dim ? pb->bc[k][1] : 0;
    g.scale[k] = k < pb->dim ? 2.0 / ((pb->xhi[k] - pb->xlo[k]) / pb->nelem[k]) : 0.0;
    g.nv1[k] = pb->nvel[k];
    g.vlo[k] = pb->vlo[k];
    g.du[k] = (pb->vhi[k] - pb->vlo[k]) / (pb->nvel[k] - 1);
  }
  g.tabw = pb->nvel[0] + pb->nvel[1] + pb->nvel[2] + 1;
  g.ne = s->L.ne;
  g.nx = s->L.nx;
  g.nv = s->L.nv;
  g.nvb = s->L.nvb;
  g.nchunk = s->L.nchunk;
  // velocity slots: octants of the signs of the transported components. FP64
  // hexahedra on the plane-split kernels keep the lexicographic order (no
  // split): they measured 4 % faster with it on the 16^3 x 16^3 Taylor-Green
  // box, where the one-lane FP32 hexahedra ran 6 % faster with the octants.
  set_velocity_slots(g, !(pb->dim == 3 && pb->precision == BGK_FP64 &&
                          !hex_one_lane(pb->order, pb->precision)));
  build_ops(g.n1, g.dim, s->op);
  if (brick && pb->dim == 3) brick_order(g.nelem, s->order_host);
  if (brick) {
    // the row entries each velocity chunk of the stage kernels reads
    const int vb = velocities_per_block(pb->dim, pb->order, pb->precision);
    s->rcols_host.resize(g.nchunk);
    for (int c = 0; c < g.nchunk; ++c)
      s->rcols_host[c] = row_cols(g, c * vb, (int)std::min<int64_t>((int64_t)(c + 1) * vb, g.nv));
  }
  setup_walls(s);
  if (brick) s->sweep_seg = sweep_segment(g, pb->precision, pb->mu_ref > 0.0);
  if (brick) {
    // XCDs sharing a velocity chunk in the stage launches (xcd_chunk_remap):
    // all eight for column sweeps (tgv3d FP32 3.15 against 3.25 ms per
    // launch, box2d FP64 1 % faster), four for the plane-split hexahedra
    // (tgv3d FP64 1.5 %, BF16 increments 1 % faster); contiguous ranges for
    // the per-element one-lane kernels (the Mach-2 box 2 % slower with eight).
    // BGK_XCD_PART overrides the choice (0: contiguous ranges).
    const char* env = getenv("BGK_XCD_PART");
    s->xcd_part = env                                            ? atoi(env)
                  : s->sweep_seg > 0                             ? 8
                  : pb->dim == 3 && !hex_one_lane(pb->order, pb->precision) ? 4
                                                                 : 0;
  }
}

}  // namespace

extern "C" {

const char* bgk_status_str(bgk_status st) {
  switch (st) {
    case BGK_OK: return "BGK_OK";
    case BGK_ERR_INVALID_ARG: return "BGK_ERR_INVALID_ARG";
    case BGK_ERR_UNSUPPORTED: return "BGK_ERR_UNSUPPORTED";
    case BGK_ERR_OUT_OF_MEMORY: return "BGK_ERR_OUT_OF_MEMORY";
    case BGK_ERR_DEVICE: return "BGK_ERR_DEVICE";
    case BGK_ERR_NEWTON: return "BGK_ERR_NEWTON";
    case BGK_ERR_NONFINITE: return "BGK_ERR_NONFINITE";
    case BGK_ERR_STATE: return "BGK_ERR_STATE";
  }
  return "BGK_UNKNOWN";
}

const char* bgk_last_error(void) { return g_last_error.c_str(); }

bgk_status bgk_query_footprint(const bgk_problem* pb, size_t* bytes, int64_t* nx, int64_t* nv) {
  bgk_status st = validate(pb);
  if (st) return st;
  Layout L = layout_of(pb);
  // one launch dimension holds < 2^32 work-items (threads)
  if ((double)L.nchunk * (double)L.ne * kBlock >= 4294967296.0 ||
      (double)L.nx * 16.0 >= 4294967296.0)
    return fail(BGK_ERR_UNSUPPORTED, "problem too large for one launch grid");
  if (bytes) *bytes = L.total;
  if (nx) *nx = L.nx;
  if (nv) *nv = L.nv;
  return BGK_OK;
}

bgk_status bgk_create(const bgk_problem* pb, void* ws, size_t bytes, void* stream,
                      bgk_solver** out) {
  if (!out) return fail(BGK_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  size_t need = 0;
  bgk_status st = bgk_query_footprint(pb, &need, nullptr, nullptr);
  if (st) return st;
  if (!ws) return fail(BGK_ERR_INVALID_ARG, "workspace is NULL");
  if (((uintptr_t)ws) % kAlign) return fail(BGK_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  if (bytes < need)
    return fail(BGK_ERR_OUT_OF_MEMORY, "workspace %zu bytes < footprint %zu", bytes, need);
  bgk_solver* s = new (std::nothrow) bgk_solver();
  if (!s) return fail(BGK_ERR_OUT_OF_MEMORY, "host allocation failed");
  init_solver(s, pb, (char*)ws, (hipStream_t)stream, true);
  *out = s;
  return BGK_OK;
}

bgk_status bgk_destroy(bgk_solver* s) {
  if (s && s->in_batch) return fail(BGK_ERR_STATE, "solver is a batch member; remove or poll it");
  if (s)
    for (hipEvent_t e : s->pool) (void)hipEventDestroy(e);
  delete s;
  return BGK_OK;
}

bgk_status bgk_set_stream(bgk_solver* s, void* hip_stream) {
  if (!s) return fail(BGK_ERR_INVALID_ARG, "NULL solver");
  if (s->in_batch) return fail(BGK_ERR_STATE, "solver is a batch member");
  HIP_TRY(hipStreamSynchronize(s->stream));
  if (s->timing) {
    s->used = 0;
    s->kinds.clear();
  }
  s->stream = (hipStream_t)hip_stream;
  return BGK_OK;
}

bgk_status bgk_node_coords(const bgk_solver* s, double* x) {
  if (!s || !x) return fail(BGK_ERR_INVALID_ARG, "NULL argument");
  double xi[kMaxN1];
  gauss_nodes(s->g.n1, xi);
  const int d = s->g.dim, n1 = s->g.n1, ns = s->g.ns;
  for (int64_t e = 0; e < s->g.ne; ++e) {
    int64_t r = e;
    int ek[3] = {0, 0, 0};
    for (int k = 0; k < d; ++k) {
      ek[k] = (int)(r % s->g.nelem[k]);
      r /= s->g.nelem[k];
    }
    for (int i = 0; i < ns; ++i) {
      int q = i;
      for (int k = 0; k < d; ++k) {
        const int a = q % n1;
        q /= n1;
        const double h = (s->pb.xhi[k] - s->pb.xlo[k]) / s->pb.nelem[k];
        x[(e * ns + i) * d + k] = s->pb.xlo[k] + h * (ek[k] + 0.5 * (1.0 + xi[a]));
      }
    }
  }
  return BGK_OK;
}

bgk_status bgk_velocity_grid(const bgk_solver* s, double* u, double* w) {
  if (!s) return fail(BGK_ERR_INVALID_ARG, "NULL solver");
  const DevGeom& g = s->g;
  for (int64_t j = 0; j < g.nv; ++j) {
    const int b[3] = {(int)(j % g.nv1[0]), (int)((j / g.nv1[0]) % g.nv1[1]),
                      (int)(j / ((int64_t)g.nv1[0] * g.nv1[1]))};
    double wj = 1.0;
    for (int c = 0; c < 3; ++c) {
      if (u) u[3 * j + c] = g.vlo[c] + b[c] * g.du[c];
      double wc = g.du[c];
      if (b[c] == 0 || b[c] == g.nv1[c] - 1) wc *= 0.5;
      wj *= wc;
    }
    if (w) w[j] = wj;
  }
  return BGK_OK;
}

bgk_status bgk_set_state(bgk_solver* s, const double* f, int32_t where) {
  if (!s || !f) return fail(BGK_ERR_INVALID_ARG, "NULL argument");
  if (where != BGK_HOST && where != BGK_DEVICE) return fail(BGK_ERR_INVALID_ARG, "bad where");
  const int64_t n = s->L.nx * s->L.nv;
  if (where == BGK_DEVICE) {
    HIP_TRY(launch_to_storage(s->precision, s->g, f, s->f(0), 0, n, s->stream));
  } else {
    bgk_status st = host_to_storage(s, f, s->f(0), n, (char*)s->f(1),
                                    s->L.f[2] + s->L.fsz[2] - s->L.f[1]);
    if (st) return st;
  }
  s->cur = 0;
  return reset_state_flags(s);
}

bgk_status bgk_set_maxwellian(bgk_solver* s, const double* prim, int32_t where) {
  if (!s || !prim) return fail(BGK_ERR_INVALID_ARG, "NULL argument");
  if (where != BGK_HOST && where != BGK_DEVICE) return fail(BGK_ERR_INVALID_ARG, "bad where");
  const double* dprim = prim;
  if (where == BGK_HOST) {
    for (int64_t i = 0; i < s->L.nx; ++i)
      if (!(prim[5 * i] > 0.0) || !(prim[5 * i + 4] > 0.0))
        return fail(BGK_ERR_INVALID_ARG, "node %lld: rho and theta must be > 0", (long long)i);
    HIP_TRY(hipMemcpyAsync(s->prim(), prim, (size_t)s->L.nx * 5 * 8, hipMemcpyHostToDevice,
                           s->stream));
    dprim = s->prim();
  }
  HIP_TRY(launch_maxwellian(s->precision, s->g, dprim, s->f(0), s->stream));
  s->cur = 0;
  bgk_status st = reset_state_flags(s);
  if (where == BGK_HOST) HIP_TRY(hipStreamSynchronize(s->stream));
  return st;
}

bgk_status bgk_get_state(bgk_solver* s, double* f, int32_t where) {
  if (!s || !f) return fail(BGK_ERR_INVALID_ARG, "NULL argument");
  if (!s->has_state) return fail(BGK_ERR_STATE, "no state installed");
  if (where != BGK_HOST && where != BGK_DEVICE) return fail(BGK_ERR_INVALID_ARG, "bad where");
  const int64_t n = s->L.nx * s->L.nv;
  if (where == BGK_DEVICE) {
    HIP_TRY(launch_from_storage(s->precision, s->g, s->state(), f, 0, n, s->stream));
  } else {
    // staging: device memory that does not hold the state
    char* stage = (char*)(s->cur == 0 ? s->f(1) : s->f(0));
    const size_t cap = s->cur == 0 ? s->L.f[2] + s->L.fsz[2] - s->L.f[1] : s->L.fsz[0];
    bgk_status st = storage_to_host(s, s->state(), f, n, stage, cap);
    if (st) return st;
  }
  return check_failed(s);
}

bgk_status bgk_residual(bgk_solver* s, const double* f_in, double* r_out, int32_t where) {
  if (!s || !r_out) return fail(BGK_ERR_INVALID_ARG, "NULL argument");
  if (where != BGK_HOST && where != BGK_DEVICE) return fail(BGK_ERR_INVALID_ARG, "bad where");
  if (s->failed) return fail(BGK_ERR_STATE, "solver failed earlier; install a new state");
  if (!f_in && !s->has_state) return fail(BGK_ERR_STATE, "no state installed");
  {
    bgk_status st = ensure_counters(s);
    if (st) return st;
  }
  const int64_t n = s->L.nx * s->L.nv;
  const void* fin = s->state();
  if (f_in) {
    // f_in goes to the state-precision buffer that does not hold the state
    void* dst = s->f(1 - s->cur);
    if (where == BGK_DEVICE) {
      HIP_TRY(launch_to_storage(s->precision, s->g, f_in, dst, 0, n, s->stream));
    } else {
      // staged through f2
      bgk_status st = host_to_storage(s, f_in, dst, n, (char*)s->f(2), s->L.fsz[2]);
      if (st) return st;
    }
    fin = dst;
    bgk_status st = moments_of(s, fin);
    if (st) return st;
    s->partials_valid = false;  // the partials now belong to f_in
  } else {
    bgk_status st = ensure_partials(s);
    if (st) return st;
  }
  NewtonArgs N = newton_args(s);
  HIP_TRY(launch_newton(N, s->stream));
  {
    bgk_status st = wall_densities(s, fin, s->stream);
    if (st) return st;
  }
  StageArgs A = stage_args(s);
  A.fin = fin;
  if (where == BGK_DEVICE) {
    A.out = r_out;
    HIP_TRY(launch_stage(s->precision, 1, A, s->stream));
    return BGK_OK;
  }
  // host output: element ranges that fit the f2 region as FP64
  const size_t per_elem = (size_t)s->L.ns * s->L.nv * 8;
  const int64_t cap = (int64_t)(s->L.fsz[2] / per_elem);
  if (cap < 1)
    return fail(BGK_ERR_UNSUPPORTED, "host residual with FP32 storage needs >= 2 elements; "
                "use device buffers");
  A.order = nullptr;  // element ranges: lexicographic
  for (int64_t e0 = 0; e0 < s->L.ne; e0 += cap) {
    A.e0 = e0;
    A.ecount = std::min(cap, s->L.ne - e0);
    A.out_e0 = e0;
    A.out = s->f(2);
    HIP_TRY(launch_stage(s->precision, 1, A, s->stream));
    HIP_TRY(hipMemcpyAsync(r_out + e0 * s->L.ns * s->L.nv, s->f(2), (size_t)A.ecount * per_elem,
                           hipMemcpyDeviceToHost, s->stream));
  }
  return check_failed(s);
}

}  // extern "C"

namespace {

// Queue nsteps SSP-RK3 steps of one solver on stream st (the partials of the
// state must be valid). Timing marks only when `timed` (never under capture).
bgk_status rk3_launch(bgk_solver* s, double dt, int32_t nsteps, hipStream_t st, bool timed) {
  static const double kA[3] = {0.0, 0.75, 1.0 / 3.0};
  static const double kB[3] = {1.0, 0.25, 2.0 / 3.0};
  bgk_status rc;
  NewtonArgs N = newton_args(s);
  N.Q = nullptr;
  StageArgs A = stage_args(s);
  A.dt = dt;
  const bool inc = s->precision == BGK_BF16;
  if (timed) {
    if (s->used > 0) s->kinds.push_back(2);  // host gap between calls: not a kernel
    if ((rc = mark(s))) return rc;
  }
  for (int32_t step = 0; step < nsteps; ++step) {
    // FP64/FP32: f(0) = f^n -> f(1) -> f(2) -> f(0) (the last stage reads f^n
    // only at its own point, so it may overwrite it). BF16: F = f(cur) is
    // f^n; the first increment goes to f(1 - cur) (as BF16), the second to
    // f(2), and f^(n+1) to f(1 - cur) in FP32, which then holds the state.
    const int fa = s->cur, fb = 1 - s->cur;
    A.fn = s->f(fa);
    for (int k = 0; k < 3; ++k) {
      HIP_TRY(launch_newton(N, st));
      if (!inc && (rc = wall_densities(s, s->f(k), st))) return rc;
      if (timed) {
        s->kinds.push_back(0);
        if ((rc = mark(s))) return rc;
      }
      if (inc) {
        A.fin = s->f(fa);
        A.din = k == 0 ? nullptr : (const uint16_t*)(k == 1 ? s->f(fb) : s->f(2));
        A.out = k == 1 ? s->f(2) : s->f(fb);
        A.out_full = k == 2;
      } else {
        A.fin = s->f(k);
        A.out = s->f((k + 1) % 3);
      }
      A.a = kA[k];
      A.b = kB[k];
      HIP_TRY(launch_stage(s->precision, 0, A, st));
      if (timed) {
        s->kinds.push_back(1);
        if ((rc = mark(s))) return rc;
      }
    }
    if (inc) s->cur = fb;
  }
  return BGK_OK;
}

}  // namespace

extern "C" {

bgk_status bgk_rk3_step(bgk_solver* s, double dt, int32_t nsteps) {
  if (!s) return fail(BGK_ERR_INVALID_ARG, "NULL solver");
  if (!(dt > 0.0) || !isfinite(dt)) return fail(BGK_ERR_INVALID_ARG, "dt must be > 0");
  if (nsteps < 0) return fail(BGK_ERR_INVALID_ARG, "nsteps < 0");
  if (!s->has_state) return fail(BGK_ERR_STATE, "no state installed");
  if (s->failed) return fail(BGK_ERR_STATE, "solver failed earlier; install a new state");
  if (s->in_batch) return fail(BGK_ERR_STATE, "solver is a batch member; step the batch");
  bgk_status st = ensure_partials(s);
  if (st) return st;
  return rk3_launch(s, dt, nsteps, s->stream, s->timing);
}

bgk_status bgk_timing_enable(bgk_solver* s, int32_t on) {
  if (!s) return fail(BGK_ERR_INVALID_ARG, "NULL solver");
  if (!on && s->timing) {
    HIP_TRY(hipStreamSynchronize(s->stream));
    s->used = 0;
    s->kinds.clear();
  }
  s->timing = on != 0;
  return BGK_OK;
}

bgk_status bgk_timing_read(bgk_solver* s, bgk_timing* out) {
  if (!s || !out) return fail(BGK_ERR_INVALID_ARG, "NULL argument");
  memset(out, 0, sizeof(*out));
  HIP_TRY(hipStreamSynchronize(s->stream));
  for (size_t i = 0; i < s->kinds.size() && i + 1 < s->used; ++i) {
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, s->pool[i], s->pool[i + 1]));
    if (s->kinds[i] == 1) {
      out->stage_launches += 1;
      out->stage_ms += ms;
    } else if (s->kinds[i] == 0) {
      out->newton_launches += 1;
      out->newton_ms += ms;
    }
  }
  s->used = 0;
  s->kinds.clear();
  return BGK_OK;
}

bgk_status bgk_moments(bgk_solver* s, double* Q, int32_t where) {
  if (!s || !Q) return fail(BGK_ERR_INVALID_ARG, "NULL argument");
  if (!s->has_state) return fail(BGK_ERR_STATE, "no state installed");
  if (where != BGK_HOST && where != BGK_DEVICE) return fail(BGK_ERR_INVALID_ARG, "bad where");
  bgk_status st = ensure_partials(s);
  if (st) return st;
  double* dst = where == BGK_DEVICE ? Q : s->Q();
  HIP_TRY(launch_reduce_partials(s->g, s->partials(), dst, s->stream));
  if (where == BGK_HOST)
    HIP_TRY(hipMemcpyAsync(Q, s->Q(), (size_t)s->L.nx * 5 * 8, hipMemcpyDeviceToHost, s->stream));
  return check_failed(s);
}

bgk_status bgk_collision_moments(bgk_solver* s, double* Cm, int32_t where) {
  if (!s || !Cm) return fail(BGK_ERR_INVALID_ARG, "NULL argument");
  if (!s->has_state) return fail(BGK_ERR_STATE, "no state installed");
  if (where != BGK_HOST && where != BGK_DEVICE) return fail(BGK_ERR_INVALID_ARG, "bad where");
  if (s->failed) return fail(BGK_ERR_STATE, "solver failed earlier; install a new state");
  if (s->in_batch) return fail(BGK_ERR_STATE, "solver is a batch member");
  const size_t bytes = (size_t)s->L.nx * 5 * 8;
  if (!(s->pb.mu_ref > 0.0)) {  // collisions off: the term is zero
    if (where == BGK_HOST) {
      memset(Cm, 0, bytes);
      return BGK_OK;
    }
    HIP_TRY(hipMemsetAsync(Cm, 0, bytes, s->stream));
    return check_failed(s);
  }
  bgk_status st = ensure_counters(s);
  if (st) return st;
  if ((st = ensure_partials(s))) return st;
  NewtonArgs N = newton_args(s);
  N.Q = nullptr;
  HIP_TRY(launch_newton(N, s->stream));
  StageArgs A = stage_args(s);
  A.fin = s->state();
  double* dst = where == BGK_DEVICE ? Cm : s->Q();
  HIP_TRY(launch_collision_moments(s->precision, A, dst, s->stream));
  s->partials_valid = false;  // the partials buffer served as scratch
  if (where == BGK_HOST)
    HIP_TRY(hipMemcpyAsync(Cm, s->Q(), bytes, hipMemcpyDeviceToHost, s->stream));
  return check_failed(s);
}

bgk_status bgk_stable_dt(bgk_solver* s, double cfl, double* dt) {
  if (!s || !dt) return fail(BGK_ERR_INVALID_ARG, "NULL argument");
  if (!(cfl > 0.0)) return fail(BGK_ERR_INVALID_ARG, "cfl must be > 0");
  const DevGeom& g = s->g;
  double smax = 0.0;
  for (int bz = 0; bz < g.nv1[2]; ++bz)
    for (int by = 0; by < g.nv1[1]; ++by)
      for (int bx = 0; bx < g.nv1[0]; ++bx) {
        const int b[3] = {bx, by, bz};
        double sum = 0.0;
        for (int k = 0; k < g.dim; ++k) sum += fabs(g.vlo[k] + b[k] * g.du[k]) * (0.5 * g.scale[k]);
        smax = std::max(smax, sum);
      }
  double out = cfl / smax;
  if (s->pb.mu_ref > 0.0) {
    if (!s->has_state) return fail(BGK_ERR_STATE, "no state installed");
    double* Qh = new (std::nothrow) double[(size_t)s->L.nx * 5];
    if (!Qh) return fail(BGK_ERR_OUT_OF_MEMORY, "host allocation failed");
    bgk_status st = bgk_moments(s, Qh, BGK_HOST);
    if (st) {
      delete[] Qh;
      return st;
    }
    double tmin = INFINITY;
    for (int64_t i = 0; i < s->L.nx; ++i) {
      const double* q = Qh + 5 * i;
      const double rho = q[0];
      const double UU = (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / (rho * rho);
      const double P = (s->gamma - 1.0) * (q[4] - 0.5 * rho * UU);
      const double th = P / rho;
      const double tr = th / s->pb.theta_ref, S = s->pb.sutherland;
      const double mu = S > 0.0 ? s->pb.mu_ref * tr * sqrt(tr) * (s->pb.theta_ref + S) / (th + S)
                                : s->pb.mu_ref * pow(tr, s->pb.omega);
      const double tau = mu / P;
      tmin = std::min(tmin, tau);
    }
    delete[] Qh;
    out = std::min(out, tmin);
  }
  *dt = out;
  return BGK_OK;
}

bgk_status bgk_diagnostics(bgk_solver* s, bgk_diag* out) {
  if (!s || !out) return fail(BGK_ERR_INVALID_ARG, "NULL argument");
  unsigned long long d[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (s->counters_ready) {
    HIP_TRY(hipStreamSynchronize(s->stream));
    HIP_TRY(hipMemcpy(d, s->diag(), sizeof(d), hipMemcpyDeviceToHost));
  }
  out->newton_it_max = (int64_t)d[0];
  out->newton_fail = (int64_t)d[1];
  out->limiter_hits = (int64_t)d[2];
  out->limiter_bad = (int64_t)d[3];
  out->stages = (int64_t)d[4];
  out->positivity_violations = (int64_t)d[5];
  if (d[1] > 0) {
    s->failed = true;
    return fail(BGK_ERR_NEWTON, "%llu node solve(s) failed", d[1]);
  }
  return BGK_OK;
}

bgk_status bgk_synchronize(bgk_solver* s) {
  if (!s) return fail(BGK_ERR_INVALID_ARG, "NULL solver");
  return check_failed(s);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Residual without allocation: the solver's device memory is a file-scope
// device array (one copy per GPU the library runs on, held until the process
// ends). Host code reaches that memory only through the address
// hipGetSymbolAddress returns for the current device; the array's name in
// host code is not a device address.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[BGK_NOALLOC_SCRATCH_BYTES];

// Set n 64-bit words to a value (a kernel, where a memset node is not wanted:
// the entry point below may sit under graph capture).
__global__ void __launch_bounds__(256) k_fill_u64(unsigned long long* p, int64_t n,
                                                   unsigned long long v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Store one row-entry descriptor (a kernel, for the same reason).
__global__ void k_store_rowcols(RowCols* p, RowCols v) {
  if (threadIdx.x == 0) *p = v;
}

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Address of the scratch array on the current device, looked up once per device.
bgk_status scratch_address(void** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(BGK_ERR_UNSUPPORTED, "device %d >= %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(BGK_ERR_DEVICE, "hipGetSymbolAddress returned NULL for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return BGK_OK;
}

// Residual layout inside the scratch array: one internal copy of the input,
// then the partials, equilibrium parameters and rows, and the counters (the
// solver's other regions are not used by a residual evaluation).
Layout residual_layout(const bgk_problem* pb) {
  Layout L = layout_of(pb);
  size_t off = 0;
  L.f[0] = L.f[1] = L.f[2] = 0;
  off = align_up(L.fbytes);
  L.partials = off;
  off = align_up(off + (size_t)L.nx * L.nchunk * 5 * sizeof(double));
  L.params = off;
  off = align_up(off + (size_t)L.nx * 8 * sizeof(double));
  L.etab = off;
  off = align_up(off + (size_t)L.nx * (pb->nvel[0] + pb->nvel[1] + pb->nvel[2] + 1) *
                           sizeof(double));
  L.diag = off;
  off = align_up(off + 8 * sizeof(unsigned long long));
  L.rcols = off;  // one entry (every row entry) for every velocity chunk
  off = align_up(off + sizeof(RowCols));
  L.order = L.Q = L.prim = L.wallp = L.wall_part = L.wall_rho = off;
  L.total = off;
  return L;
}

}  // namespace

extern "C" {

bgk_status bgk_residual_noalloc(const bgk_problem* pb, const double* f_in, double* r_out,
                                void* hip_stream) {
  if (!pb || !f_in || !r_out) return fail(BGK_ERR_INVALID_ARG, "NULL argument");
  bgk_status st = bgk_query_footprint(pb, nullptr, nullptr, nullptr);
  if (st) return st;
  for (int k = 0; k < pb->dim; ++k)
    if (pb->bc[k][0] == BGK_BC_DIFFUSE || pb->bc[k][1] == BGK_BC_DIFFUSE)
      return fail(BGK_ERR_UNSUPPORTED, "bgk_residual_noalloc: diffuse walls are not supported");
  const Layout L = residual_layout(pb);
  if (L.total > (size_t)BGK_NOALLOC_SCRATCH_BYTES)
    return fail(BGK_ERR_OUT_OF_MEMORY,
                "bgk_residual_noalloc: problem needs %zu bytes of scratch, the static array holds %zu",
                L.total, (size_t)BGK_NOALLOC_SCRATCH_BYTES);
  void* base = nullptr;
  if ((st = scratch_address(&base))) return st;
  // solver object on the stack: lexicographic element order, no diffuse walls,
  // so nothing is allocated on the host either
  bgk_solver s;
  init_solver(&s, pb, (char*)base, (hipStream_t)hip_stream, false);
  s.L = L;
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(256), 0, s.stream, s.diag(), (int64_t)8, 0ull);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_store_rowcols, dim3(1), dim3(64), 0, s.stream, s.rcols(),
                     row_cols_all(s.g));
  HIP_TRY(hipGetLastError());
  const int64_t n = L.nx * L.nv;
  HIP_TRY(launch_to_storage(s.precision, s.g, f_in, s.f(0), 0, n, s.stream));
  if ((st = moments_of(&s, s.f(0)))) return st;
  NewtonArgs N = newton_args(&s);
  N.Q = nullptr;
  HIP_TRY(launch_newton(N, s.stream));
  StageArgs A = stage_args(&s);
  A.fin = s.f(0);
  A.out = r_out;
  HIP_TRY(launch_stage(s.precision, 1, A, s.stream));
  return BGK_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches: resident solvers advanced together. The arguments of every member
// live in descriptor tables in the batch's device workspace: the StageArgs of
// its three RK stages, its NewtonArgs and the WallArgs of its stages, and per
// launch a BatchList naming the members it covers with the prefix sums of
// their work units. A replay runs up to kSub sub-steps; each is three RK
// stages of [equilibrium solves per team size, wall fluxes per family and wall
// densities, one stage launch per kernel family (dimension, order, storage
// precision)], every launch covering all members of its list, with the grid
// set to the list's work units. Admission and completion rewrite the tables
// (copied on the batch stream, ahead of the launches that read them).
// ---------------------------------------------------------------------------
namespace {

constexpr int kSub = 4;            // sub-steps per replay (a member takes up to 4 steps)
constexpr int kMaxFamilies = 12;   // dimension 1-2 x order 1-3 x FP64/FP32
// Stage work items (element x velocity chunk) from which a member fills the
// device alone (32 work-groups per compute unit) and runs its RK stages with
// its solo launches: the 2-D boxes of the serving mix above about 4e8 DOF
// (the FP64 column sweep is some 8 % faster than the per-element items there).
constexpr int64_t kSoloUnits = 8192;
constexpr int kTeamLists = 3;      // equilibrium teams of 16, 4, 2 lanes
constexpr int kAllList = kMaxFamilies + kTeamLists;  // every member (wall densities)
constexpr int kListsPerSub = kAllList + 1;
constexpr int kTeamOfList[kTeamLists] = {16, 4, 2};

struct TableLayout {
  size_t args, nargs, wargs, lists, total;
};

TableLayout table_layout() {
  TableLayout t;
  size_t off = 0;
  t.args = off;
  off = align_up(off + sizeof(StageArgs) * kMaxBatchMembers * 3);
  t.nargs = off;
  off = align_up(off + sizeof(NewtonArgs) * kMaxBatchMembers);
  t.wargs = off;
  off = align_up(off + sizeof(WallArgs) * kMaxBatchMembers * 3);
  t.lists = off;
  off = align_up(off + sizeof(BatchList) * kSub * kListsPerSub);
  t.total = off;
  return t;
}

int team_index(int team) { return team == 16 ? 0 : team == 4 ? 1 : 2; }

// work units of a member: stage work items, equilibrium work-groups
int64_t member_units(const bgk_solver* s) { return s->L.ne * s->L.nchunk; }
int64_t member_newton_blocks(const bgk_solver* s) {
  return (s->L.nx * newton_team(s->L.nx) + 255) / 256;
}

}  // namespace

struct bgk_batch {
  hipStream_t stream;
  int32_t max_members;
  char* ws;
  TableLayout tl;
  struct Member {
    bgk_solver* s;
    double dt;
    int64_t remaining;
    int64_t per_replay;  // steps per replay (set when the tables are written)
    int slot;
    int family;
    // a member that fills the device alone runs its RK stages with its solo
    // launches (column sweeps where its solver sweeps) instead of the family
    // launch; its equilibrium and wall work stays in the batched launches
    bool solo = false;
    StageArgs sargs[3];  // its stage arguments (set when the tables are written)
  };
  struct Family {
    int dim, order, precision;
    size_t tab_bytes;  // dynamic LDS of its stage launches (equilibrium rows)
  };
  struct Finished {
    bgk_solver* s;
    int64_t replay;  // the replay that completed its steps
    int slot;        // kept until the member is polled (its counter staging)
  };
  std::vector<Member> members;
  std::vector<Finished> finished;  // stepped to completion, not yet polled
  std::vector<int> free_slots;
  // replay completion: event ev[r % kEvents] is recorded after replay r; a
  // finished member's failure counters are copied to pinned diag[slot] ahead
  // of that event. At most kAhead replays are queued beyond the last one known
  // to have completed.
  static constexpr int kEvents = 32, kAhead = 8;
  hipEvent_t ev[kEvents] = {};
  int64_t replays = 0;
  unsigned long long* diag = nullptr;  // pinned [max_members][2]
  std::vector<Family> fams;           // families the lists can name
  bool tables_dirty = true;
  // work units of every list as last written: [sub][list] stage, newton,
  // wall-flux, wall-density (the launch grids)
  int32_t units[kSub][kListsPerSub][4];
  // pinned host staging of the tables, two buffers used in turn; an event
  // marks when the copy out of each has executed
  char* host[2] = {nullptr, nullptr};
  hipEvent_t copied[2] = {nullptr, nullptr};
  bool copy_pending[2] = {false, false};
  int next_host = 0;
  StageArgs* d_args() const { return (StageArgs*)(ws + tl.args); }
  NewtonArgs* d_nargs() const { return (NewtonArgs*)(ws + tl.nargs); }
  WallArgs* d_wargs() const { return (WallArgs*)(ws + tl.wargs); }
  BatchList* d_list(int sub, int l) const {
    return (BatchList*)(ws + tl.lists) + sub * kListsPerSub + l;
  }
};

namespace {

// Steps per replay: the member moving the most bytes per step takes one; a
// member moving W times fewer takes the largest power of two <= W (at most
// kSub and its remaining steps), so small requests are not paced by the
// largest.
void balance(bgk_batch* b) {
  double wmax = 0.0;
  for (auto& m : b->members) wmax = std::max(wmax, (double)m.s->L.fbytes);
  for (auto& m : b->members) {
    const double ratio = wmax / std::max(1.0, (double)m.s->L.fbytes);
    int64_t k = 1;
    while (2.0 * k <= ratio && 2 * k <= kSub) k *= 2;
    m.per_replay = std::min<int64_t>(k, m.remaining);
  }
}

// Write every descriptor into the next host staging buffer and queue its copy
// to the device tables on the batch stream.
bgk_status upload_tables(bgk_batch* b) {
  balance(b);
  const int h = b->next_host;
  b->next_host ^= 1;
  if (b->copy_pending[h]) HIP_TRY(hipEventSynchronize(b->copied[h]));
  char* host = b->host[h];
  StageArgs* args = (StageArgs*)(host + b->tl.args);
  NewtonArgs* nargs = (NewtonArgs*)(host + b->tl.nargs);
  WallArgs* wargs = (WallArgs*)(host + b->tl.wargs);
  BatchList* lists = (BatchList*)(host + b->tl.lists);
  static const double kA[3] = {0.0, 0.75, 1.0 / 3.0};
  static const double kB[3] = {1.0, 0.25, 2.0 / 3.0};
  for (auto& m : b->members) {
    bgk_solver* s = m.s;
    m.solo = member_units(s) >= kSoloUnits;
    // the arguments bgk_rk3_step passes for FP64/FP32 storage
    StageArgs A = stage_args(s);
    A.dt = m.dt;
    A.fn = s->f(0);
    for (int k = 0; k < 3; ++k) {
      A.fin = s->f(k);
      A.out = s->f((k + 1) % 3);
      A.a = kA[k];
      A.b = kB[k];
      args[m.slot * 3 + k] = A;
      m.sargs[k] = A;
      WallArgs W = s->wall;
      W.fin = s->f(k);
      wargs[m.slot * 3 + k] = W;
    }
    NewtonArgs N = newton_args(s);
    N.Q = nullptr;
    nargs[m.slot] = N;
  }
  for (int sub = 0; sub < kSub; ++sub) {
    BatchList* L = lists + sub * kListsPerSub;
    for (int l = 0; l < kListsPerSub; ++l) {
      L[l].n = 0;
      L[l].stage_off[0] = L[l].newton_off[0] = L[l].wflux_off[0] = L[l].wrho_off[0] = 0;
    }
    for (auto& m : b->members) {
      if (m.per_replay <= sub) continue;
      const bgk_solver* s = m.s;
      const int64_t wf = s->wall.nside ? s->wall.blk0[s->wall.nside] : 0;
      const int64_t wr = s->wall.nside ? (s->wall.npoints + 255) / 256 : 0;
      const int ls[3] = {m.family, kMaxFamilies + team_index(newton_team(s->L.nx)), kAllList};
      for (int l : ls) {
        BatchList& B = L[l];
        const int i = B.n++;
        B.slot[i] = m.slot;
        B.stage_off[i + 1] =
            B.stage_off[i] + (int32_t)(l == m.family && !m.solo ? member_units(s) : 0);
        B.newton_off[i + 1] = B.newton_off[i] + (int32_t)member_newton_blocks(s);
        B.wflux_off[i + 1] = B.wflux_off[i] + (int32_t)wf;
        B.wrho_off[i + 1] = B.wrho_off[i] + (int32_t)wr;
      }
    }
    for (int l = 0; l < kListsPerSub; ++l) {
      const BatchList& B = L[l];
      b->units[sub][l][0] = B.stage_off[B.n];
      b->units[sub][l][1] = B.newton_off[B.n];
      b->units[sub][l][2] = B.wflux_off[B.n];
      b->units[sub][l][3] = B.wrho_off[B.n];
    }
  }
  HIP_TRY(hipMemcpyAsync(b->ws, host, b->tl.total, hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipEventRecord(b->copied[h], b->stream));
  b->copy_pending[h] = true;
  b->tables_dirty = false;
  return BGK_OK;
}

// One replay: the launches of every sub-step whose lists are not empty.
bgk_status replay(bgk_batch* b) {
  hipError_t e = hipSuccess;
  for (int sub = 0; sub < kSub && e == hipSuccess; ++sub) {
    if (b->units[sub][kAllList][1] == 0) break;  // no member takes this sub-step
    for (int stage = 0; stage < 3 && e == hipSuccess; ++stage) {
      for (int t = 0; t < kTeamLists && e == hipSuccess; ++t)
        e = launch_newton_batch(kTeamOfList[t], b->d_nargs(), b->d_list(sub, kMaxFamilies + t),
                                (unsigned)b->units[sub][kMaxFamilies + t][1], b->stream);
      for (size_t f = 0; f < b->fams.size() && e == hipSuccess; ++f)
        e = launch_wall_flux_batch(b->fams[f].precision, b->fams[f].dim, b->fams[f].order, stage,
                                   b->d_wargs(), b->d_list(sub, (int)f),
                                   (unsigned)b->units[sub][f][2], b->stream);
      if (e == hipSuccess)
        e = launch_wall_rho_batch(stage, b->d_wargs(), b->d_list(sub, kAllList),
                                  (unsigned)b->units[sub][kAllList][3], b->stream);
      for (size_t f = 0; f < b->fams.size() && e == hipSuccess; ++f)
        e = launch_stage_batch(b->fams[f].precision, b->fams[f].dim, b->fams[f].order, stage,
                               b->d_args(), b->d_list(sub, (int)f), b->fams[f].tab_bytes,
                               (unsigned)b->units[sub][f][0], b->stream);
      for (size_t i = 0; i < b->members.size() && e == hipSuccess; ++i) {
        const bgk_batch::Member& m = b->members[i];
        if (m.solo && m.per_replay > sub)
          e = launch_stage(m.s->precision, 0, m.sargs[stage], b->stream);
      }
    }
  }
  if (e != hipSuccess) return fail(BGK_ERR_DEVICE, "batch launch: %s", hipGetErrorString(e));
  return BGK_OK;
}

void destroy_batch_host(bgk_batch* b) {
  for (int h = 0; h < 2; ++h) {
    if (b->host[h]) (void)hipHostFree(b->host[h]);
    if (b->copied[h]) (void)hipEventDestroy(b->copied[h]);
  }
  for (hipEvent_t e : b->ev)
    if (e) (void)hipEventDestroy(e);
  if (b->diag) (void)hipHostFree(b->diag);
}

// Hand back finished members in completion order: all of them once their
// replay has executed (block), or those whose replay already has (no wait).
bgk_status batch_collect(bgk_batch* b, bgk_solver** done, int32_t* status, int32_t cap,
                         int32_t* ndone, bool block) {
  *ndone = 0;
  int32_t n = 0;
  size_t i = 0;
  for (; i < b->finished.size() && n < cap; ++i) {
    const bgk_batch::Finished& f = b->finished[i];
    hipEvent_t e = b->ev[f.replay % bgk_batch::kEvents];
    // a later record of the same event marks a later replay on the same
    // stream, whose completion implies this one's
    if (block) {
      HIP_TRY(hipEventSynchronize(e));
    } else {
      const hipError_t q = hipEventQuery(e);
      if (q == hipErrorNotReady) break;
      if (q != hipSuccess) return fail(BGK_ERR_DEVICE, "event query: %s", hipGetErrorString(q));
    }
    bgk_solver* s = f.s;
    s->in_batch = false;
    const unsigned long long nfail = b->diag[f.slot * 2 + 1];
    int32_t st = BGK_OK;
    if (nfail > 0) {
      s->failed = true;
      st = BGK_ERR_NEWTON;
    }
    b->free_slots.push_back(f.slot);
    done[n] = s;
    status[n] = st;
    ++n;
  }
  b->finished.erase(b->finished.begin(), b->finished.begin() + i);
  *ndone = n;
  return BGK_OK;
}

}  // namespace

extern "C" {

bgk_status bgk_batch_query_footprint(int32_t max_members, size_t* bytes) {
  if (!bytes) return fail(BGK_ERR_INVALID_ARG, "bytes is NULL");
  if (max_members < 1 || max_members > kMaxBatchMembers)
    return fail(BGK_ERR_INVALID_ARG, "max_members must be in 1..%d", kMaxBatchMembers);
  *bytes = table_layout().total;
  return BGK_OK;
}

bgk_status bgk_batch_create(void* hip_stream, int32_t max_members, void* d_workspace, size_t bytes,
                            bgk_batch** out) {
  if (!out) return fail(BGK_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  size_t need = 0;
  bgk_status st = bgk_batch_query_footprint(max_members, &need);
  if (st) return st;
  if (!d_workspace) return fail(BGK_ERR_INVALID_ARG, "workspace is NULL");
  if (((uintptr_t)d_workspace) % kAlign)
    return fail(BGK_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  if (bytes < need)
    return fail(BGK_ERR_OUT_OF_MEMORY, "batch workspace %zu bytes < footprint %zu", bytes, need);
  bgk_batch* b = new (std::nothrow) bgk_batch();
  if (!b) return fail(BGK_ERR_OUT_OF_MEMORY, "host allocation failed");
  b->stream = (hipStream_t)hip_stream;
  b->max_members = max_members;
  b->ws = (char*)d_workspace;
  b->tl = table_layout();
  memset(b->units, 0, sizeof(b->units));
  for (int i = max_members - 1; i >= 0; --i) b->free_slots.push_back(i);
  for (int h = 0; h < 2; ++h) {
    hipError_t e = hipHostMalloc((void**)&b->host[h], b->tl.total, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->copied[h], hipEventDisableTiming);
    if (e != hipSuccess) {
      destroy_batch_host(b);
      delete b;
      return fail(BGK_ERR_DEVICE, "batch staging: %s", hipGetErrorString(e));
    }
    memset(b->host[h], 0, b->tl.total);
  }
  hipError_t e = hipHostMalloc((void**)&b->diag, (size_t)max_members * 2 * sizeof(unsigned long long),
                               hipHostMallocDefault);
  for (int i = 0; i < bgk_batch::kEvents && e == hipSuccess; ++i)
    e = hipEventCreateWithFlags(&b->ev[i], hipEventDisableTiming);
  if (e != hipSuccess) {
    destroy_batch_host(b);
    delete b;
    return fail(BGK_ERR_DEVICE, "batch events: %s", hipGetErrorString(e));
  }
  *out = b;
  return BGK_OK;
}

bgk_status bgk_batch_add(bgk_batch* b, bgk_solver* s, double dt, int64_t nsteps) {
  if (!b || !s) return fail(BGK_ERR_INVALID_ARG, "NULL argument");
  if (!(dt > 0.0) || !isfinite(dt)) return fail(BGK_ERR_INVALID_ARG, "dt must be > 0");
  if (nsteps < 1) return fail(BGK_ERR_INVALID_ARG, "nsteps < 1");
  if (b->free_slots.empty())
    return fail(BGK_ERR_OUT_OF_MEMORY, "batch is full (%d members)", b->max_members);
  if (s->stream != b->stream) return fail(BGK_ERR_INVALID_ARG, "solver and batch streams differ");
  if (s->in_batch) return fail(BGK_ERR_STATE, "solver already in a batch");
  if (!s->has_state) return fail(BGK_ERR_STATE, "no state installed");
  if (s->failed) return fail(BGK_ERR_STATE, "solver failed earlier; install a new state");
  if (s->timing) return fail(BGK_ERR_STATE, "disable timing before adding to a batch");
  if (s->precision == BGK_BF16)
    return fail(BGK_ERR_UNSUPPORTED, "BF16 storage alternates its state buffer between steps; "
                "step it with bgk_rk3_step");
  if (s->pb.dim > 2)
    return fail(BGK_ERR_UNSUPPORTED, "batches hold 1-D and 2-D problems; step hexahedral "
                "problems with bgk_rk3_step");
  {
    // the work-unit prefix sums of a launch are 32-bit
    int64_t units = member_units(s), nb = member_newton_blocks(s);
    for (auto& m : b->members) {
      units += member_units(m.s);
      nb += member_newton_blocks(m.s);
    }
    if (units > INT32_MAX || nb > INT32_MAX)
      return fail(BGK_ERR_UNSUPPORTED, "batch work would exceed 2^31 work-groups per launch; "
                  "step this solver with bgk_rk3_step");
  }
  bgk_status st = ensure_partials(s);
  if (st) return st;
  // family of the member's stage kernels
  int fam = -1;
  for (size_t f = 0; f < b->fams.size(); ++f)
    if (b->fams[f].dim == s->pb.dim && b->fams[f].order == s->pb.order &&
        b->fams[f].precision == s->precision)
      fam = (int)f;
  const size_t tab = s->pb.mu_ref > 0.0 ? (size_t)s->L.ns * s->g.tabw * sizeof(double) : 0;
  if (fam < 0) {
    if ((int)b->fams.size() >= kMaxFamilies) return fail(BGK_ERR_UNSUPPORTED, "too many families");
    b->fams.push_back({s->pb.dim, s->pb.order, s->precision, tab});
    fam = (int)b->fams.size() - 1;
  }
  b->fams[fam].tab_bytes = std::max(b->fams[fam].tab_bytes, tab);
  const int slot = b->free_slots.back();
  b->free_slots.pop_back();
  s->in_batch = true;
  b->members.push_back({s, dt, nsteps, 1, slot, fam});
  b->tables_dirty = true;
  return BGK_OK;
}

bgk_status bgk_batch_step(bgk_batch* b, int32_t nsteps) {
  if (!b) return fail(BGK_ERR_INVALID_ARG, "NULL batch");
  if (nsteps < 0) return fail(BGK_ERR_INVALID_ARG, "nsteps < 0");
  for (int32_t k = 0; k < nsteps && !b->members.empty(); ++k) {
    // keep at most kAhead replays queued beyond the last completed one
    if (b->replays >= bgk_batch::kAhead)
      HIP_TRY(hipEventSynchronize(b->ev[(b->replays - bgk_batch::kAhead) % bgk_batch::kEvents]));
    if (b->tables_dirty) {
      bgk_status st = upload_tables(b);
      if (st) return st;
    }
    bgk_status st = replay(b);
    if (st) return st;
    size_t w = 0;
    for (size_t i = 0; i < b->members.size(); ++i) {
      bgk_batch::Member& m = b->members[i];
      m.remaining -= m.per_replay;
      if (m.remaining == 0) {
        // its failure counters as of this replay, read at the poll
        HIP_TRY(hipMemcpyAsync(b->diag + m.slot * 2, m.s->diag(), 2 * sizeof(unsigned long long),
                               hipMemcpyDeviceToHost, b->stream));
        b->finished.push_back({m.s, b->replays, m.slot});
        b->tables_dirty = true;
      } else {
        if (m.per_replay > m.remaining) b->tables_dirty = true;  // re-balance near the end
        b->members[w++] = m;
      }
    }
    b->members.resize(w);
    HIP_TRY(hipEventRecord(b->ev[b->replays % bgk_batch::kEvents], b->stream));
    ++b->replays;
  }
  return BGK_OK;
}

bgk_status bgk_batch_poll(bgk_batch* b, bgk_solver** done, int32_t* status, int32_t cap,
                          int32_t* ndone) {
  if (!b || !ndone || (cap > 0 && (!done || !status)))
    return fail(BGK_ERR_INVALID_ARG, "NULL argument");
  return batch_collect(b, done, status, cap, ndone, true);
}

bgk_status bgk_batch_poll_ready(bgk_batch* b, bgk_solver** done, int32_t* status, int32_t cap,
                                int32_t* ndone) {
  if (!b || !ndone || (cap > 0 && (!done || !status)))
    return fail(BGK_ERR_INVALID_ARG, "NULL argument");
  return batch_collect(b, done, status, cap, ndone, false);
}

bgk_status bgk_batch_remove(bgk_batch* b, bgk_solver* s) {
  if (!b || !s) return fail(BGK_ERR_INVALID_ARG, "NULL argument");
  for (size_t i = 0; i < b->members.size(); ++i) {
    if (b->members[i].s == s) {
      HIP_TRY(hipStreamSynchronize(b->stream));
      s->in_batch = false;
      b->free_slots.push_back(b->members[i].slot);
      b->members.erase(b->members.begin() + i);
      b->tables_dirty = true;
      return BGK_OK;
    }
  }
  return fail(BGK_ERR_INVALID_ARG, "solver is not an active member");
}

int32_t bgk_batch_size(const bgk_batch* b) { return b ? (int32_t)b->members.size() : 0; }

bgk_status bgk_batch_destroy(bgk_batch* b) {
  if (!b) return BGK_OK;
  (void)hipStreamSynchronize(b->stream);
  for (auto& m : b->members) m.s->in_batch = false;
  for (auto& f : b->finished) f.s->in_batch = false;
  destroy_batch_host(b);
  delete b;
  return BGK_OK;
}

}  // extern "C"
