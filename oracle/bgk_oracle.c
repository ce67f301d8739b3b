/*
 * bgk_oracle.c -- plain, slow FP64 CPU reference for the discrete-velocity
 * Boltzmann-BGK phase-space residual and its SSP-RK3 step.
 *
 * TEST INFRASTRUCTURE. This is the oracle the HIP path is checked against.
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
 * load it. It shares no code, header, table or helper with the HIP path.
 *
 * Method (Dzanic & Martinelli, arXiv 2308.06196):
 *   Sec. 2     Boltzmann equation with BGK relaxation C = (g - f)/tau; moments
 *              Q = [rho, rho U, E] = int f psi du with psi = [1, u, u.u/2];
 *              Maxwellian g(rho, U, theta); P = (gamma-1)(E - rho U.U/2),
 *              theta = P/rho; tau = mu/P.
 *   Sec. 2.1   nodal phase-space unknowns f_ij = f(x_i, u_j);
 *              flux reconstruction with correction functions that recover
 *              nodal DG and an upwind common interface flux; Zhang-Shu
 *              positivity limiter; uniform Cartesian velocity grid with the
 *              trapezoidal integration operator M; discretely conservative
 *              equilibrium (the DVM equilibrium exp(alpha . psi) whose
 *              discrete moments equal those of f), found by Newton's method
 *              with its closed-form Jacobian.
 *   Sec. 2.2   explicit time stepping (three-stage SSP Runge-Kutta here).
 *   The non-conservative model the paper contrasts with the DVM equilibrium
 *   (Sec. 2.1) relaxes to the continuous Maxwellian of (rho, U, theta)
 *   sampled at the velocity nodes (problem field equilibrium = 1).
 *
 * Readings where the paper is silent (all shared with the HIP path through
 * the documented problem statement, never through code):
 *   - the Maxwellian normalisation uses the velocity dimension m = 3;
 *   - gamma defaults to (m+2)/m = 5/3 (monatomic gas);
 *   - mu = mu_ref (theta/theta_ref)^omega, or Sutherland's law
 *     mu_ref (theta/theta_ref)^{3/2} (theta_ref + S)/(theta + S) when a
 *     constant S > 0 is given; mu_ref <= 0 switches collisions off;
 *   - Newton starts from the continuous Maxwellian of Q, stops once the
 *     scaled moment residual is <= tol, then takes one final polishing step;
 *     a step that would make alpha_4 >= 0 is halved until alpha_4 < 0;
 *   - specular walls mirror the wall-normal velocity component;
 *   - diffuse (Maxwell, fully accommodating) walls re-emit, into the
 *     velocities pointing away from the wall, the wall Maxwellian sampled at
 *     the nodes, scaled at every flux point so that the discrete mass flux
 *     through the wall vanishes (the paper defers wall conditions to another
 *     work);
 *   - the limiter acts after every Runge-Kutta stage on the solution nodes,
 *     with the Gauss-weighted element mean.
 *
 * Every sum over the velocity grid is taken directly over all N_v nodes
 * (no separable shortcut), with compensated (Neumaier) summation for moments.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXN 8

typedef struct {
  int32_t dim, order;
  int32_t nelem[3];
  double xlo[3], xhi[3];
  int32_t bc[3][2]; /* 0 periodic, 1 specular wall, 2 diffuse wall */
  int32_t nvel[3];
  double vlo[3], vhi[3];
  double mu_ref, theta_ref, omega, gamma;
  int32_t limiter, newton_maxit;
  double newton_tol;
  int32_t equilibrium;      /* 0 discretely conservative, 1 continuous Maxwellian */
  double wall_theta[3][2];  /* diffuse wall temperature */
  double wall_vel[3][2][3]; /* diffuse wall velocity */
  double sutherland;        /* > 0: Sutherland constant S (else power law) */
} orc_problem;

typedef struct {
  int64_t newton_it_max;   /* largest number of Newton residual evaluations */
  int64_t newton_fail;     /* nodes whose Newton solve failed */
  int64_t limiter_hits;    /* (element, velocity) slices that were contracted */
  int64_t limiter_bad;     /* slices whose mean was <= 0 */
} orc_diag;

/* ------------------------------------------------------------------------ */
/* One-dimensional polynomial tools                                          */
/* ------------------------------------------------------------------------ */

/* Legendre P_0..P_n and derivatives at x via Bonnet's recursion and
 * P'_{k+1} = P'_{k-1} + (2k+1) P_k. */
static void legendre_all(int n, double x, double* P, double* dP) {
  P[0] = 1.0;
  dP[0] = 0.0;
  if (n >= 1) {
    P[1] = x;
    dP[1] = 1.0;
  }
  for (int k = 1; k < n; ++k) {
    P[k + 1] = ((2.0 * k + 1.0) * x * P[k] - k * P[k - 1]) / (k + 1.0);
    dP[k + 1] = dP[k - 1] + (2.0 * k + 1.0) * P[k];
  }
}

/* Gauss-Legendre nodes (ascending) and weights: roots of P_n by Newton's
 * method, weights 2 / ((1 - x^2) P_n'(x)^2). */
int orc_gauss_legendre(int n, double* x, double* w) {
  if (n < 1 || n > ORC_MAXN) return 1;
  double P[ORC_MAXN + 2], dP[ORC_MAXN + 2];
  for (int i = 0; i < n; ++i) {
    double r = cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      legendre_all(n, r, P, dP);
      double dr = P[n] / dP[n];
      r -= dr;
      if (fabs(dr) < 1e-16) break;
    }
    legendre_all(n, r, P, dP);
    /* the initial guesses run from +1 to -1: store in ascending order */
    x[n - 1 - i] = r;
    w[n - 1 - i] = 2.0 / ((1.0 - r * r) * dP[n] * dP[n]);
  }
  return 0;
}

/* Lagrange basis on nodes xi[0..n): D[a*n+b] = l_b'(xi_a), lamL[b] = l_b(-1),
 * lamR[b] = l_b(+1). Products written out from the definition
 * l_b(x) = prod_{m != b} (x - xi_m) / (xi_b - xi_m). */
static double lagrange_value(int n, const double* xi, int b, double x) {
  double v = 1.0;
  for (int m = 0; m < n; ++m)
    if (m != b) v *= (x - xi[m]) / (xi[b] - xi[m]);
  return v;
}

static double lagrange_deriv(int n, const double* xi, int b, double x) {
  double s = 0.0;
  for (int k = 0; k < n; ++k) {
    if (k == b) continue;
    double t = 1.0 / (xi[b] - xi[k]);
    for (int m = 0; m < n; ++m)
      if (m != b && m != k) t *= (x - xi[m]) / (xi[b] - xi[m]);
    s += t;
  }
  return s;
}

void orc_lagrange(int n, const double* xi, double* D, double* lamL, double* lamR) {
  for (int b = 0; b < n; ++b) {
    lamL[b] = lagrange_value(n, xi, b, -1.0);
    lamR[b] = lagrange_value(n, xi, b, 1.0);
    for (int a = 0; a < n; ++a) D[a * n + b] = lagrange_deriv(n, xi, b, xi[a]);
  }
}

/* Derivatives at xi_a of Huynh's correction functions that recover nodal DG:
 * the right Radau polynomial g_L = ((-1)^(p+1)/2)(P_{p+1} - P_p) (one at
 * xi = -1, zero at +1) and the left Radau polynomial g_R = (P_{p+1} + P_p)/2. */
void orc_dg_correction(int p, const double* xi, double* GL, double* GR) {
  double P[ORC_MAXN + 2], dP[ORC_MAXN + 2];
  double sgn = ((p + 1) % 2 == 0) ? 1.0 : -1.0;
  for (int a = 0; a <= p; ++a) {
    legendre_all(p + 1, xi[a], P, dP);
    GL[a] = 0.5 * sgn * (dP[p + 1] - dP[p]);
    GR[a] = 0.5 * (dP[p + 1] + dP[p]);
  }
}

/* ------------------------------------------------------------------------ */
/* Problem geometry                                                          */
/* ------------------------------------------------------------------------ */

typedef struct {
  int d, p, n1, ns;
  int64_t ne, nx, nv;
  int nv1[3];
  double h[3];
  double xi[ORC_MAXN], wq[ORC_MAXN];
  double D[ORC_MAXN * ORC_MAXN], lamL[ORC_MAXN], lamR[ORC_MAXN];
  double GL[ORC_MAXN], GR[ORC_MAXN];
  double W[512];    /* tensor-product Gauss weights per element node */
  double* u;        /* [nv][3] */
  double* w;        /* [nv] trapezoid weights */
  double gamma;
} orc_ops;

static int ops_init(const orc_problem* pr, orc_ops* op) {
  memset(op, 0, sizeof(*op));
  op->d = pr->dim;
  op->p = pr->order;
  if (op->d < 1 || op->d > 3 || op->p < 0 || op->p + 1 > ORC_MAXN) return 1;
  op->n1 = op->p + 1;
  op->ns = 1;
  for (int k = 0; k < op->d; ++k) op->ns *= op->n1;
  if (op->ns > 512) return 1;
  op->ne = 1;
  for (int k = 0; k < op->d; ++k) {
    if (pr->nelem[k] < 1) return 1;
    op->ne *= pr->nelem[k];
    op->h[k] = (pr->xhi[k] - pr->xlo[k]) / pr->nelem[k];
  }
  op->nx = op->ne * op->ns;
  op->nv = 1;
  for (int c = 0; c < 3; ++c) {
    if (pr->nvel[c] < 2) return 1;
    op->nv1[c] = pr->nvel[c];
    op->nv *= pr->nvel[c];
  }
  orc_gauss_legendre(op->n1, op->xi, op->wq);
  orc_lagrange(op->n1, op->xi, op->D, op->lamL, op->lamR);
  orc_dg_correction(op->p, op->xi, op->GL, op->GR);
  for (int i = 0; i < op->ns; ++i) {
    double Wi = 1.0;
    int r = i;
    for (int k = 0; k < op->d; ++k) {
      Wi *= op->wq[r % op->n1];
      r /= op->n1;
    }
    op->W[i] = Wi;
  }
  op->u = (double*)malloc(sizeof(double) * 3 * op->nv);
  op->w = (double*)malloc(sizeof(double) * op->nv);
  if (!op->u || !op->w) return 1;
  /* uniform grid with end points, trapezoid weights (half weight at ends) */
  double du[3];
  for (int c = 0; c < 3; ++c) du[c] = (pr->vhi[c] - pr->vlo[c]) / (pr->nvel[c] - 1);
  for (int64_t j = 0; j < op->nv; ++j) {
    int b[3];
    b[0] = (int)(j % op->nv1[0]);
    b[1] = (int)((j / op->nv1[0]) % op->nv1[1]);
    b[2] = (int)(j / ((int64_t)op->nv1[0] * op->nv1[1]));
    double wj = 1.0;
    for (int c = 0; c < 3; ++c) {
      op->u[3 * j + c] = pr->vlo[c] + b[c] * du[c];
      double wc = du[c];
      if (b[c] == 0 || b[c] == op->nv1[c] - 1) wc *= 0.5;
      wj *= wc;
    }
    op->w[j] = wj;
  }
  op->gamma = pr->gamma > 0.0 ? pr->gamma : 5.0 / 3.0;
  return 0;
}

static void ops_free(orc_ops* op) {
  free(op->u);
  free(op->w);
  op->u = op->w = NULL;
}

void orc_velocity_grid(const orc_problem* pr, double* u, double* w) {
  orc_ops op;
  if (ops_init(pr, &op)) return;
  memcpy(u, op.u, sizeof(double) * 3 * op.nv);
  memcpy(w, op.w, sizeof(double) * op.nv);
  ops_free(&op);
}

/* x[(e*ns + i)*dim + k]: solution-node coordinates, element e lexicographic
 * (axis 0 fastest), node i lexicographic (axis 0 fastest). */
void orc_node_coords(const orc_problem* pr, double* x) {
  orc_ops op;
  if (ops_init(pr, &op)) return;
  for (int64_t e = 0; e < op.ne; ++e) {
    int64_t er = e;
    int ek[3] = {0, 0, 0};
    for (int k = 0; k < op.d; ++k) {
      ek[k] = (int)(er % pr->nelem[k]);
      er /= pr->nelem[k];
    }
    for (int i = 0; i < op.ns; ++i) {
      int r = i;
      for (int k = 0; k < op.d; ++k) {
        int a = r % op.n1;
        r /= op.n1;
        x[(e * op.ns + i) * op.d + k] =
            pr->xlo[k] + op.h[k] * (ek[k] + 0.5 * (1.0 + op.xi[a]));
      }
    }
  }
  ops_free(&op);
}

/* ------------------------------------------------------------------------ */
/* Velocity-space operations (Sec. 2 and Sec. 2.1, velocity discretization)  */
/* ------------------------------------------------------------------------ */

static void neumaier_add(double* s, double* c, double v) {
  double t = *s + v;
  if (fabs(*s) >= fabs(v))
    *c += (*s - t) + v;
  else
    *c += (v - t) + *s;
  *s = t;
}

static void psi_of(const double* u, double* psi) {
  psi[0] = 1.0;
  psi[1] = u[0];
  psi[2] = u[1];
  psi[3] = u[2];
  psi[4] = 0.5 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
}

/* Q = M . [f (x) psi] over one node's velocity slice (trapezoid weights). */
static void node_moments(const orc_ops* op, const double* fj, double* Q) {
  double s[5] = {0, 0, 0, 0, 0}, c[5] = {0, 0, 0, 0, 0};
  for (int64_t j = 0; j < op->nv; ++j) {
    double psi[5];
    psi_of(op->u + 3 * j, psi);
    double wf = op->w[j] * fj[j];
    for (int m = 0; m < 5; ++m) neumaier_add(&s[m], &c[m], wf * psi[m]);
  }
  for (int m = 0; m < 5; ++m) Q[m] = s[m] + c[m];
}

void orc_moments(const orc_problem* pr, const double* f, double* Q) {
  orc_ops op;
  if (ops_init(pr, &op)) return;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < op.nx; ++i) node_moments(&op, f + i * op.nv, Q + 5 * i);
  ops_free(&op);
}

/* Sample the continuous Maxwellian rho/(2 pi theta)^{3/2} exp(-|u-U|^2/(2 theta))
 * at every phase-space node; prim[i] = (rho, Ux, Uy, Uz, theta). */
void orc_maxwellian(const orc_problem* pr, const double* prim, double* f) {
  orc_ops op;
  if (ops_init(pr, &op)) return;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < op.nx; ++i) {
    const double* q = prim + 5 * i;
    double rho = q[0], th = q[4];
    double nrm = rho / pow(2.0 * M_PI * th, 1.5);
    for (int64_t j = 0; j < op.nv; ++j) {
      const double* u = op.u + 3 * j;
      double dx = u[0] - q[1], dy = u[1] - q[2], dz = u[2] - q[3];
      f[i * op.nv + j] = nrm * exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * th));
    }
  }
  ops_free(&op);
}

/* Solve J x = b for a symmetric positive definite 5x5 J by Cholesky.
 * Returns nonzero when J is not numerically positive definite. */
static int chol5_solve(const double J[5][5], const double* b, double* x) {
  double L[5][5];
  memset(L, 0, sizeof(L));
  for (int i = 0; i < 5; ++i) {
    for (int k = 0; k <= i; ++k) {
      double s = J[i][k];
      for (int m = 0; m < k; ++m) s -= L[i][m] * L[k][m];
      if (i == k) {
        if (!(s > 0.0)) return 1;
        L[i][i] = sqrt(s);
      } else {
        L[i][k] = s / L[k][k];
      }
    }
  }
  double y[5];
  for (int i = 0; i < 5; ++i) {
    double s = b[i];
    for (int m = 0; m < i; ++m) s -= L[i][m] * y[m];
    y[i] = s / L[i][i];
  }
  for (int i = 4; i >= 0; --i) {
    double s = y[i];
    for (int m = i + 1; m < 5; ++m) s -= L[m][i] * x[m];
    x[i] = s / L[i][i];
  }
  return 0;
}

/* Continuous Maxwellian at the (rho, U, theta) of the moments Q, written as
 * exp(alpha . psi): alpha = (ln(rho/(2 pi theta)^{3/2}) - |U|^2/(2 theta),
 * U/theta, -1/theta) (Sec. 2, Maxwellian; reading R1 for the exponent).
 * Returns 2 when Q is not realizable. This is the equilibrium of the
 * non-conservative model and the start of the Newton iteration below. */
static int continuous_alpha(double gm, const double* Q, double* alpha) {
  double rho = Q[0];
  if (!(rho > 0.0)) return 2;
  double U[3] = {Q[1] / rho, Q[2] / rho, Q[3] / rho};
  double UU = U[0] * U[0] + U[1] * U[1] + U[2] * U[2];
  double P = (gm - 1.0) * (Q[4] - 0.5 * rho * UU);
  double th = P / rho;
  if (!(th > 0.0)) return 2;
  alpha[0] = log(rho / pow(2.0 * M_PI * th, 1.5)) - UU / (2.0 * th);
  alpha[1] = U[0] / th;
  alpha[2] = U[1] / th;
  alpha[3] = U[2] / th;
  alpha[4] = -1.0 / th;
  return 0;
}

/* Discretely conservative equilibrium for one node: find alpha with
 * sum_j w_j psi_j exp(alpha . psi_j) = Q by Newton's method with the
 * closed-form Jacobian J = sum_j w_j psi_j psi_j^T exp(alpha . psi_j).
 * Returns 0 on success, 1 when not converged within maxit, 2 when Q is not
 * realizable (rho <= 0 or theta <= 0) or J loses definiteness.
 * iters = number of residual evaluations; resid = last scaled residual. */
static int newton_node(const orc_ops* op, const double* Q, int maxit, double tol, double* alpha,
                       int* iters, double* resid) {
  *iters = 0;
  *resid = INFINITY;
  if (continuous_alpha(op->gamma, Q, alpha)) return 2;
  const double rho = Q[0], th = -1.0 / alpha[4];
  double sc[5] = {rho, rho * sqrt(th), rho * sqrt(th), rho * sqrt(th), Q[4]};
  for (int it = 0;; ++it) {
    double s[5] = {0, 0, 0, 0, 0}, c[5] = {0, 0, 0, 0, 0};
    double J[5][5];
    memset(J, 0, sizeof(J));
    for (int64_t j = 0; j < op->nv; ++j) {
      double psi[5];
      psi_of(op->u + 3 * j, psi);
      double ap = alpha[0] * psi[0] + alpha[1] * psi[1] + alpha[2] * psi[2] +
                  alpha[3] * psi[3] + alpha[4] * psi[4];
      double wg = op->w[j] * exp(ap);
      for (int a = 0; a < 5; ++a) {
        neumaier_add(&s[a], &c[a], wg * psi[a]);
        for (int b = 0; b < 5; ++b) J[a][b] += wg * psi[a] * psi[b];
      }
    }
    double F[5], r = 0.0;
    for (int a = 0; a < 5; ++a) {
      F[a] = (s[a] + c[a]) - Q[a];
      double ra = fabs(F[a]) / sc[a];
      if (!(ra <= r)) r = ra; /* propagates NaN */
    }
    *iters = it + 1;
    *resid = r;
    int conv = (r <= tol);
    if (!conv && it >= maxit) return 1;
    double dlt[5];
    if (chol5_solve((const double(*)[5])J, F, dlt)) return 2;
    double an[5];
    for (int a = 0; a < 5; ++a) an[a] = alpha[a] - dlt[a];
    for (int h = 0; h < 60 && !(an[4] < 0.0); ++h) {
      for (int a = 0; a < 5; ++a) dlt[a] *= 0.5;
      for (int a = 0; a < 5; ++a) an[a] = alpha[a] - dlt[a];
    }
    if (!(an[4] < 0.0)) return 2;
    for (int a = 0; a < 5; ++a) alpha[a] = an[a];
    if (conv) return 0; /* the step just taken was the polishing step */
  }
}

int orc_newton_node(const orc_problem* pr, const double* Q, double* alpha, int* iters,
                    double* resid) {
  orc_ops op;
  if (ops_init(pr, &op)) return 3;
  int st = newton_node(&op, Q, pr->newton_maxit, pr->newton_tol, alpha, iters, resid);
  ops_free(&op);
  return st;
}

/* Primitive recovery and relaxation time for one node (readings in header). */
static void node_tau(const orc_problem* pr, const orc_ops* op, const double* Q, double* tau) {
  double rho = Q[0];
  double UU = (Q[1] * Q[1] + Q[2] * Q[2] + Q[3] * Q[3]) / (rho * rho);
  double P = (op->gamma - 1.0) * (Q[4] - 0.5 * rho * UU);
  double th = P / rho;
  double mu;
  if (pr->sutherland > 0.0) { /* Sutherland's law */
    double S = pr->sutherland;
    mu = pr->mu_ref * pow(th / pr->theta_ref, 1.5) * (pr->theta_ref + S) / (th + S);
  } else { /* power law */
    mu = pr->mu_ref * pow(th / pr->theta_ref, pr->omega);
  }
  *tau = mu / P;
}

/* BGK collision term C_j = (g_j - f_j)/tau at one node, g = exp(alpha . psi). */
static void node_collision(const orc_problem* pr, const orc_ops* op, const double* fj, double* Cj,
                           orc_diag* dg) {
  if (!(pr->mu_ref > 0.0)) {
    for (int64_t j = 0; j < op->nv; ++j) Cj[j] = 0.0;
    return;
  }
  double Q[5], alpha[5], tau, res;
  int its;
  node_moments(op, fj, Q);
  int st;
  if (pr->equilibrium == 1) { /* non-conservative model: no Newton solve */
    its = 0;
    st = continuous_alpha(op->gamma, Q, alpha);
  } else {
    st = newton_node(op, Q, pr->newton_maxit, pr->newton_tol, alpha, &its, &res);
  }
  if (its > dg->newton_it_max) dg->newton_it_max = its;
  if (st) dg->newton_fail += 1;
  node_tau(pr, op, Q, &tau);
  for (int64_t j = 0; j < op->nv; ++j) {
    double psi[5];
    psi_of(op->u + 3 * j, psi);
    double ap = alpha[0] * psi[0] + alpha[1] * psi[1] + alpha[2] * psi[2] + alpha[3] * psi[3] +
                alpha[4] * psi[4];
    Cj[j] = (exp(ap) - fj[j]) / tau;
  }
}

/* ------------------------------------------------------------------------ */
/* Transport: FR with DG-recovering corrections and upwind common fluxes     */
/* ------------------------------------------------------------------------ */

/* Index of the velocity with component k mirrored (b_k -> N_k - 1 - b_k). */
static int64_t mirror_vel(const orc_ops* op, int64_t j, int k) {
  int b[3];
  b[0] = (int)(j % op->nv1[0]);
  b[1] = (int)((j / op->nv1[0]) % op->nv1[1]);
  b[2] = (int)(j / ((int64_t)op->nv1[0] * op->nv1[1]));
  b[k] = op->nv1[k] - 1 - b[k];
  return b[0] + (int64_t)op->nv1[0] * (b[1] + (int64_t)op->nv1[1] * b[2]);
}

/* Neighbour element along axis k on side s (-1 left, +1 right); -1 = wall. */
static int64_t neighbour(const orc_problem* pr, const orc_ops* op, int64_t e, int k, int s) {
  int ek[3] = {0, 0, 0};
  int64_t er = e;
  for (int m = 0; m < op->d; ++m) {
    ek[m] = (int)(er % pr->nelem[m]);
    er /= pr->nelem[m];
  }
  int nk = ek[k] + s;
  if (nk < 0 || nk >= pr->nelem[k]) {
    if (pr->bc[k][s < 0 ? 0 : 1] != 0) return -1;
    nk = (nk + pr->nelem[k]) % pr->nelem[k];
  }
  ek[k] = nk;
  int64_t out = 0, stride = 1;
  for (int m = 0; m < op->d; ++m) {
    out += ek[m] * stride;
    stride *= pr->nelem[m];
  }
  return out;
}

/* T[i*nv + j] = discrete (u_j . grad f) at node i of element e. */
/* Unit-density Maxwellian of the diffuse wall on side `side` of axis k at
 * velocity u (wall temperature and velocity from the problem). */
static double wall_maxwellian(const orc_problem* pr, int k, int side, const double* u) {
  double th = pr->wall_theta[k][side];
  const double* U = pr->wall_vel[k][side];
  double d2 = 0.0;
  for (int c = 0; c < 3; ++c) d2 += (u[c] - U[c]) * (u[c] - U[c]);
  return exp(-d2 / (2.0 * th)) / pow(2.0 * M_PI * th, 1.5);
}

/* Density of the gas re-emitted by a diffuse wall at one flux point (reading
 * in the header): the discrete mass flux leaving the domain through the wall,
 * sum over outgoing velocities of w |u_k| f_trace, divided by the flux the
 * unit-density wall Maxwellian carries back in, so the net mass flux through
 * the wall is zero. side 0 = left face (outgoing: u_k < 0), 1 = right face. */
static double wall_density(const orc_problem* pr, const orc_ops* op, const double* fe, int k,
                           int side, int base, int stride) {
  const int n1 = op->n1;
  const int64_t nv = op->nv;
  const double* lam = side == 0 ? op->lamL : op->lamR;
  double out = 0.0, in = 0.0;
  for (int64_t j = 0; j < nv; ++j) {
    double a = op->u[3 * j + k];
    int outgoing = side == 0 ? a < 0.0 : a > 0.0;
    if (outgoing) {
      double tr = 0.0;
      for (int b = 0; b < n1; ++b) tr += lam[b] * fe[(base + b * stride) * nv + j];
      out += op->w[j] * fabs(a) * tr;
    } else if (a != 0.0) {
      in += op->w[j] * fabs(a) * wall_maxwellian(pr, k, side, op->u + 3 * j);
    }
  }
  return out / in;
}

static void element_transport(const orc_problem* pr, const orc_ops* op, const double* f, int64_t e,
                              double* T) {
  const int n1 = op->n1, ns = op->ns;
  const int64_t nv = op->nv;
  for (int64_t q = 0; q < (int64_t)ns * nv; ++q) T[q] = 0.0;
  const double* fe = f + e * ns * nv;
  for (int k = 0; k < op->d; ++k) {
    int stride = 1;
    for (int m = 0; m < k; ++m) stride *= n1;
    int64_t eL = neighbour(pr, op, e, k, -1);
    int64_t eR = neighbour(pr, op, e, k, +1);
    const double* fL_el = eL >= 0 ? f + eL * ns * nv : NULL;
    const double* fR_el = eR >= 0 ? f + eR * ns * nv : NULL;
    double sk = 2.0 / op->h[k];
    const int diffL = !fL_el && pr->bc[k][0] == 2, diffR = !fR_el && pr->bc[k][1] == 2;
    for (int base = 0; base < ns; ++base) {
      if ((base / stride) % n1 != 0) continue; /* first node of a line along k */
      double rhoL = diffL ? wall_density(pr, op, fe, k, 0, base, stride) : 0.0;
      double rhoR = diffR ? wall_density(pr, op, fe, k, 1, base, stride) : 0.0;
      for (int64_t j = 0; j < nv; ++j) {
        double a = op->u[3 * j + k];
        double line[ORC_MAXN];
        for (int b = 0; b < n1; ++b) line[b] = fe[(base + b * stride) * nv + j];
        double fLo = 0.0, fRo = 0.0;
        for (int b = 0; b < n1; ++b) {
          fLo += op->lamL[b] * line[b];
          fRo += op->lamR[b] * line[b];
        }
        /* exterior trace at the left face: right trace of the left neighbour,
         * at a specular wall the own left trace at the mirrored velocity, at a
         * diffuse wall the re-emitted wall Maxwellian */
        double extL = 0.0, extR = 0.0;
        if (fL_el) {
          for (int b = 0; b < n1; ++b) extL += op->lamR[b] * fL_el[(base + b * stride) * nv + j];
        } else if (diffL) {
          extL = rhoL * wall_maxwellian(pr, k, 0, op->u + 3 * j);
        } else {
          int64_t jm = mirror_vel(op, j, k);
          for (int b = 0; b < n1; ++b) extL += op->lamL[b] * fe[(base + b * stride) * nv + jm];
        }
        if (fR_el) {
          for (int b = 0; b < n1; ++b) extR += op->lamL[b] * fR_el[(base + b * stride) * nv + j];
        } else if (diffR) {
          extR = rhoR * wall_maxwellian(pr, k, 1, op->u + 3 * j);
        } else {
          int64_t jm = mirror_vel(op, j, k);
          for (int b = 0; b < n1; ++b) extR += op->lamR[b] * fe[(base + b * stride) * nv + jm];
        }
        /* upwind common fluxes in the +x_k direction */
        double HL = a > 0.0 ? a * extL : a * fLo;
        double HR = a > 0.0 ? a * fRo : a * extR;
        for (int ia = 0; ia < n1; ++ia) {
          double df = 0.0;
          for (int b = 0; b < n1; ++b) df += op->D[ia * n1 + b] * line[b];
          T[(int64_t)(base + ia * stride) * nv + j] +=
              sk * (a * df + (HL - a * fLo) * op->GL[ia] + (HR - a * fRo) * op->GR[ia]);
        }
      }
    }
  }
}

/* Residual L = -T + C for element e into out[ns*nv]; scratch C[nv]. */
static void element_residual(const orc_problem* pr, const orc_ops* op, const double* f, int64_t e,
                             double* out, double* C, orc_diag* dg) {
  element_transport(pr, op, f, e, out);
  const int64_t nv = op->nv;
  for (int i = 0; i < op->ns; ++i) {
    const double* fj = f + (e * op->ns + i) * nv;
    node_collision(pr, op, fj, C, dg);
    double* o = out + (int64_t)i * nv;
    for (int64_t j = 0; j < nv; ++j) o[j] = -o[j] + C[j];
  }
}

static void diag_merge(orc_diag* dst, const orc_diag* src) {
  if (src->newton_it_max > dst->newton_it_max) dst->newton_it_max = src->newton_it_max;
  dst->newton_fail += src->newton_fail;
  dst->limiter_hits += src->limiter_hits;
  dst->limiter_bad += src->limiter_bad;
}

static void residual_with_ops(const orc_problem* pr, const orc_ops* op, const double* f, double* L,
                              orc_diag* dg) {
#pragma omp parallel
  {
    orc_diag loc = {0, 0, 0, 0};
    double* C = (double*)malloc(sizeof(double) * op->nv);
#pragma omp for schedule(static)
    for (int64_t e = 0; e < op->ne; ++e)
      element_residual(pr, op, f, e, L + e * op->ns * op->nv, C, &loc);
    free(C);
#pragma omp critical
    diag_merge(dg, &loc);
  }
}

void orc_transport(const orc_problem* pr, const double* f, double* T) {
  orc_ops op;
  if (ops_init(pr, &op)) return;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < op.ne; ++e) element_transport(pr, &op, f, e, T + e * op.ns * op.nv);
  ops_free(&op);
}

void orc_collision(const orc_problem* pr, const double* f, double* C, orc_diag* dg) {
  orc_ops op;
  if (ops_init(pr, &op)) return;
  orc_diag tot = {0, 0, 0, 0};
#pragma omp parallel
  {
    orc_diag loc = {0, 0, 0, 0};
#pragma omp for schedule(static)
    for (int64_t i = 0; i < op.nx; ++i) node_collision(pr, &op, f + i * op.nv, C + i * op.nv, &loc);
#pragma omp critical
    diag_merge(&tot, &loc);
  }
  if (dg) *dg = tot;
  ops_free(&op);
}

void orc_residual(const orc_problem* pr, const double* f, double* L, orc_diag* dg) {
  orc_ops op;
  if (ops_init(pr, &op)) return;
  orc_diag tot = {0, 0, 0, 0};
  residual_with_ops(pr, &op, f, L, &tot);
  if (dg) *dg = tot;
  ops_free(&op);
}

/* Residual of the listed elements only: out[q*ns*nv ...] for elems[q]. The
 * full state f is read (neighbours), only the listed outputs are formed. */
void orc_residual_elems(const orc_problem* pr, const double* f, const int64_t* elems, int64_t nel,
                        double* out, orc_diag* dg) {
  orc_ops op;
  if (ops_init(pr, &op)) return;
  orc_diag tot = {0, 0, 0, 0};
#pragma omp parallel
  {
    orc_diag loc = {0, 0, 0, 0};
    double* C = (double*)malloc(sizeof(double) * op.nv);
#pragma omp for schedule(static)
    for (int64_t q = 0; q < nel; ++q)
      element_residual(pr, &op, f, elems[q], out + q * op.ns * op.nv, C, &loc);
    free(C);
#pragma omp critical
    diag_merge(&tot, &loc);
  }
  if (dg) *dg = tot;
  ops_free(&op);
}

/* ------------------------------------------------------------------------ */
/* Positivity limiter and SSP-RK3                                            */
/* ------------------------------------------------------------------------ */

/* Zhang-Shu: per (element, velocity) slice, if the minimum over the solution
 * nodes is negative, contract towards the Gauss-weighted mean with
 * beta = min(|mean / (mean - min)|, 1). */
static void element_limiter(const orc_ops* op, double* fe, orc_diag* dg) {
  const int ns = op->ns;
  const int64_t nv = op->nv;
  double wsum = 0.0;
  for (int i = 0; i < ns; ++i) wsum += op->W[i];
  for (int64_t j = 0; j < nv; ++j) {
    double mean = 0.0, fmin = INFINITY;
    for (int i = 0; i < ns; ++i) {
      double v = fe[(int64_t)i * nv + j];
      mean += op->W[i] * v;
      if (v < fmin) fmin = v;
    }
    mean /= wsum;
    if (!(fmin < 0.0)) continue;
    dg->limiter_hits += 1;
    if (!(mean > 0.0)) dg->limiter_bad += 1;
    if (mean == fmin) continue;
    double beta = fabs(mean / (mean - fmin));
    if (beta > 1.0) beta = 1.0;
    for (int i = 0; i < ns; ++i) {
      double* v = &fe[(int64_t)i * nv + j];
      *v = mean + beta * (*v - mean);
    }
  }
}

static void limiter_with_ops(const orc_ops* op, double* f, orc_diag* dg) {
#pragma omp parallel
  {
    orc_diag loc = {0, 0, 0, 0};
#pragma omp for schedule(static)
    for (int64_t e = 0; e < op->ne; ++e) element_limiter(op, f + e * op->ns * op->nv, &loc);
#pragma omp critical
    diag_merge(dg, &loc);
  }
}

void orc_limiter(const orc_problem* pr, double* f, orc_diag* dg) {
  orc_ops op;
  if (ops_init(pr, &op)) return;
  orc_diag tot = {0, 0, 0, 0};
  limiter_with_ops(&op, f, &tot);
  if (dg) *dg = tot;
  ops_free(&op);
}

/* nsteps of Shu-Osher SSP-RK3, each stage followed by the limiter when on:
 *   f1 = f + dt L(f)
 *   f2 = 3/4 f + 1/4 (f1 + dt L(f1))
 *   f  = 1/3 f + 2/3 (f2 + dt L(f2))                                        */
int orc_rk3_step(const orc_problem* pr, double* f, double dt, int nsteps, orc_diag* dg) {
  orc_ops op;
  if (ops_init(pr, &op)) return 1;
  int64_t n = op.nx * op.nv;
  double* f1 = (double*)malloc(sizeof(double) * n);
  double* f2 = (double*)malloc(sizeof(double) * n);
  double* L = (double*)malloc(sizeof(double) * n);
  if (!f1 || !f2 || !L) {
    free(f1);
    free(f2);
    free(L);
    ops_free(&op);
    return 1;
  }
  orc_diag tot = {0, 0, 0, 0};
  const double A[3] = {0.0, 0.75, 1.0 / 3.0};
  const double B[3] = {1.0, 0.25, 2.0 / 3.0};
  for (int s = 0; s < nsteps; ++s) {
    const double* in[3] = {f, f1, f2};
    double* out[3] = {f1, f2, f};
    for (int st = 0; st < 3; ++st) {
      residual_with_ops(pr, &op, in[st], L, &tot);
      double a = A[st], b = B[st];
      double* o = out[st];
      const double* x = in[st];
#pragma omp parallel for schedule(static)
      for (int64_t q = 0; q < n; ++q) o[q] = a * f[q] + b * (x[q] + dt * L[q]);
      if (pr->limiter) limiter_with_ops(&op, o, &tot);
    }
  }
  free(f1);
  free(f2);
  free(L);
  ops_free(&op);
  if (dg) *dg = tot;
  return 0;
}

/* Time step: dt = min(cfl / max_j sum_{k<d} |u_jk|/h_k, tau_min(f)). */
double orc_stable_dt(const orc_problem* pr, const double* f, double cfl) {
  orc_ops op;
  if (ops_init(pr, &op)) return -1.0;
  double smax = 0.0;
  for (int64_t j = 0; j < op.nv; ++j) {
    double s = 0.0;
    for (int k = 0; k < op.d; ++k) s += fabs(op.u[3 * j + k]) / op.h[k];
    if (s > smax) smax = s;
  }
  double dt = cfl / smax;
  if (pr->mu_ref > 0.0) {
    double tmin = INFINITY;
    for (int64_t i = 0; i < op.nx; ++i) {
      double Q[5], tau;
      node_moments(&op, f + i * op.nv, Q);
      node_tau(pr, &op, Q, &tau);
      if (tau < tmin) tmin = tau;
    }
    if (tmin < dt) dt = tmin;
  }
  ops_free(&op);
  return dt;
}
