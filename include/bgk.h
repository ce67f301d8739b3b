/*
 * bgk.h -- C-ABI of libbgk, the MI355X (gfx950) hot path of a high-order
 * discrete-velocity Boltzmann-BGK solver.
 *
 * Method: T. Dzanic and L. Martinelli, "Towards full molecular gas dynamics
 * simulations of complex flows via the Boltzmann equation" (arXiv 2308.06196).
 *   Sec. 2        Boltzmann equation with the BGK model: the conserved
 *                 variables Q = [rho, rho U, E] are moments of f against the
 *                 collision invariants psi = [1, u, u.u/2]; C = (g - f)/tau;
 *                 g is a Maxwellian; P = (gamma-1)(E - rho U.U/2),
 *                 theta = P/rho, tau = mu/P.
 *   Sec. 2.1      nodal unknowns f_ij = f(x_i, u_j); flux reconstruction with
 *                 DG-recovering correction functions and an upwind common
 *                 interface flux; Zhang-Shu positivity limiter; uniform
 *                 Cartesian velocity grid with trapezoidal quadrature M;
 *                 discretely conservative equilibrium found by Newton's
 *                 method on a perturbed macroscopic state.
 *   Sec. 2.2      explicit time stepping (three-stage SSP Runge-Kutta here).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every call returns bgk_status (0 = BGK_OK) and never aborts or throws.
 *    On failure a message is available from bgk_last_error() (thread-local).
 *  - Geometry: the domain is the box [xlo, xhi] in d = dim dimensions with
 *    nelem[k] uniform elements per axis. Elements are numbered
 *    lexicographically, axis 0 fastest. Each element holds (order+1)^dim
 *    solution nodes at the tensor-product Gauss-Legendre points, numbered
 *    lexicographically, axis 0 fastest.
 *  - Velocity grid: always three components; component c has nvel[c] >= 2
 *    equispaced nodes u = vlo[c] + b (vhi[c]-vlo[c])/(nvel[c]-1) including
 *    both end points, trapezoidal weights. Velocity j = bx + nvel[0] (by +
 *    nvel[1] bz).
 *  - Canonical state layout ("exchange layout"): FP64 f[elem][node][vel],
 *    velocity fastest; size nx*nv doubles with nx = nelem_total*(order+1)^dim
 *    and nv = nvel[0]*nvel[1]*nvel[2]. The library stores f internally in
 *    the precision chosen by bgk_problem.precision and converts on exchange.
 *  - Memory ownership: the caller allocates one device workspace of at least
 *    the size given by bgk_query_footprint and passes it to bgk_create; the
 *    library never allocates device memory and never frees caller memory.
 *    Host pointers are not retained after a call returns.
 *  - Streams: all device work of a solver is ordered on the HIP stream given
 *    at create (NULL = the default stream). Entry points that hand results
 *    to host memory, or that read device-side error flags, synchronise that
 *    stream; bgk_rk3_step and bgk_residual with device buffers do not.
 *  - Errors: argument errors leave the solver unchanged. Numerical failures
 *    (Newton not converged, non-realizable or non-finite moments) mark the
 *    solver failed; they are reported by the next synchronising call, and
 *    later calls return BGK_ERR_STATE until bgk_set_state or
 *    bgk_set_maxwellian installs a new state.
 *  - Threading: one solver must not be used from two threads at once;
 *    distinct solvers are independent.
 */
#ifndef BGK_H
#define BGK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BGK_OK = 0,
  BGK_ERR_INVALID_ARG = 1,   /* bad argument; nothing changed */
  BGK_ERR_UNSUPPORTED = 2,   /* valid but not built (e.g. order > 3) */
  BGK_ERR_OUT_OF_MEMORY = 3, /* workspace smaller than the footprint */
  BGK_ERR_DEVICE = 4,        /* a HIP runtime call failed */
  BGK_ERR_NEWTON = 5,        /* conservative equilibrium not found */
  BGK_ERR_NONFINITE = 6,     /* non-finite or non-realizable moments */
  BGK_ERR_STATE = 7          /* solver failed earlier / no state installed */
} bgk_status;

typedef enum { BGK_BC_PERIODIC = 0, BGK_BC_SPECULAR = 1, BGK_BC_DIFFUSE = 2 } bgk_bc;

/* Equilibrium the collision term relaxes to. CONSERVATIVE: the discrete
 * Maxwellian exp(alpha . psi) whose trapezoid moments equal those of f
 * (Newton, Sec. 2.1 velocity discretization). CONTINUOUS: the continuous
 * Maxwellian at the (rho, U, theta) of f sampled at the velocity nodes, which
 * does not conserve the discrete moments (the non-conservative model the
 * paper compares against; no Newton solve). */
typedef enum { BGK_EQ_CONSERVATIVE = 0, BGK_EQ_CONTINUOUS = 1 } bgk_equilibrium;

/* Storage precision of f. FP64: everything in FP64. FP32: f stored and the
 * transport/relaxation/Runge-Kutta arithmetic in FP32; moments, Newton solve
 * and relaxation time in FP64. BF16: the state f^n is stored in FP32 and the
 * two intermediate Runge-Kutta stages as BF16 increments over it (stage s
 * reads f^n + increment: the explicit stepping of Sec. 2.2, written as
 * f^(s) = f^n + D_s),
 * arithmetic as for FP32; per-step rounding is then relative to the
 * increment, not to f (BF16 values of f itself would swamp the per-step
 * change). A BF16 solver cannot join a batch (its state buffer alternates
 * between steps) and has no diffuse walls (BGK_ERR_UNSUPPORTED). */
typedef enum { BGK_FP64 = 0, BGK_FP32 = 1, BGK_BF16 = 2 } bgk_precision;

typedef enum { BGK_HOST = 0, BGK_DEVICE = 1 } bgk_where;

/* Problem statement (Sec. 2, Sec. 2.1).
 *   dim, order       spatial dimension d in {1,2,3}; FR order p in {1,2,3}.
 *   nelem, xlo, xhi  uniform Cartesian box; entries beyond dim are ignored.
 *   bc[k][0|1]       left/right boundary of axis k: BGK_BC_PERIODIC (both
 *                    sides must then be periodic) or BGK_BC_SPECULAR
 *                    (mirror of the wall-normal velocity; needs
 *                    vlo[k] == -vhi[k]).
 *   nvel, vlo, vhi   velocity grid (see conventions).
 *   mu_ref, theta_ref, omega
 *                    viscosity law mu = mu_ref (theta/theta_ref)^omega and
 *                    tau = mu/P (Sec. 2); mu_ref <= 0 turns the collision
 *                    term off.
 *   sutherland       > 0 selects Sutherland's law instead of the power law:
 *                    mu = mu_ref (theta/theta_ref)^{3/2} (theta_ref + S) /
 *                    (theta + S) with S = sutherland (temperature units of
 *                    theta); omega is then ignored.
 *   gamma            ratio of specific heats; <= 0 selects 5/3 (monatomic,
 *                    three velocity components).
 *   precision        bgk_precision.
 *   limiter          0 off, 1 Zhang-Shu positivity limiter after each stage.
 *   newton_maxit     Newton iteration cap (<= 0 selects 20).
 *   newton_tol       scaled moment-residual tolerance (<= 0 selects 1e-14).
 *   equilibrium      bgk_equilibrium.
 *   wall_theta[k][s], wall_vel[k][s]
 *                    temperature and velocity of a BGK_BC_DIFFUSE wall on
 *                    side s of axis k (ignored for other boundaries).
 */
typedef struct {
  int32_t dim, order;
  int32_t nelem[3];
  double xlo[3], xhi[3];
  int32_t bc[3][2];
  int32_t nvel[3];
  double vlo[3], vhi[3];
  double mu_ref, theta_ref, omega;
  double gamma;
  int32_t precision, limiter;
  int32_t newton_maxit;
  double newton_tol;
  int32_t equilibrium;
  double wall_theta[3][2];
  double wall_vel[3][2][3];
  double sutherland;
} bgk_problem;

/* Counters accumulated on the device since the last state installation. */
typedef struct {
  int64_t newton_it_max;  /* most Newton residual evaluations at one node */
  int64_t newton_fail;    /* node solves that failed (any stage)          */
  int64_t limiter_hits;   /* (element, velocity) slices contracted         */
  int64_t limiter_bad;    /* slices whose mean was <= 0                    */
  int64_t stages;         /* residual evaluations performed                */
  int64_t positivity_violations; /* BF16 storage: (element or plane,
                          * velocity) slices whose stored stage (F plus the
                          * BF16 increment) has a negative value while the
                          * stage values themselves are all >= 0; negative
                          * increments are truncated towards zero, so this
                          * stays 0 while f^n >= 0                          */
} bgk_diag;

/* Kernel time inside bgk_rk3_step, measured with HIP events recorded on
 * the solver's stream around every launch while timing is enabled. */
typedef struct {
  int64_t stage_launches; /* fused stage kernels (transport+relaxation+RK+limiter) */
  double stage_ms;        /* their summed duration                            */
  int64_t newton_launches;/* per-node equilibrium solves                      */
  double newton_ms;
} bgk_timing;

typedef struct bgk_solver bgk_solver;

/* Device workspace bytes needed for problem *pb, and the node/velocity
 * counts (nx, nv). Any output pointer may be NULL. Host-only; no device
 * work. BGK_ERR_INVALID_ARG / BGK_ERR_UNSUPPORTED for bad problems. */
bgk_status bgk_query_footprint(const bgk_problem* pb, size_t* workspace_bytes, int64_t* nx,
                               int64_t* nv);

/* Create a solver over caller-owned device memory d_workspace (>= footprint
 * bytes, 256-byte aligned, on the current HIP device) and stream
 * hip_stream (a hipStream_t or NULL). The workspace is owned by the caller
 * and must outlive the solver. No state is installed yet. Create does
 * not touch the workspace: the device counters (bgk_diag) are cleared by
 * the first call that queues device work. */
bgk_status bgk_create(const bgk_problem* pb, void* d_workspace, size_t bytes, void* hip_stream,
                      bgk_solver** out);

/* Release the host-side solver object; never touches the workspace.
 * BGK_ERR_STATE (nothing released) while the solver is a batch member. */
bgk_status bgk_destroy(bgk_solver* s);

/* Move the solver to another HIP stream (NULL = default stream) after
 * waiting for the work queued on the current one. Not for batch members. */
bgk_status bgk_set_stream(bgk_solver* s, void* hip_stream);

/* Solution-node coordinates into host x[nx][dim] (Gauss-Legendre points
 * mapped to each element; Sec. 2.1 nodal expansion). */
bgk_status bgk_node_coords(const bgk_solver* s, double* x);

/* Velocity nodes u[nv][3] and trapezoid weights w[nv] into host memory
 * (Sec. 2.1, velocity discretization). */
bgk_status bgk_velocity_grid(const bgk_solver* s, double* u, double* w);

/* Install f (canonical FP64 layout, nx*nv doubles, host or device per
 * where), converting to the storage precision. Clears the failure state
 * and the diagnostics counters. */
bgk_status bgk_set_state(bgk_solver* s, const double* f, int32_t where);

/* Install the continuous Maxwellian rho/(2 pi theta)^{3/2}
 * exp(-|u-U|^2/(2 theta)) (Sec. 2) sampled at every phase-space node;
 * prim[nx][5] = (rho, Ux, Uy, Uz, theta), host or device per where.
 * Requires rho > 0 and theta > 0 at every node (checked for host input). */
bgk_status bgk_set_maxwellian(bgk_solver* s, const double* prim, int32_t where);

/* Copy the state to f (canonical FP64 layout), host or device. Synchronises. */
bgk_status bgk_get_state(bgk_solver* s, double* f, int32_t where);

/* Phase-space residual r = L(f) = -(u . grad_h f) + (g(f) - f)/tau, the
 * right-hand side of the semi-discrete Boltzmann-BGK system (Sec. 2.1: FR
 * transport with upwind fluxes plus the discretely conservative BGK term),
 * without the limiter. f_in (canonical FP64, or NULL for the installed
 * state) and r_out (canonical FP64) are both host or both device per
 * where. For FP32 storage f_in is rounded to FP32 first. The installed
 * state is not modified. Device buffers: asynchronous on the stream.
 * Host buffers are staged through the workspace element by element
 * range; with FP32 storage this needs at least two elements
 * (BGK_ERR_UNSUPPORTED otherwise). */
bgk_status bgk_residual(bgk_solver* s, const double* f_in, double* r_out, int32_t where);

/* Advance the installed state by nsteps steps of size dt with the
 * three-stage SSP Runge-Kutta scheme of Shu and Osher, applying the
 * limiter (if enabled) after every stage (Sec. 2.1 limiter, Sec. 2.2
 * explicit stepping):
 *   f1 = f + dt L(f); f2 = 3/4 f + 1/4 (f1 + dt L(f1));
 *   f  = 1/3 f + 2/3 (f2 + dt L(f2)).
 * Asynchronous on the stream; numerical failures surface at the next
 * synchronising call. */
bgk_status bgk_rk3_step(bgk_solver* s, double dt, int32_t nsteps);

/* Conserved variables Q[nx][5] = M . [f (x) psi] of the installed state
 * (Sec. 2 moments with the Sec. 2.1 trapezoid operator), FP64, host or
 * device. Synchronises. */
bgk_status bgk_moments(bgk_solver* s, double* Q, int32_t where);

/* Discrete moments Cm[nx][5] = M . [C (x) psi] of the BGK collision term
 * C = (g - f)/tau of the installed state (Sec. 2 relaxation; Sec. 2.1: the
 * discretely conservative equilibrium makes these vanish), FP64, host or
 * device per where. C is formed exactly as the stage kernels form it (the
 * same FP64 equilibrium rows from the same equilibrium solve, the same stored
 * values of f, the same FP64 arithmetic, in every storage precision), and its
 * moments are accumulated in FP64 in a fixed order, so Cm measures the
 * conservation of the collision term the solver applies. Zero when
 * collisions are off. Synchronises; the next step recomputes the moment
 * partials of the state. */
bgk_status bgk_collision_moments(bgk_solver* s, double* Cm, int32_t where);

/* Maximum scratch of bgk_residual_noalloc: a static device array of this many
 * bytes per GPU the library runs on, held until the process ends. */
#define BGK_NOALLOC_SCRATCH_BYTES (64ull << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * residual r = L(f) of bgk_residual for problem *pb without a solver or
 * workspace. f_in and r_out are device buffers in the canonical FP64 layout
 * (nx*nv doubles each, caller-owned); everything else the kernels use (the
 * internal copy of f in the storage precision, moment partials, equilibrium
 * parameters and rows, counters) lives in the library's static scratch array
 * of BGK_NOALLOC_SCRATCH_BYTES bytes. Calls no hipMalloc, hipFree or memset:
 * kernels only, queued on hip_stream (a hipStream_t or NULL), asynchronous;
 * the counters are cleared by a kernel at the start of every call. The
 * result equals bgk_residual's for the same problem and input.
 * Errors: BGK_ERR_INVALID_ARG / BGK_ERR_UNSUPPORTED as bgk_query_footprint;
 * BGK_ERR_UNSUPPORTED for diffuse walls; BGK_ERR_OUT_OF_MEMORY (nothing
 * queued) when the problem needs more scratch than the array holds (about
 * 2.5M phase-space DOF in FP64 storage). Numerical failures are not reported
 * (nothing synchronises): r_out then holds NaN where an equilibrium solve
 * failed. Every call on one GPU shares that GPU's scratch array: calls that
 * overlap in time on one GPU (different streams, or threads) race; calls on
 * one stream are ordered. */
bgk_status bgk_residual_noalloc(const bgk_problem* pb, const double* f_in, double* r_out,
                                void* hip_stream);

/* Time step dt = min(cfl / max_j sum_{k<d} |u_jk| / h_k, min_nodes tau) of
 * the installed state. Synchronises. */
bgk_status bgk_stable_dt(bgk_solver* s, double cfl, double* dt);

/* Read the device counters. Synchronises. Returns BGK_ERR_NEWTON if any
 * node solve failed since the state was installed (out is still filled). */
bgk_status bgk_diagnostics(bgk_solver* s, bgk_diag* out);

/* Enable (on != 0) or disable event timing of the launches queued by
 * bgk_rk3_step. Measurement aid for the throughput/roofline report; events
 * are created by the HIP runtime on first use and kept by the solver. */
bgk_status bgk_timing_enable(bgk_solver* s, int32_t on);

/* Synchronise, sum the recorded kernel durations into *out and clear the
 * record. */
bgk_status bgk_timing_read(bgk_solver* s, bgk_timing* out);

/* Wait for the solver's queued work and report any numerical failure. */
bgk_status bgk_synchronize(bgk_solver* s);

/* ------------------------------------------------------------------------
 * Batches (serving): resident FP64- or FP32-storage solvers of 1-D and 2-D
 * problems (the SSP-RK3 steps of Sec. 2.2, the same kernels' arithmetic as
 * bgk_rk3_step) advanced together. The arguments of every member live in
 * descriptor tables in a caller-supplied device workspace. A replay runs up
 * to four sub-steps, each three RK stages of [the equilibrium solves of the
 * members per team size, the diffuse-wall densities, one stage launch per
 * kernel family (dimension, order, storage precision)], each launch covering
 * all members of its kind with one work-group per work unit; a member of
 * 8192 stage work units (element x velocity chunk) or more, which fills the
 * device alone, runs its stages with the launches bgk_rk3_step makes for it
 * (column sweeps where its solver sweeps) in place of its family's. The member that
 * moves the most bytes per step takes one step per replay, a member moving W
 * times fewer takes the largest power of two <= min(W, 4) (at most its
 * remaining steps), so small requests are not paced by the largest. Members
 * never exchange data and every work unit runs the same arithmetic as in
 * bgk_rk3_step, so each member's result is bitwise the one it gets alone.
 * Admission, completion and removal rewrite the tables (copied on the batch
 * stream from pinned host staging, ahead of the launches that read them). A
 * batch does not own its members: the caller keeps every solver and its
 * workspace alive until the solver has been polled or removed, then may
 * destroy it.
 * ------------------------------------------------------------------------ */
typedef struct bgk_batch bgk_batch;

/* Bytes of device workspace a batch of max_members (1..64) members needs
 * (descriptor tables; independent of the members' sizes). */
bgk_status bgk_batch_query_footprint(int32_t max_members, size_t* bytes);

/* Create a batch on hip_stream (NULL = default stream) with room for
 * max_members (1..64) concurrent members. d_workspace: device memory of at
 * least bgk_batch_query_footprint(max_members) bytes, 256-byte aligned, owned
 * by the caller and kept until bgk_batch_destroy returns. Allocates two
 * pinned host staging buffers of the same size (released by destroy).
 * BGK_ERR_OUT_OF_MEMORY if bytes is too small. */
bgk_status bgk_batch_create(void* hip_stream, int32_t max_members, void* d_workspace, size_t bytes,
                            bgk_batch** out);

/* Add solver s (state installed, FP64 or FP32 storage, 1-D or 2-D problem,
 * created on the batch's stream, timing off, not in another batch) to advance
 * nsteps >= 1 steps of size dt. BGK_ERR_OUT_OF_MEMORY when the batch is full;
 * BGK_ERR_UNSUPPORTED for BF16 increments or hexahedra (step those with
 * bgk_rk3_step). */
bgk_status bgk_batch_add(bgk_batch* b, bgk_solver* s, double dt, int64_t nsteps);

/* Queue nsteps replays (see above; a member stops after its own step count
 * and becomes pollable). Asynchronous on the batch stream, except that it
 * waits while more than 8 replays are queued beyond the last one the device
 * has completed (so a caller admitting new members between calls is never
 * far behind the device). */
bgk_status bgk_batch_step(bgk_batch* b, int32_t nsteps);

/* Hand back up to cap members that have completed their steps, in
 * completion order, waiting until the device has executed their last
 * replay: done[i] and its status status[i] (BGK_OK, or BGK_ERR_NEWTON when
 * an equilibrium solve of the member failed; the solver is then marked
 * failed). They leave the batch and their slots become free; *ndone is the
 * count. Later replays may still be running when it returns. */
bgk_status bgk_batch_poll(bgk_batch* b, bgk_solver** done, int32_t* status, int32_t cap,
                          int32_t* ndone);

/* As bgk_batch_poll, but without waiting: only members whose last replay the
 * device has already executed (possibly none). */
bgk_status bgk_batch_poll_ready(bgk_batch* b, bgk_solver** done, int32_t* status, int32_t cap,
                                int32_t* ndone);

/* Remove an active member before completion (waits for queued work). */
bgk_status bgk_batch_remove(bgk_batch* b, bgk_solver* s);

/* Number of active members (0 for NULL). */
int32_t bgk_batch_size(const bgk_batch* b);

/* Wait for queued work and release the batch (members and workspace are not
 * touched). */
bgk_status bgk_batch_destroy(bgk_batch* b);

const char* bgk_status_str(bgk_status st);
const char* bgk_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BGK_H */
