// bgk_launch.hpp -- host-side launch interface between the C-ABI runtime and
// the gfx950 kernels. Internal to libbgk.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "bgk_device.hpp"

namespace bgk {

// Velocities covered by one work-group of the stage kernel (the moment
// partials are per such chunk).
int velocities_per_block(int dim, int order, int precision);
// Hexahedra of this order and storage precision run the one-lane-per-velocity
// stage kernels (else the plane-split ones).
bool hex_one_lane(int order, int precision);

// Elements per work item of the column-sweep stage kernels for this mesh,
// velocity grid and storage precision on the current device (0: no sweep).
int sweep_segment(const DevGeom& g, int precision, bool collide);
// mode 0: fused RK stage (a variant that does not read f^n when a = 0);
// 1: residual L(f) in FP64; 2: moment partials only.
hipError_t launch_stage(int precision, int mode, const StageArgs& A, hipStream_t s);
hipError_t launch_newton(const NewtonArgs& A, hipStream_t s);
// Re-emitted densities of the diffuse-wall flux points of the stage input.
hipError_t launch_wall(int precision, const WallArgs& W, hipStream_t s);
hipError_t launch_reduce_partials(const DevGeom& g, const double* partials, double* Q,
                                  hipStream_t s);
// Moments of the collision term of the stage input A.fin into Cm[nx][5]
// (uses A.partials as scratch).
hipError_t launch_collision_moments(int precision, const StageArgs& A, double* Cm,
                                    hipStream_t s);
// Team size of the equilibrium solve for a mesh of nx nodes.
int newton_team(int64_t nx);
// Batched launches over descriptor tables in device memory (1-D and 2-D
// members, FP64 or FP32 storage): RK stage `stage` of the members of one
// kernel family, the equilibrium solves of the members of one team size, the
// diffuse-wall fluxes of one family and the wall densities of all members.
// grid: the list's work units (one per work-group); 0 launches nothing.
hipError_t launch_stage_batch(int precision, int dim, int order, int stage, const StageArgs* args,
                              const BatchList* list, size_t tab_bytes, unsigned grid,
                              hipStream_t s);
hipError_t launch_newton_batch(int team, const NewtonArgs* args, const BatchList* list,
                               unsigned grid, hipStream_t s);
hipError_t launch_wall_flux_batch(int precision, int dim, int order, int stage,
                                  const WallArgs* args, const BatchList* list, unsigned grid,
                                  hipStream_t s);
hipError_t launch_wall_rho_batch(int stage, const WallArgs* args, const BatchList* list,
                                 unsigned grid, hipStream_t s);
hipError_t launch_maxwellian(int precision, const DevGeom& g, const double* prim, void* f,
                             hipStream_t s);
hipError_t launch_to_storage(int precision, const DevGeom& g, const double* in, void* out,
                             int64_t i0, int64_t m, hipStream_t s);
hipError_t launch_from_storage(int precision, const DevGeom& g, const void* in, double* out,
                               int64_t i0, int64_t m, hipStream_t s);

}  // namespace bgk
