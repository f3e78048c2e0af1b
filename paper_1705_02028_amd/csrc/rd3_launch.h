// Host-side launchers of the three-dimensional kernels (rd3_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "rd3_device.h"

namespace rd3 {

// Z and |u| + c of the state src ([5][nv]).
hipError_t launch3_z(const Dev3& d, const double* src, hipStream_t s);
// One tetrahedron pass: stage 1 (or Euler) reads d.Z of W (keep: store the
// N parts and the residual for stage 2); stage 2 reads d.Z of Ws.
hipError_t launch3_tet(const Dev3& d, int stage, int scheme, bool keep, hipStream_t s);
// Vertex sums and update: mode 0 Euler, 1 first stage, 2 second stage.
hipError_t launch3_gather(const Dev3& d, int mode, hipStream_t s);
// CFL limit of d.sig times cfl -> *d.dt (d.bmin holds cfl_blocks(nv) values).
int cfl_blocks(int64_t nv);
hipError_t launch3_cfl(const Dev3& d, double cfl, hipStream_t s);
hipError_t launch3_set_dt(const Dev3& d, double dt, hipStream_t s);

}  // namespace rd3
