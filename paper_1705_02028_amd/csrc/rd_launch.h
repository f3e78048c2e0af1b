// Host-side launchers of the gfx950 kernels (defined in rd_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "rd_adjoint.h"
#include "rd_device.h"
#include "rd_tiles.h"

namespace rd {

constexpr int kBlock = 256;
constexpr int kCflSpan = 4 * kBlock;  // vertices per block of the CFL reduction

// Segmented min-reduction layout for the CFL limit: vertex block b covers
// vertices [blk_v0[b], blk_v1[b]) (at most kCflSpan) of one mesh; mesh m owns blocks
// [mesh_b0[m], mesh_b0[m+1]).
struct CflPlan {
  int32_t nblocks = 0, nmesh = 0;
  const int32_t* blk_v0 = nullptr;
  const int32_t* blk_v1 = nullptr;
  const int32_t* mesh_b0 = nullptr;
  double* part = nullptr;
  double* vpart = nullptr;  // [2 nblocks] Bx speed range per block
};

// cfl: also write l_max lambda_max per corner (stage 1 only)
hipError_t launch_tri(const Dev& d, int fp32, int scheme, int stage, bool save, bool cfl, hipStream_t s);
hipError_t launch_gather(const Dev& d, int fp32, int mode, double* out_soa, hipStream_t s);
// tiled: the stage-2 wall term reads W* rebuilt from R1
hipError_t launch_wall(const Dev& d, bool stage2, hipStream_t s, bool tiled = false);
hipError_t launch_cfl(const Dev& d, const CflPlan& p, double cfl, hipStream_t s);
// Bx sensor range: smallest and largest |v| per mesh -> d.vr, over the same
// vertex blocks as the CFL reduction; mode 0 at W^n, 1 at W* (Ws), 2 at W*
// rebuilt from R1 (tiled form)
hipError_t launch_vrange(const Dev& d, const CflPlan& p, int mode, hipStream_t s);
// part 0: l_max lambda_max per triangle (FP64); part 1: per-vertex bounds
// (sums of the terms of the vertex's triangles, float when fp32: as the FP32
// triangle pass writes them) and block minima; part 3: the same from the bounds the
// tiled passes store in d.cflv; part 2: per-mesh minimum -> d.dt
hipError_t launch_cfl_part(const Dev& d, const CflPlan& p, double cfl, int part, hipStream_t s, int fp32 = 0);
hipError_t launch_set_state(const Dev& d, const double* soa, int fp32, hipStream_t s);
hipError_t launch_refresh(const Dev& d, int fp32, hipStream_t s);
hipError_t launch_get_state(const Dev& d, const D4* src, double* soa, hipStream_t s);
hipError_t launch_aos_to_soa(const D4* src, double* soa, int64_t n, hipStream_t s);
// FP64 kept triangle residuals (keepT) to component-major arrays
hipError_t launch_keep_to_soa(const void* keep, double* soa, int64_t n, hipStream_t s);
hipError_t launch_set_scalar(double* p, double v, hipStream_t s);
hipError_t launch_set_int(int* p, int v, hipStream_t s);
// p[0..n) = v
hipError_t launch_fill_int(int* p, int v, int64_t n, hipStream_t s);
// *dst |= *src
hipError_t launch_or_int(int* dst, const int* src, hipStream_t s);
hipError_t launch_copy4(D4* dst, const D4* src, int64_t n, hipStream_t s);
hipError_t launch_soa_to_aos(const double* soa, D4* dst, int64_t n, hipStream_t s);
// Tiled form (rd_tiles.hip): one workgroup per tile of min(tl.tt, kBlock)
// threads in stage 1, half as many (at least 64) in stage 2, whose tile pass
// idles its waves less at the barriers with two triangles per thread (a
// thread takes several triangles of a larger tile).
inline int tile_threads(const Tiles& tl, int stage) {
  int t = stage == 2 ? tl.tt / 2 : tl.tt;
  t = t < 64 ? 64 : t;
  return t < kBlock ? t : kBlock;
}
// stage 1 (also Euler): R1 and, with cfl, the CFL bounds of interior
// vertices; stage 2: the new state of interior vertices.
hipError_t launch_tile(const Dev& d, const Tiles& tl, int fp32, int scheme, int stage, bool save, bool cfl,
                       hipStream_t s);
// The same for the shared vertices.
hipError_t launch_shared(const Dev& d, const Tiles& tl, int fp32, int stage, bool cfl, hipStream_t s);
// Forward-Euler update from R1.
hipError_t launch_euler_apply(const Dev& d, int fp32, hipStream_t s);
// Dynamic LDS bytes of a tile workgroup.
size_t tile_lds_bytes(const Tiles& tl, int fp32, int stage, bool cfl);

// The adjoint's first-stage vertex pass: W* from the stage-1 parts and the
// stage-2 reverse records (Z at W*, W* - W^n, mu2) of every vertex.
hipError_t launch_adj_star(const Dev& d, const AdjDev& a, hipStream_t s);
// Reverse of one step (FP64): stage-2 triangles and gather (rk2), then
// stage-1 triangles and gather; dL/dW^n goes to out [4][nv].
hipError_t launch_adjoint(const Dev& d, const AdjDev& a, int scheme, int rk2, double* out, hipStream_t s);

}  // namespace rd
