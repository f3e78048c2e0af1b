// gfx950 kernels of the two-pass residual-distribution step, the CFL
// reduction, state conversion and the adjoint, with their launchers.
//
// Launch shapes: one thread per triangle (triangle passes) or per vertex
// (gather, CFL), 256-thread workgroups, block ids renumbered per XCD.
#include "rd_adjoint.h"
#include "rd_kcommon.h"
#include "rd_launch.h"

namespace rd {

// One thread per triangle. (A persistent grid with the next triangle's loads
// software-pipelined was measured slower: fewer waves in flight and, with
// per-workgroup chunks, scattered working sets.)
template <typename R, int SCHEME, int STAGE, bool SAVE, bool CFL, bool LUMP>
__global__ __launch_bounds__(kBlock, (TriKernelWaves<R, SCHEME, STAGE, SAVE, CFL>::value)) void k_tri(Dev d) {
  const int64_t t = xcd_block() * kBlock + threadIdx.x;
  if (t < d.nt) tri_body<R, SCHEME, STAGE, SAVE, CFL, LUMP>(t, d);
}

template <typename R, int MODE>
__global__ __launch_bounds__(kBlock) void k_gather(Dev d, double* out_soa) {
  const int64_t v = xcd_block() * kBlock + threadIdx.x;
  if (v < d.nv) gather_body<R, MODE>(v, d, out_soa);
}

template <bool STAGE2, bool TILED>
__global__ __launch_bounds__(kBlock) void k_wall(Dev d) {
  const int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (b < d.nwv) wall_body<STAGE2, TILED>(b, d);
}

__global__ __launch_bounds__(kBlock) void k_cfl_tri(Dev d) {
  const int64_t t = xcd_block() * kBlock + threadIdx.x;
  if (t < d.nt) cfl_tri_body(t, d);
}

// Per-vertex CFL bounds 2 V_i / sum l_max lambda_max (summed over the terms of
// the vertex's triangles, or read from the bounds the tiled passes store) and
// their block minima.
template <bool FROM_CFLV, typename R>
__global__ __launch_bounds__(kBlock) void k_cfl_vertex(Dev d, CflPlan p) {
  const int b = blockIdx.x;
  double x = INFINITY;
#pragma unroll
  for (int u = 0; u < kCflSpan / kBlock; ++u) {
    const int64_t v = (int64_t)p.blk_v0[b] + u * kBlock + threadIdx.x;
    if (v < p.blk_v1[b]) x = rmin(x, FROM_CFLV ? d.cflv[v] : cfl_vertex_bound<R>(v, d));
  }
  const double m = block_min(x);
  if (threadIdx.x == 0) p.part[b] = m;
}

// Per-mesh minimum over the mesh's blocks -> dt.
__global__ __launch_bounds__(kBlock) void k_cfl_final(Dev d, CflPlan p, double cfl) {
  const int m = blockIdx.x;
  double x = INFINITY;
  for (int b = p.mesh_b0[m] + threadIdx.x; b < p.mesh_b0[m + 1]; b += kBlock) x = rmin(x, p.part[b]);
  x = block_min(x);
  if (threadIdx.x == 0) d.dt[m] = cfl * x;
}

// Smallest and largest flow speed |v| over each CFL block's vertices (the Bx
// sensor's range), at W^n (MODE 0), at W* held in Ws (MODE 1) or at W*
// formed from the stage-1 residual (MODE 2, tiled form); then per mesh.
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_vrange(Dev d, CflPlan p) {
  const int b = blockIdx.x;
  double lo = INFINITY, hi = 0.0;
#pragma unroll
  for (int u = 0; u < kCflSpan / kBlock; ++u) {
    const int64_t v = (int64_t)p.blk_v0[b] + u * kBlock + threadIdx.x;
    if (v < p.blk_v1[b]) {
      const D4 w = MODE == 0 ? d.W[v] : (MODE == 1 ? d.Ws[v] : star_state(d, v, d.bc ? d.bc[v] : -1,
                                                                            d.vmesh ? d.vmesh[v] : 0));
      const double sp = flow_speed(w);
      lo = rmin(lo, sp);
      hi = rmax(hi, sp);
    }
  }
  lo = block_min(lo);
  __syncthreads();
  hi = -block_min(-hi);
  if (threadIdx.x == 0) {
    p.vpart[2 * b] = lo;
    p.vpart[2 * b + 1] = hi;
  }
}

__global__ __launch_bounds__(kBlock) void k_vrange_final(Dev d, CflPlan p) {
  const int m = blockIdx.x;
  double lo = INFINITY, hi = 0.0;
  for (int b = p.mesh_b0[m] + threadIdx.x; b < p.mesh_b0[m + 1]; b += kBlock) {
    lo = rmin(lo, p.vpart[2 * b]);
    hi = rmax(hi, p.vpart[2 * b + 1]);
  }
  lo = block_min(lo);
  __syncthreads();
  hi = -block_min(-hi);
  if (threadIdx.x == 0) {
    d.vr[3 * m] = lo;
    d.vr[3 * m + 1] = hi;
  }
}

__global__ __launch_bounds__(kBlock) void k_set_state(Dev d, const double* soa, int fp32) {
  const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (v >= d.nv) return;
  const double w[4] = {soa[v], soa[d.nv + v], soa[2 * d.nv + v], soa[3 * d.nv + v]};
  st4<double>(d.W, v, w);
  vertex_epilogue(d, v, w, fp32 != 0);
}

__global__ __launch_bounds__(kBlock) void k_refresh(Dev d, int fp32) {
  const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (v >= d.nv) return;
  const D4 w = d.W[v];
  vertex_epilogue(d, v, w.v, fp32 != 0);
}

__global__ __launch_bounds__(kBlock) void k_aos_to_soa(const D4* src, double* soa, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const D4 w = src[i];
  for (int k = 0; k < 4; ++k) soa[k * n + i] = w.v[k];
}

__global__ void k_set_scalar(double* p, double v) { p[0] = v; }
__global__ void k_set_int(int* p, int v) { p[0] = v; }
__global__ void k_or_int(int* dst, const int* src) { dst[0] = dst[0] | src[0]; }
__global__ __launch_bounds__(kBlock) void k_fill_int(int* p, int v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = v;
}


__global__ __launch_bounds__(kBlock) void k_copy4(D4* dst, const D4* src, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// ------------------------------------------------------------- adjoint --

// The reverse triangle kernels run one wavefront per SIMD (their registers
// fill the SIMD); one-wavefront workgroups let each SIMD start its next
// wavefront as soon as its own finishes.
constexpr int kAdjBlock = 64;

template <int SCHEME>
__global__ __launch_bounds__(kAdjBlock) void k_adj_tri2(Dev d, AdjDev a) {
  const int64_t t = xcd_block() * kAdjBlock + threadIdx.x;
  if (t < d.nt) adj_tri2_body<SCHEME>(t, d, a);
}

template <int SCHEME>
__global__ __launch_bounds__(kAdjBlock) void k_adj_tri1(Dev d, AdjDev a, int rk2) {
  const int64_t t = xcd_block() * kAdjBlock + threadIdx.x;
  if (t < d.nt) adj_tri1_body<SCHEME>(t, d, a, rk2 != 0);
}

__global__ __launch_bounds__(kBlock) void k_adj_star(Dev d, AdjDev a) {
  const int64_t v = xcd_block() * kBlock + threadIdx.x;
  if (v < d.nv) adj_star_body(v, d, a);
}

__global__ __launch_bounds__(kBlock) void k_adj_euler_prep(Dev d, AdjDev a) {
  const int64_t v = xcd_block() * kBlock + threadIdx.x;
  if (v < d.nv) adj_euler_prep_body(v, d, a);
}

__global__ __launch_bounds__(kBlock) void k_adj_gather2(Dev d, AdjDev a) {
  const int64_t v = xcd_block() * kBlock + threadIdx.x;
  if (v < d.nv) adj_gather2_body(v, d, a);
}

__global__ __launch_bounds__(kBlock) void k_adj_gather1(Dev d, AdjDev a, int rk2, double* out) {
  const int64_t v = xcd_block() * kBlock + threadIdx.x;
  if (v < d.nv) adj_gather1_body(v, d, a, rk2 != 0, out);
}

__global__ __launch_bounds__(kBlock) void k_soa_to_aos(const double* soa, D4* dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double w[4] = {soa[i], soa[n + i], soa[2 * n + i], soa[3 * n + i]};
  st4<double>(dst, i, w);
}

__global__ __launch_bounds__(kBlock) void k_zero4(D4* dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double z[4] = {0.0, 0.0, 0.0, 0.0};
  st4<double>(dst, i, z);
}

template <int SCHEME>
static void adj_tris(const Dev& d, const AdjDev& a, int stage, int rk2, hipStream_t s) {
  const unsigned g = (unsigned)((d.nt + kAdjBlock - 1) / kAdjBlock);
  if (stage == 2) hipLaunchKernelGGL((k_adj_tri2<SCHEME>), dim3(g), dim3(kAdjBlock), 0, s, d, a);
  else hipLaunchKernelGGL((k_adj_tri1<SCHEME>), dim3(g), dim3(kAdjBlock), 0, s, d, a, rk2);
}

hipError_t launch_adjoint(const Dev& d, const AdjDev& a, int scheme, int rk2, double* out, hipStream_t s) {
  auto tris = [&](int stage) {
    switch (scheme) {
      case SCH_N: adj_tris<SCH_N>(d, a, stage, rk2, s); break;
      case SCH_LDA: adj_tris<SCH_LDA>(d, a, stage, rk2, s); break;
      case SCH_B: adj_tris<SCH_B>(d, a, stage, rk2, s); break;
      case SCH_BMAX: adj_tris<SCH_BMAX>(d, a, stage, rk2, s); break;
      default: adj_tris<SCH_BMIN>(d, a, stage, rk2, s); break;
    }
  };
  if (rk2) {
    tris(2);
    hipLaunchKernelGGL(k_adj_gather2, dim3(nblk(d.nv)), dim3(kBlock), 0, s, d, a);
  } else {
    hipLaunchKernelGGL(k_adj_euler_prep, dim3(nblk(d.nv)), dim3(kBlock), 0, s, d, a);
  }
  tris(1);
  hipLaunchKernelGGL(k_adj_gather1, dim3(nblk(d.nv)), dim3(kBlock), 0, s, d, a, rk2, out);
  return hipGetLastError();
}

hipError_t launch_adj_star(const Dev& d, const AdjDev& a, hipStream_t s) {
  if (d.nv == 0) return hipSuccess;
  hipLaunchKernelGGL(k_adj_star, dim3(nblk(d.nv)), dim3(kBlock), 0, s, d, a);
  return hipGetLastError();
}

hipError_t launch_soa_to_aos(const double* soa, D4* dst, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_soa_to_aos, dim3(nblk(n)), dim3(kBlock), 0, s, soa, dst, n);
  return hipGetLastError();
}

template <typename R, int SCHEME, int STAGE, bool SAVE, bool CFL, bool LUMP = false>
static hipError_t tri_launch(const Dev& d, hipStream_t s) {
  hipLaunchKernelGGL((k_tri<R, SCHEME, STAGE, SAVE, CFL, LUMP>), dim3(nblk(d.nt)), dim3(kBlock), 0, s, d);
  return hipGetLastError();
}

template <typename R, int SCHEME>
static hipError_t tri_dispatch(const Dev& d, int stage, bool save, bool cfl, hipStream_t s) {
  if (stage == 1 && save && cfl) return tri_launch<R, SCHEME, 1, true, true>(d, s);
  if (stage == 1 && save) return tri_launch<R, SCHEME, 1, true, false>(d, s);
  if (stage == 1 && cfl) return tri_launch<R, SCHEME, 1, false, true>(d, s);
  if (stage == 1) return tri_launch<R, SCHEME, 1, false, false>(d, s);
  if (d.slump) return tri_launch<R, SCHEME, 2, false, false, true>(d, s);
  return tri_launch<R, SCHEME, 2, false, false>(d, s);
}

template <typename R>
static hipError_t tri_scheme(const Dev& d, int scheme, int stage, bool save, bool cfl, hipStream_t s) {
  switch (scheme) {
    case SCH_N: return tri_dispatch<R, SCH_N>(d, stage, save, cfl, s);
    case SCH_LDA: return tri_dispatch<R, SCH_LDA>(d, stage, save, cfl, s);
    case SCH_B: return tri_dispatch<R, SCH_B>(d, stage, save, cfl, s);
    case SCH_BMAX: return tri_dispatch<R, SCH_BMAX>(d, stage, save, cfl, s);
    case SCH_BMIN: return tri_dispatch<R, SCH_BMIN>(d, stage, save, cfl, s);
    case SCH_BX: return tri_dispatch<R, SCH_BX>(d, stage, save, cfl, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_tri(const Dev& d, int fp32, int scheme, int stage, bool save, bool cfl, hipStream_t s) {
  if (d.nt == 0) return hipSuccess;
  return fp32 ? tri_scheme<float>(d, scheme, stage, save, cfl, s)
              : tri_scheme<double>(d, scheme, stage, save, cfl, s);
}

template <typename R>
static hipError_t gather_mode(const Dev& d, int mode, double* out, hipStream_t s) {
  const dim3 g(nblk(d.nv)), b(kBlock);
  switch (mode) {
    case G_EULER: hipLaunchKernelGGL((k_gather<R, G_EULER>), g, b, 0, s, d, out); break;
    case G_STAGE1: hipLaunchKernelGGL((k_gather<R, G_STAGE1>), g, b, 0, s, d, out); break;
    case G_STAGE2: hipLaunchKernelGGL((k_gather<R, G_STAGE2>), g, b, 0, s, d, out); break;
    case G_RESIDUAL: hipLaunchKernelGGL((k_gather<R, G_RESIDUAL>), g, b, 0, s, d, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_gather(const Dev& d, int fp32, int mode, double* out_soa, hipStream_t s) {
  if (d.nv == 0) return hipSuccess;
  return fp32 ? gather_mode<float>(d, mode, out_soa, s) : gather_mode<double>(d, mode, out_soa, s);
}

hipError_t launch_wall(const Dev& d, bool stage2, hipStream_t s, bool tiled) {
  if (d.nwv == 0) return hipSuccess;
  if (stage2 && tiled) hipLaunchKernelGGL((k_wall<true, true>), dim3(nblk(d.nwv)), dim3(kBlock), 0, s, d);
  else if (stage2) hipLaunchKernelGGL((k_wall<true, false>), dim3(nblk(d.nwv)), dim3(kBlock), 0, s, d);
  else hipLaunchKernelGGL((k_wall<false, false>), dim3(nblk(d.nwv)), dim3(kBlock), 0, s, d);
  return hipGetLastError();
}

hipError_t launch_cfl_part(const Dev& d, const CflPlan& p, double cfl, int part, hipStream_t s, int fp32) {
  if (part == 0) hipLaunchKernelGGL(k_cfl_tri, dim3(nblk(d.nt)), dim3(kBlock), 0, s, d);
  else if (part == 1 && fp32) hipLaunchKernelGGL((k_cfl_vertex<false, float>), dim3(p.nblocks), dim3(kBlock), 0, s, d, p);
  else if (part == 1) hipLaunchKernelGGL((k_cfl_vertex<false, double>), dim3(p.nblocks), dim3(kBlock), 0, s, d, p);
  else if (part == 3) hipLaunchKernelGGL((k_cfl_vertex<true, double>), dim3(p.nblocks), dim3(kBlock), 0, s, d, p);
  else hipLaunchKernelGGL(k_cfl_final, dim3(p.nmesh), dim3(kBlock), 0, s, d, p, cfl);
  return hipGetLastError();
}

hipError_t launch_vrange(const Dev& d, const CflPlan& p, int mode, hipStream_t s) {
  if (p.nblocks == 0) return hipSuccess;
  if (mode == 0) hipLaunchKernelGGL(k_vrange<0>, dim3(p.nblocks), dim3(kBlock), 0, s, d, p);
  else if (mode == 1) hipLaunchKernelGGL(k_vrange<1>, dim3(p.nblocks), dim3(kBlock), 0, s, d, p);
  else if (mode == 2) hipLaunchKernelGGL(k_vrange<2>, dim3(p.nblocks), dim3(kBlock), 0, s, d, p);
  else return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_vrange_final, dim3(p.nmesh), dim3(kBlock), 0, s, d, p);
  return hipGetLastError();
}

hipError_t launch_cfl(const Dev& d, const CflPlan& p, double cfl, hipStream_t s) {
  for (int part = 0; part < 3; ++part) {
    hipError_t e = launch_cfl_part(d, p, cfl, part, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_set_state(const Dev& d, const double* soa, int fp32, hipStream_t s) {
  hipLaunchKernelGGL(k_set_state, dim3(nblk(d.nv)), dim3(kBlock), 0, s, d, soa, fp32);
  return hipGetLastError();
}

hipError_t launch_refresh(const Dev& d, int fp32, hipStream_t s) {
  hipLaunchKernelGGL(k_refresh, dim3(nblk(d.nv)), dim3(kBlock), 0, s, d, fp32);
  return hipGetLastError();
}

hipError_t launch_get_state(const Dev& d, const D4* src, double* soa, hipStream_t s) {
  hipLaunchKernelGGL(k_aos_to_soa, dim3(nblk(d.nv)), dim3(kBlock), 0, s, src, soa, d.nv);
  return hipGetLastError();
}

hipError_t launch_aos_to_soa(const D4* src, double* soa, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_aos_to_soa, dim3(nblk(n)), dim3(kBlock), 0, s, src, soa, n);
  return hipGetLastError();
}

hipError_t launch_set_scalar(double* p, double v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(1), 0, s, p, v);
  return hipGetLastError();
}

hipError_t launch_set_int(int* p, int v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, p, v);
  return hipGetLastError();
}

hipError_t launch_fill_int(int* p, int v, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_int, dim3(nblk(n)), dim3(kBlock), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_or_int(int* dst, const int* src, hipStream_t s) {
  hipLaunchKernelGGL(k_or_int, dim3(1), dim3(1), 0, s, dst, src);
  return hipGetLastError();
}

hipError_t launch_copy4(D4* dst, const D4* src, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy4, dim3(nblk(n)), dim3(kBlock), 0, s, dst, src, n);
  return hipGetLastError();
}

}  // namespace rd
