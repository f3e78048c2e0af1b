// gfx950 kernels of the tiled step: one workgroup per triangle tile, the
// tile's vertex data staged in LDS (see rd_tiles.h for the phases), then a
// vertex pass over the shared vertices.
#include "rd_kcommon.h"
#include "rd_launch.h"

namespace rd {

template <typename R, int SCHEME, bool SAVE, bool CFL>
__global__ __launch_bounds__(kBlock, TriWaves<R>::value) void k_tile1(Dev d, Tiles tl) {
  extern __shared__ D4 lds_raw[];
  const int64_t tile = xcd_block();
  TileLds<R> L;
  tile_lds<R>(tl, 1, CFL, reinterpret_cast<char*>(lds_raw), &L);
  const int32_t nthr = blockDim.x, tid = threadIdx.x;
  const int32_t nlv = tl.vbeg[tile + 1] - tl.vbeg[tile];
  for (int32_t l = tid; l < nlv; l += nthr) tile_load1<R, CFL>(tile, l, d, tl, L);
  __syncthreads();
  const int32_t ntri = tl.tbeg[tile + 1] - tl.tbeg[tile];
  for (int32_t j = tid; j < ntri; j += nthr) tile_tri<R, SCHEME, 1, SAVE, CFL>(tile, j, d, tl, L);
  __syncthreads();
  const int32_t nvi = tl.nvi[tile];
  for (int32_t l = tid; l < nvi; l += nthr) tile_sum1<R, CFL>(tile, l, d, tl, L);
}

template <typename R, int SCHEME, bool LUMP>
__global__ __launch_bounds__(kBlock, TriWaves<R>::value) void k_tile2(Dev d, Tiles tl) {
  extern __shared__ D4 lds_raw[];
  const int64_t tile = xcd_block();
  TileLds<R> L;
  tile_lds<R>(tl, 2, false, reinterpret_cast<char*>(lds_raw), &L);
  const int32_t nthr = blockDim.x, tid = threadIdx.x;
  const int32_t nlv = tl.vbeg[tile + 1] - tl.vbeg[tile];
  for (int32_t l = tid; l < nlv; l += nthr) tile_load2<R>(tile, l, d, tl, L);
  __syncthreads();
  const int32_t ntri = tl.tbeg[tile + 1] - tl.tbeg[tile];
  for (int32_t j = tid; j < ntri; j += nthr) tile_tri<R, SCHEME, 2, false, false, LUMP>(tile, j, d, tl, L);
  __syncthreads();
  const int32_t nvi = tl.nvi[tile];
  for (int32_t l = tid; l < nvi; l += nthr) tile_sum2<R>(tile, l, d, tl, L);
}

template <typename R, bool CFL>
__global__ __launch_bounds__(kBlock) void k_shared1(Dev d, Tiles tl) {
  const int64_t k = xcd_block() * kBlock + threadIdx.x;
  if (k < tl.nsv) shared_sum1<R, CFL>(k, d, tl);
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_shared2(Dev d, Tiles tl) {
  const int64_t k = xcd_block() * kBlock + threadIdx.x;
  if (k < tl.nsv) shared_sum2<R>(k, d, tl);
}

__global__ __launch_bounds__(kBlock) void k_euler_apply(Dev d, int fp32) {
  const int64_t v = xcd_block() * kBlock + threadIdx.x;
  if (v < d.nv) euler_apply(v, d, fp32 != 0);
}

size_t tile_lds_bytes(const Tiles& tl, int fp32, int stage, bool cfl) {
  return fp32 ? tile_lds<float>(tl, stage, cfl, nullptr, nullptr)
              : tile_lds<double>(tl, stage, cfl, nullptr, nullptr);
}

template <typename R, int SCHEME>
static hipError_t tile_go(const Dev& d, const Tiles& tl, int stage, bool save, bool cfl, hipStream_t s) {
  const dim3 g(tl.ntiles), b(tile_threads(tl, stage));
  const size_t lds = tile_lds<R>(tl, stage, cfl, nullptr, nullptr);
  if (stage == 2 && d.slump) hipLaunchKernelGGL((k_tile2<R, SCHEME, true>), g, b, lds, s, d, tl);
  else if (stage == 2) hipLaunchKernelGGL((k_tile2<R, SCHEME, false>), g, b, lds, s, d, tl);
  else if (save && cfl) hipLaunchKernelGGL((k_tile1<R, SCHEME, true, true>), g, b, lds, s, d, tl);
  else if (save) hipLaunchKernelGGL((k_tile1<R, SCHEME, true, false>), g, b, lds, s, d, tl);
  else if (cfl) hipLaunchKernelGGL((k_tile1<R, SCHEME, false, true>), g, b, lds, s, d, tl);
  else hipLaunchKernelGGL((k_tile1<R, SCHEME, false, false>), g, b, lds, s, d, tl);
  return hipGetLastError();
}

template <typename R>
static hipError_t tile_scheme(const Dev& d, const Tiles& tl, int scheme, int stage, bool save, bool cfl,
                              hipStream_t s) {
  switch (scheme) {
    case SCH_N: return tile_go<R, SCH_N>(d, tl, stage, save, cfl, s);
    case SCH_LDA: return tile_go<R, SCH_LDA>(d, tl, stage, save, cfl, s);
    case SCH_B: return tile_go<R, SCH_B>(d, tl, stage, save, cfl, s);
    case SCH_BMAX: return tile_go<R, SCH_BMAX>(d, tl, stage, save, cfl, s);
    case SCH_BMIN: return tile_go<R, SCH_BMIN>(d, tl, stage, save, cfl, s);
    case SCH_BX: return tile_go<R, SCH_BX>(d, tl, stage, save, cfl, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_tile(const Dev& d, const Tiles& tl, int fp32, int scheme, int stage, bool save, bool cfl,
                       hipStream_t s) {
  if (tl.ntiles == 0) return hipSuccess;
  if (tl.tt < 1) return hipErrorInvalidValue;
  return fp32 ? tile_scheme<float>(d, tl, scheme, stage, save, cfl, s)
              : tile_scheme<double>(d, tl, scheme, stage, save, cfl, s);
}

hipError_t launch_shared(const Dev& d, const Tiles& tl, int fp32, int stage, bool cfl, hipStream_t s) {
  if (tl.nsv == 0) return hipSuccess;
  const dim3 g(nblk(tl.nsv)), b(kBlock);
  if (stage == 2) {
    if (fp32) hipLaunchKernelGGL((k_shared2<float>), g, b, 0, s, d, tl);
    else hipLaunchKernelGGL((k_shared2<double>), g, b, 0, s, d, tl);
  } else if (cfl) {
    if (fp32) hipLaunchKernelGGL((k_shared1<float, true>), g, b, 0, s, d, tl);
    else hipLaunchKernelGGL((k_shared1<double, true>), g, b, 0, s, d, tl);
  } else {
    if (fp32) hipLaunchKernelGGL((k_shared1<float, false>), g, b, 0, s, d, tl);
    else hipLaunchKernelGGL((k_shared1<double, false>), g, b, 0, s, d, tl);
  }
  return hipGetLastError();
}

hipError_t launch_euler_apply(const Dev& d, int fp32, hipStream_t s) {
  if (d.nv == 0) return hipSuccess;
  hipLaunchKernelGGL(k_euler_apply, dim3(nblk(d.nv)), dim3(kBlock), 0, s, d, fp32);
  return hipGetLastError();
}

}  // namespace rd
