// Device helpers shared by the kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include "rd_launch.h"

namespace rd {

// Consecutive workgroup ids are dispatched round-robin over the 8 XCDs of an
// MI355X, each with its own L2. This renumbering gives each XCD one
// contiguous range of workgroups (triangles, tiles or vertices), which keeps
// the vertex data a range touches in that XCD's L2.
__device__ __forceinline__ int64_t xcd_block() {
  const int64_t b = blockIdx.x, nb = gridDim.x;
  const int64_t x = b % 8, q = nb / 8, r = nb % 8;
  return x * q + (x < r ? x : r) + b / 8;
}

// Minimum waves per SIMD the triangle kernels are compiled for: 4 for FP32;
// for FP64, 3 where the kernel fits 168 VGPRs (every stage-1 kernel but the
// N one with both outputs, and the N and LDA stage-2 kernels; the N stage-2
// one and the LDA one with selective lumping spill one or two registers),
// else 2. (Parking the corner coefficients in LDS across the solve to fit 3
// waves was measured slower than 2 waves without it.)
template <typename R> struct TriWaves { static constexpr int value = 2; };
template <> struct TriWaves<float> { static constexpr int value = 4; };
template <typename R, int SCHEME, int STAGE, bool SAVE, bool CFL>
struct TriKernelWaves {
  static constexpr bool three = sizeof(R) == sizeof(double) &&
                                (STAGE == 1 ? !(SCHEME == SCH_N && SAVE && CFL) : SCHEME <= SCH_LDA);
  static constexpr int value = three ? 3 : TriWaves<R>::value;
  // fast FP64 reciprocals (rcp), except in the three-wave instances whose
  // schedule would then spill (stage 2, and the Bx stage 1 with its sensor)
  static constexpr bool fast_div = !(three && (STAGE == 2 || SCHEME == SCH_BX));
};

// Minimum over a kBlock-thread workgroup (result valid in every thread).
__device__ __forceinline__ double block_min(double x) {
  __shared__ double red[kBlock];
  red[threadIdx.x] = x;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = rmin(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  return red[0];
}

static inline unsigned nblk(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace rd
