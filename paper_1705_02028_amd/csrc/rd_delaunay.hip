// Mesh generation on the GPU (Section 2, Delaunay refinement with exact
// predicates; Section 4.1, its parallel form): one thread per element for
// every pass; the per-element bodies are in rd_delaunay_kern.h.
//
// Flips: rounds of independent flips. Each round: every interior edge that
// may be illegal (one of its triangles changed since the edge last passed)
// is tested once, by its lower-numbered triangle (in-circle test: FP64 with an
// error bound, exact expansion arithmetic for the undecided ones, in a
// separate pass over a compacted list); every illegal edge claims both its
// triangles with an integer atomic minimum of its key (3 t + i), so the
// lowest key wins each triangle and the result does not depend on
// scheduling; an edge flips when it holds both claims; then every triangle
// points its neighbour entries at whichever of a flipped pair now holds the
// shared edge. The lowest illegal edge always holds both claims, so each
// round flips at least one edge, and Lawson's argument bounds the total
// number of flips. An illegal edge (its fourth vertex strictly inside the
// circle) always has a strictly convex quadrilateral, so a flip never
// inverts a triangle.
//
// Refinement iteration: every triangle tests itself (size, quality,
// encroached boundary edge); each candidate point is located by a walk and
// tested for encroachment; each candidate locks its cavity with its priority
// (atomic maximum), and the candidates that hold their whole cavity are
// inserted together; prefix sums number the new vertices and triangles, so
// the result does not depend on scheduling. Optionally the vertices and
// triangles are then renumbered in Morton order (a stable radix sort).
#include <hipcub/hipcub.hpp>

#include "rd_delaunay.h"

namespace rd {
namespace dl {

constexpr int kBlock = 256;

__global__ __launch_bounds__(kBlock) void k_reset(Mesh m) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  reset_body(m, t);
}

__global__ __launch_bounds__(kBlock) void k_mark(Mesh m, int32_t pass) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int r = t < m.nt ? mark_body(m, t, pass) : 0;
  for (int i = 0; i < 3; ++i) {
    wave_add(&m.count[1], (r >> i) & 1);
    const int k = wave_add(&m.count[2], (r >> (4 + i)) & 1);
    if ((r >> (4 + i)) & 1) m.undecided[k] = 3 * t + i;
  }
}

__global__ __launch_bounds__(kBlock) void k_exact(Mesh m, int64_t first, int64_t last) {
  const int64_t k = first + (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool illegal = k < last && exact_body(m, k, m.work + (k - first) * pred::kIncircleScratch);
  wave_add(&m.count[1], illegal);
}

__global__ __launch_bounds__(kBlock) void k_flip(Mesh m, int32_t round, int32_t pass) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  wave_add(&m.count[0], t < m.nt && flip_body(m, t, round, pass));
}

__global__ __launch_bounds__(kBlock) void k_fix(Mesh m, int32_t round) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t < m.nt) fix_body(m, t, round);
}

__global__ __launch_bounds__(kBlock) void k_quality(Mesh m, Refine r) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int q = t < m.nt ? quality_body(m, r, t) : kNone;
  wave_add(&r.count[0], q == kCandidate);
  wave_add(&r.count[1], q == kTooFar);
}

__global__ __launch_bounds__(kBlock) void k_locate(Mesh m, Refine r) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t < m.nt) locate_body(m, r, t);
}

__global__ __launch_bounds__(kBlock) void k_lock(Mesh m, Refine r) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t < m.nt) lock_body(m, r, t);
}

__global__ __launch_bounds__(kBlock) void k_check(Mesh m, Refine r) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t < m.nt) check_body(m, r, t);
}

__global__ __launch_bounds__(kBlock) void k_insert(Mesh m, Refine r, int32_t it, int32_t pass) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t < m.nt) insert_body(m, r, t, it, pass);
}

__global__ __launch_bounds__(kBlock) void k_fixsplit(Mesh m, Refine r, int32_t it) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t < m.nt) fixsplit_body(m, r, t, it);
}

__global__ __launch_bounds__(kBlock) void k_vkeys(Mesh m, Order o, int64_t nv) {
  const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (v < nv) vkey_body(m, o, v);
}

__global__ __launch_bounds__(kBlock) void k_tkeys(Mesh m, Order o) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t < m.nt) tkey_body(m, o, t);
}

__global__ __launch_bounds__(kBlock) void k_invert(Order o, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) invert_body(o, i);
}

__global__ __launch_bounds__(kBlock) void k_vapply(Mesh m, Order o, int64_t nv) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < nv) vapply_body(m, o, i);
}

__global__ __launch_bounds__(kBlock) void k_vrename(Mesh m, Order o) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t < m.nt) vrename_body(m, o, t);
}

__global__ __launch_bounds__(kBlock) void k_tapply(Mesh m, Order o) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < m.nt) tapply_body(m, o, i);
}

static unsigned nblocks(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

int64_t exact_scratch() { return pred::kIncircleScratch; }

hipError_t launch_reset(const Mesh& m, hipStream_t s) {
  hipLaunchKernelGGL(k_reset, dim3(nblocks(m.nt > 3 ? m.nt : 3)), dim3(kBlock), 0, s, m);
  return hipGetLastError();
}
hipError_t launch_mark(const Mesh& m, int32_t pass, hipStream_t s) {
  hipLaunchKernelGGL(k_mark, dim3(nblocks(m.nt)), dim3(kBlock), 0, s, m, pass);
  return hipGetLastError();
}
hipError_t launch_exact(const Mesh& m, int64_t first, int64_t last, hipStream_t s) {
  if (last <= first) return hipSuccess;
  hipLaunchKernelGGL(k_exact, dim3(nblocks(last - first)), dim3(kBlock), 0, s, m, first, last);
  return hipGetLastError();
}
hipError_t launch_flip(const Mesh& m, int32_t round, int32_t pass, hipStream_t s) {
  hipLaunchKernelGGL(k_flip, dim3(nblocks(m.nt)), dim3(kBlock), 0, s, m, round, pass);
  return hipGetLastError();
}
hipError_t launch_fix(const Mesh& m, int32_t round, hipStream_t s) {
  hipLaunchKernelGGL(k_fix, dim3(nblocks(m.nt)), dim3(kBlock), 0, s, m, round);
  return hipGetLastError();
}

hipError_t launch_quality(const Mesh& m, const Refine& r, hipStream_t s) {
  hipLaunchKernelGGL(k_quality, dim3(nblocks(m.nt)), dim3(kBlock), 0, s, m, r);
  return hipGetLastError();
}
hipError_t launch_locate(const Mesh& m, const Refine& r, hipStream_t s) {
  hipLaunchKernelGGL(k_locate, dim3(nblocks(m.nt)), dim3(kBlock), 0, s, m, r);
  return hipGetLastError();
}
hipError_t launch_lock(const Mesh& m, const Refine& r, hipStream_t s) {
  hipLaunchKernelGGL(k_lock, dim3(nblocks(m.nt)), dim3(kBlock), 0, s, m, r);
  return hipGetLastError();
}
hipError_t launch_check(const Mesh& m, const Refine& r, hipStream_t s) {
  hipLaunchKernelGGL(k_check, dim3(nblocks(m.nt)), dim3(kBlock), 0, s, m, r);
  return hipGetLastError();
}
hipError_t launch_insert(const Mesh& m, const Refine& r, int32_t it, int32_t pass, hipStream_t s) {
  hipLaunchKernelGGL(k_insert, dim3(nblocks(m.nt)), dim3(kBlock), 0, s, m, r, it, pass);
  return hipGetLastError();
}
hipError_t launch_fixsplit(const Mesh& m, const Refine& r, int32_t it, int64_t nt_after, hipStream_t s) {
  Mesh a = m;
  a.nt = nt_after;
  hipLaunchKernelGGL(k_fixsplit, dim3(nblocks(nt_after)), dim3(kBlock), 0, s, a, r, it);
  return hipGetLastError();
}

hipError_t launch_vkeys(const Mesh& m, const Order& o, int64_t nv, hipStream_t s) {
  hipLaunchKernelGGL(k_vkeys, dim3(nblocks(nv)), dim3(kBlock), 0, s, m, o, nv);
  return hipGetLastError();
}
hipError_t launch_tkeys(const Mesh& m, const Order& o, hipStream_t s) {
  hipLaunchKernelGGL(k_tkeys, dim3(nblocks(m.nt)), dim3(kBlock), 0, s, m, o);
  return hipGetLastError();
}
size_t sort_tmp_bytes(int64_t n) {
  size_t bytes = 0;
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                           (const int32_t*)nullptr, (int32_t*)nullptr, (int)n);
  return bytes;
}
hipError_t launch_sort(const Order& o, int64_t n, void* tmp, size_t tmp_bytes, hipStream_t s) {
  size_t bytes = tmp_bytes;
  return hipcub::DeviceRadixSort::SortPairs(tmp, bytes, o.key, o.skey, o.idx, o.perm, (int)n, 0, 32, s);
}
hipError_t launch_invert(const Order& o, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_invert, dim3(nblocks(n)), dim3(kBlock), 0, s, o, n);
  return hipGetLastError();
}
hipError_t launch_vapply(const Mesh& m, const Order& o, int64_t nv, hipStream_t s) {
  hipLaunchKernelGGL(k_vapply, dim3(nblocks(nv)), dim3(kBlock), 0, s, m, o, nv);
  return hipGetLastError();
}
hipError_t launch_vrename(const Mesh& m, const Order& o, hipStream_t s) {
  hipLaunchKernelGGL(k_vrename, dim3(nblocks(m.nt)), dim3(kBlock), 0, s, m, o);
  return hipGetLastError();
}
hipError_t launch_tapply(const Mesh& m, const Order& o, hipStream_t s) {
  hipLaunchKernelGGL(k_tapply, dim3(nblocks(m.nt)), dim3(kBlock), 0, s, m, o);
  return hipGetLastError();
}

size_t scan_tmp_bytes(int64_t n) {
  size_t bytes = 0;
  (void)hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, (const int32_t*)nullptr, (int32_t*)nullptr, (int)n);
  return bytes;
}

hipError_t launch_scan(const int32_t* src, int32_t* dst, int64_t n, void* tmp, size_t tmp_bytes, hipStream_t s) {
  size_t bytes = tmp_bytes;
  return hipcub::DeviceScan::ExclusiveSum(tmp, bytes, src, dst, (int)n, s);
}

}  // namespace dl
}  // namespace rd
