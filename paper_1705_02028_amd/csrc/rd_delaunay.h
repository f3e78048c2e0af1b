// Mesh generation on the GPU: launchers of the flip and refinement passes
// (kernels in rd_delaunay.hip, per-element bodies in rd_delaunay_kern.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "rd_delaunay_kern.h"

namespace rd {
namespace dl {

// Scratch doubles per thread of the exact in-circle pass.
int64_t exact_scratch();

// One flip round: reset the claims; test in FP64 the interior edges of the
// triangles marked for test pass `pass` (undecided ones go to m.undecided);
// test undecided edges [first, last) exactly; flip the edges that hold both
// claims (marking triangles with an illegal edge, and flipped ones, for
// pass + 1); repoint neighbours at flipped pairs.
hipError_t launch_reset(const Mesh& m, hipStream_t s);
hipError_t launch_mark(const Mesh& m, int32_t pass, hipStream_t s);
hipError_t launch_exact(const Mesh& m, int64_t first, int64_t last, hipStream_t s);
hipError_t launch_flip(const Mesh& m, int32_t round, int32_t pass, hipStream_t s);
hipError_t launch_fix(const Mesh& m, int32_t round, hipStream_t s);

// One refinement iteration over the m.nt triangles in use: candidates
// (quality and encroachment), their location and encroachment test, cavity
// locks, winners (win, tnew), then, after the host has taken the prefix sums,
// the insertion and the neighbour repair over the nt_after triangles.
hipError_t launch_quality(const Mesh& m, const Refine& r, hipStream_t s);
hipError_t launch_locate(const Mesh& m, const Refine& r, hipStream_t s);
hipError_t launch_lock(const Mesh& m, const Refine& r, hipStream_t s);
hipError_t launch_check(const Mesh& m, const Refine& r, hipStream_t s);
hipError_t launch_insert(const Mesh& m, const Refine& r, int32_t it, int32_t pass, hipStream_t s);
hipError_t launch_fixsplit(const Mesh& m, const Refine& r, int32_t it, int64_t nt_after, hipStream_t s);

// Morton ordering passes: keys of n vertices or triangles (with o.idx =
// 0..n-1), the stable sort of (key, idx) into (skey, perm), the inverse
// permutation, and the moves (into o's buffers; the caller swaps them in).
hipError_t launch_vkeys(const Mesh& m, const Order& o, int64_t nv, hipStream_t s);
hipError_t launch_tkeys(const Mesh& m, const Order& o, hipStream_t s);
size_t sort_tmp_bytes(int64_t n);
hipError_t launch_sort(const Order& o, int64_t n, void* tmp, size_t tmp_bytes, hipStream_t s);
hipError_t launch_invert(const Order& o, int64_t n, hipStream_t s);
hipError_t launch_vapply(const Mesh& m, const Order& o, int64_t nv, hipStream_t s);
hipError_t launch_vrename(const Mesh& m, const Order& o, hipStream_t s);
hipError_t launch_tapply(const Mesh& m, const Order& o, hipStream_t s);

// Exclusive prefix sum of n ints (dst may not alias src); tmp of at least
// scan_tmp_bytes(n) bytes.
size_t scan_tmp_bytes(int64_t n);
hipError_t launch_scan(const int32_t* src, int32_t* dst, int64_t n, void* tmp, size_t tmp_bytes, hipStream_t s);

}  // namespace dl
}  // namespace rd
