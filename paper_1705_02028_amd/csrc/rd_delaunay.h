// Delaunay edge flipping on the GPU: device view of a triangulation and the
// launchers of one flip round's passes (kernels in rd_delaunay.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rd {
namespace dl {

struct Mesh {
  int64_t nt = 0;
  const double* x = nullptr;
  const double* y = nullptr;
  double px = 0.0, py = 0.0;
  int32_t* tri = nullptr;      // [3][nt] corner vertices, counter-clockwise
  int32_t* nbr = nullptr;      // [3][nt] triangle across the edge opposite corner i, -1 on the boundary
  int32_t* claim = nullptr;    // [nt] lowest key of an illegal edge of t this round
  int32_t* cand = nullptr;     // [nt] bit i: the edge opposite corner i of t (t the lower triangle) is illegal
  int32_t* flipped = nullptr;  // [nt] round of t's last flip (0: never)
  int32_t* partner = nullptr;  // [nt] the other triangle of t's last flip
  int32_t* count = nullptr;    // [0] flips, [1] illegal edges, [2] undecided edges
  int64_t* undecided = nullptr;  // keys 3 t + i of the edges the FP64 test could not decide
  double* work = nullptr;        // exact-evaluation scratch, kIncircleScratch doubles per thread
};

// Scratch doubles per thread of the exact in-circle pass.
int64_t exact_scratch();

// One round: reset the claims; test every interior edge in FP64 (undecided
// ones go to m.undecided); test undecided edges [first, last) exactly; flip
// the edges that hold both claims; repoint neighbours at flipped pairs.
hipError_t launch_reset(const Mesh& m, hipStream_t s);
hipError_t launch_mark(const Mesh& m, hipStream_t s);
hipError_t launch_exact(const Mesh& m, int64_t first, int64_t last, hipStream_t s);
hipError_t launch_flip(const Mesh& m, int32_t round, hipStream_t s);
hipError_t launch_fix(const Mesh& m, int32_t round, hipStream_t s);

}  // namespace dl
}  // namespace rd
