// Delaunay edge flipping on the GPU (Section 2: the last step of every
// refinement iteration makes the triangulation Delaunay again by flipping
// edges whose opposite vertex lies inside the circumcircle, with exact
// predicates).
//
// Rounds of independent flips. Each round: every interior edge is tested
// once, by its lower-numbered triangle (in-circle test: FP64 with an error
// bound, exact expansion arithmetic for the undecided ones, in a separate
// pass over a compacted list); every illegal edge claims both its triangles
// with an integer atomic minimum of its key (3 t + i), so the lowest key
// wins each triangle and the result does not depend on scheduling; an edge
// flips when it holds both claims; then every triangle points its neighbour
// entries at whichever of a flipped pair now holds the shared edge. The
// lowest illegal edge always holds both claims, so each round flips at
// least one edge, and Lawson's argument bounds the total number of flips.
// An illegal edge (its fourth vertex strictly inside the circle) always has
// a strictly convex quadrilateral, so a flip never inverts a triangle.
#include "rd_delaunay.h"

#include <climits>

#include "rd_predicates.h"

namespace rd {
namespace dl {

constexpr int kBlock = 256;

__device__ __forceinline__ double unwrap_d(double d, double period) {
  if (period > 0.0) {
    if (d > 0.5 * period) d -= period;
    else if (d < -0.5 * period) d += period;
  }
  return d;
}

// The quadrilateral of edge i of t: a = corner i, (b, c) the edge, d the
// vertex of the neighbour u opposite it; coordinates unwrapped next to a.
struct Quad {
  double a[2], b[2], c[2], d[2];
  int32_t u, j;  // neighbour and its corner at d
};

__device__ inline Quad quad(const Mesh& m, int64_t t, int i) {
  const int64_t nt = m.nt;
  Quad q;
  const int32_t va = m.tri[i * nt + t], vb = m.tri[((i + 1) % 3) * nt + t], vc = m.tri[((i + 2) % 3) * nt + t];
  q.u = m.nbr[i * nt + t];
  q.j = 0;
  for (int k = 0; k < 3; ++k) {
    const int32_t w = m.tri[k * nt + q.u];
    if (w != vb && w != vc) q.j = k;
  }
  const int32_t vd = m.tri[q.j * nt + q.u];
  const double ax = m.x[va], ay = m.y[va];
  const int32_t ids[3] = {vb, vc, vd};
  double* dst[3] = {q.b, q.c, q.d};
  q.a[0] = ax;
  q.a[1] = ay;
  for (int k = 0; k < 3; ++k) {
    dst[k][0] = ax + unwrap_d(m.x[ids[k]] - ax, m.px);
    dst[k][1] = ay + unwrap_d(m.y[ids[k]] - ay, m.py);
  }
  return q;
}

__device__ inline void mark_illegal(const Mesh& m, int64_t t, int i, int32_t u) {
  const int32_t key = (int32_t)(3 * t + i);
  atomicOr(&m.cand[t], 1 << i);
  atomicMin(&m.claim[t], key);
  atomicMin(&m.claim[u], key);
  atomicAdd(&m.count[1], 1);
}

// FP64 in-circle test of every interior edge, once per edge.
__global__ __launch_bounds__(kBlock) void k_mark(Mesh m) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= m.nt) return;
  for (int i = 0; i < 3; ++i) {
    const int32_t u = m.nbr[i * m.nt + t];
    if (u <= t) continue;  // boundary, or tested by u
    const Quad q = quad(m, t, i);
    const int r = pred::incircle_filter(q.a, q.b, q.c, q.d);
    if (r > 0) {
      mark_illegal(m, t, i, u);
    } else if (r == 0) {
      const int32_t k = atomicAdd(&m.count[2], 1);
      m.undecided[k] = 3 * t + i;
    }
  }
}

// Exact in-circle test of the undecided edges [first, last).
__global__ __launch_bounds__(kBlock) void k_exact(Mesh m, int64_t first, int64_t last) {
  const int64_t k = first + (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= last) return;
  const int64_t key = m.undecided[k];
  const int64_t t = key / 3;
  const int i = (int)(key % 3);
  const Quad q = quad(m, t, i);
  double* w = m.work + (k - first) * pred::kIncircleScratch;
  if (pred::incircle_exact(q.a, q.b, q.c, q.d, w) > 0) mark_illegal(m, t, i, q.u);
}

// Flip every illegal edge that holds the claims of both its triangles.
__global__ __launch_bounds__(kBlock) void k_flip(Mesh m, int32_t round) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= m.nt) return;
  const int32_t bits = m.cand[t];
  if (!bits) return;
  const int64_t nt = m.nt;
  for (int i = 0; i < 3; ++i) {
    if (!(bits & (1 << i))) continue;
    const int32_t key = (int32_t)(3 * t + i);
    if (m.claim[t] != key) continue;  // t flips with a lower key, or not at all
    const int32_t u = m.nbr[i * nt + t];
    if (m.claim[u] != key) continue;
    // t = (a, b, c) with the edge (b, c) opposite a; u holds (c, b) and d
    const int32_t a = m.tri[i * nt + t], b = m.tri[((i + 1) % 3) * nt + t], c = m.tri[((i + 2) % 3) * nt + t];
    int j = 0;
    for (int k = 0; k < 3; ++k) {
      const int32_t w = m.tri[k * nt + u];
      if (w != b && w != c) j = k;
    }
    const int32_t d = m.tri[j * nt + u];
    // outer neighbours: across (a, b) and (c, a) in t; across (b, d) and (d, c) in u
    const int32_t n_ab = m.nbr[((i + 2) % 3) * nt + t], n_ca = m.nbr[((i + 1) % 3) * nt + t];
    int32_t n_bd = -1, n_dc = -1;
    for (int k = 0; k < 3; ++k) {
      const int32_t opp = m.tri[k * nt + u];
      if (opp == c) n_bd = m.nbr[k * nt + u];
      if (opp == b) n_dc = m.nbr[k * nt + u];
    }
    // t becomes (a, b, d), u becomes (d, c, a); neighbour i is across the edge opposite corner i
    m.tri[0 * nt + t] = a;
    m.tri[1 * nt + t] = b;
    m.tri[2 * nt + t] = d;
    m.nbr[0 * nt + t] = n_bd;
    m.nbr[1 * nt + t] = u;
    m.nbr[2 * nt + t] = n_ab;
    m.tri[0 * nt + u] = d;
    m.tri[1 * nt + u] = c;
    m.tri[2 * nt + u] = a;
    m.nbr[0 * nt + u] = n_ca;
    m.nbr[1 * nt + u] = t;
    m.nbr[2 * nt + u] = n_dc;
    m.flipped[t] = round;
    m.flipped[u] = round;
    m.partner[t] = u;
    m.partner[u] = t;
    atomicAdd(&m.count[0], 1);
    return;
  }
}

// Neighbour entries that point at a triangle flipped this round now point at
// whichever of the flipped pair holds the shared edge.
__global__ __launch_bounds__(kBlock) void k_fix(Mesh m, int32_t round) {
  const int64_t w = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (w >= m.nt) return;
  const int64_t nt = m.nt;
  for (int k = 0; k < 3; ++k) {
    const int32_t x = m.nbr[k * nt + w];
    if (x < 0 || m.flipped[x] != round) continue;
    const int32_t p = m.tri[((k + 1) % 3) * nt + w], q = m.tri[((k + 2) % 3) * nt + w];
    int has = 0;
    for (int r = 0; r < 3; ++r) {
      const int32_t v = m.tri[r * nt + x];
      has += (v == p) + (v == q);
    }
    m.nbr[k * nt + w] = has == 2 ? x : m.partner[x];
  }
}

__global__ __launch_bounds__(kBlock) void k_reset(Mesh m) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t < m.nt) {
    m.claim[t] = INT_MAX;
    m.cand[t] = 0;
  }
  if (t < 3) m.count[t] = 0;
}

static unsigned nblocks(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

int64_t exact_scratch() { return pred::kIncircleScratch; }

hipError_t launch_reset(const Mesh& m, hipStream_t s) {
  hipLaunchKernelGGL(k_reset, dim3(nblocks(m.nt)), dim3(kBlock), 0, s, m);
  return hipGetLastError();
}
hipError_t launch_mark(const Mesh& m, hipStream_t s) {
  hipLaunchKernelGGL(k_mark, dim3(nblocks(m.nt)), dim3(kBlock), 0, s, m);
  return hipGetLastError();
}
hipError_t launch_exact(const Mesh& m, int64_t first, int64_t last, hipStream_t s) {
  if (last <= first) return hipSuccess;
  hipLaunchKernelGGL(k_exact, dim3(nblocks(last - first)), dim3(kBlock), 0, s, m, first, last);
  return hipGetLastError();
}
hipError_t launch_flip(const Mesh& m, int32_t round, hipStream_t s) {
  hipLaunchKernelGGL(k_flip, dim3(nblocks(m.nt)), dim3(kBlock), 0, s, m, round);
  return hipGetLastError();
}
hipError_t launch_fix(const Mesh& m, int32_t round, hipStream_t s) {
  hipLaunchKernelGGL(k_fix, dim3(nblocks(m.nt)), dim3(kBlock), 0, s, m, round);
  return hipGetLastError();
}

}  // namespace dl
}  // namespace rd
