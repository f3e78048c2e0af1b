// Per-element bodies of the mesh-generation kernels (Section 2 and its GPU
// form in Section 4.1): Delaunay edge flips and Delaunay refinement.
// rd_delaunay.hip wraps each body in a kernel of one thread per element; a
// host compiler can build the same bodies (the atomics below then act on
// plain memory), so that their logic can be run one element at a time on the
// CPU.
//
// Periodic axes: a vertex is used through its image nearest to a reference
// point (its stored coordinate, or that coordinate plus or minus one period);
// on an axis that is not periodic the stored coordinate itself. Predicates are
// exact on these images. Coordinates are computed without multiply-add contraction,
// so that every build of these bodies gives the same points.
#pragma once

#include <climits>
#include <cstdint>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define DL_FN __device__ inline
#else
#define DL_FN inline
#endif

#include "rd_predicates.h"

namespace rd {
namespace dl {

#if !defined(__HIPCC__)
inline int atomicAdd(int* p, int v) {
  const int o = *p;
  *p = o + v;
  return o;
}
inline int atomicMin(int* p, int v) {
  const int o = *p;
  if (v < o) *p = v;
  return o;
}
inline int atomicOr(int* p, int v) {
  const int o = *p;
  *p = o | v;
  return o;
}
inline unsigned long long atomicMax(unsigned long long* p, unsigned long long v) {
  const unsigned long long o = *p;
  if (v > o) *p = v;
  return o;
}
#endif

// Triangulation in structure-of-arrays form with a fixed row stride (the
// capacity), so that it can grow in place.
struct Mesh {
  int64_t nt = 0;                // triangles in use
  int64_t ts = 0;                // row stride of tri, nbr (>= nt)
  double* x = nullptr;           // vertex coordinates
  double* y = nullptr;
  double px = 0.0, py = 0.0;     // periods (0: not periodic)
  int32_t* tri = nullptr;        // [3][ts] corner vertices, counter-clockwise
  int32_t* nbr = nullptr;        // [3][ts] triangle across the edge opposite corner i, -1 on the boundary
  int32_t* claim = nullptr;      // [ts] lowest key of an illegal edge of t this round
  int32_t* cand = nullptr;       // [ts] bit i: the edge opposite corner i of t (t the lower triangle) is illegal
  int32_t* flipped = nullptr;    // [ts] round of t's last flip (0: never)
  int32_t* partner = nullptr;    // [ts] the other triangle of t's last flip
  int32_t* count = nullptr;      // [0] flips, [1] illegal edges, [2] undecided edges
  int32_t* mark = nullptr;       // [ts] t's edges are tested in every test pass numbered <= mark[t]
  int64_t* undecided = nullptr;  // keys 3 t + i of the edges the FP64 test could not decide
  double* work = nullptr;        // exact-evaluation scratch, kIncircleScratch doubles per thread
};

// Refinement state, one entry per triangle (the candidate of triangle t is
// the point inserted to remove t).
struct Refine {
  int64_t nv = 0;                // vertices in use
  double r2 = 0.0;               // size bound R^2 on the circumradius (0: none)
  double b2 = 0.0;               // quality bound B^2 on (circumradius / shortest edge)^2 (0: none)
  // Size field (Section 2: the size bound may vary in space): R(x) = R s(x)
  // with s bilinear on a gnx x gny grid of node values; a periodic axis has
  // gn nodes at spacing period / gn (wrapping), a bounded one gn nodes from
  // g0 at spacing gd. sgrid null: s = 1.
  const double* sgrid = nullptr;  // [gny][gnx]
  int32_t gnx = 0, gny = 0;
  double gx0 = 0.0, gy0 = 0.0, gdx = 0.0, gdy = 0.0;
  uint32_t seed = 0;             // mixes the iteration into the priorities
  unsigned long long* prio = nullptr;  // [ts] priority of t's candidate (0: none)
  double* px = nullptr;          // [ts] candidate point (stored coordinates)
  double* py = nullptr;
  int32_t* loc = nullptr;        // [ts] triangle the candidate goes into (-1: dropped)
  int32_t* where = nullptr;      // [ts] -1 inside loc, i on its interior edge opposite corner i, 3 + i on its boundary edge
  unsigned long long* lock = nullptr;  // [ts] highest priority whose cavity holds t
  int32_t* win = nullptr;        // [ts] 1: t's candidate is inserted this iteration
  int32_t* wpos = nullptr;       // [ts] exclusive prefix sum of win: new vertex offset
  int32_t* tnew = nullptr;       // [ts] triangles the winner adds (1 on a boundary edge, else 2)
  int32_t* tpos = nullptr;       // [ts] exclusive prefix sum of tnew: new triangle offset
  int32_t* split = nullptr;      // [ts] iteration in which t was last split (0: never)
  int32_t* child = nullptr;      // [2][ts] the triangles t was split into besides itself (-1: none)
  int32_t* count = nullptr;      // [0] candidates, [1] dropped (walk or coincident), [2] dropped (cavity size)
};

constexpr int kCavity = 64;     // triangles a candidate's cavity may hold
constexpr int kWalk = 1 << 20;  // steps of one point location
constexpr int kRing = 256;      // triangles around one vertex

// Counter add aggregated over a wave: every lane of the wave must call it;
// lanes with pred add one each (one atomic per wave); returns this lane's
// slot (the counter's old value plus the number of lower lanes with pred).
#if defined(__HIPCC__)
DL_FN int wave_add(int* counter, bool pred) {
  const unsigned long long mask = __ballot(pred);
  if (!mask) return 0;
  const int lane = __lane_id();
  const int leader = __ffsll((long long)mask) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(counter, __popcll(mask));
  base = __shfl(base, leader);
  return base + __popcll(mask & ((1ull << lane) - 1ull));
}
#else
inline int wave_add(int* counter, bool pred) {
  const int base = *counter;
  if (pred) *counter = base + 1;
  return base;
}
#endif

DL_FN double image(double v, double o, double period) {
  if (period > 0.0) {
    const double d = v - o;
    if (d > 0.5 * period) return v - period;
    if (d < -0.5 * period) return v + period;
  }
  return v;
}

DL_FN double wrap(double v, double period) {
  if (period > 0.0) {
    if (v < 0.0) v += period;
    if (v >= period) v -= period;
  }
  return v;
}

DL_FN int32_t corner(const Mesh& m, int k, int64_t t) { return m.tri[k * m.ts + t]; }
DL_FN int32_t across(const Mesh& m, int k, int64_t t) { return m.nbr[k * m.ts + t]; }

// Image of vertex v nearest to (ox, oy).
DL_FN void vnear(const Mesh& m, int32_t v, double ox, double oy, double* out) {
  out[0] = image(m.x[v], ox, m.px);
  out[1] = image(m.y[v], oy, m.py);
}

// Corners of t as images nearest to o.
DL_FN void tri_near(const Mesh& m, int64_t t, const double* o, double v[3][2]) {
  for (int k = 0; k < 3; ++k) vnear(m, corner(m, k, t), o[0], o[1], v[k]);
}

// ---------------------------------------------------------------------------
// Flips (Section 2, maintaining the Delaunay property; Section 4.1, the
// parallel form): rounds of independent flips.

// The quadrilateral of edge i of t: a = corner i, (b, c) the edge, d the
// vertex of the neighbour u opposite it; images nearest to a.
struct Quad {
  double a[2], b[2], c[2], d[2];
  int32_t u, j;  // neighbour and its corner at d
};

DL_FN Quad quad(const Mesh& m, int64_t t, int i) {
  Quad q;
  const int32_t va = corner(m, i, t), vb = corner(m, (i + 1) % 3, t), vc = corner(m, (i + 2) % 3, t);
  q.u = across(m, i, t);
  q.j = 0;
  for (int k = 0; k < 3; ++k) {
    const int32_t w = corner(m, k, q.u);
    if (w != vb && w != vc) q.j = k;
  }
  const int32_t vd = corner(m, q.j, q.u);
  q.a[0] = m.x[va];
  q.a[1] = m.y[va];
  vnear(m, vb, q.a[0], q.a[1], q.b);
  vnear(m, vc, q.a[0], q.a[1], q.c);
  vnear(m, vd, q.a[0], q.a[1], q.d);
  return q;
}

// Edge i of t is illegal: claim both triangles with its key (flip_body then
// marks t for the next test pass).
DL_FN void mark_illegal(const Mesh& m, int64_t t, int i, int32_t u) {
  const int32_t key = (int32_t)(3 * t + i);
  atomicOr(&m.cand[t], 1 << i);
  atomicMin(&m.claim[t], key);
  atomicMin(&m.claim[u], key);
}

DL_FN void reset_body(const Mesh& m, int64_t t) {
  if (t < m.nt) {
    m.claim[t] = INT_MAX;
    m.cand[t] = 0;
  }
  if (t < 3) m.count[t] = 0;
}

// FP64 in-circle test of the interior edges of t that t tests (t the lower
// triangle of the edge) in test pass `pass`: those with t or its neighbour
// marked for this pass (every other edge is known to be legal: its two
// triangles are unchanged since it last passed). Returns the illegal edges
// (bits 0-2) and the undecided ones, for the exact pass (bits 4-6). Marks
// are only read here (flip_body writes them), so what a pass tests does not
// depend on timing.
DL_FN int mark_body(const Mesh& m, int64_t t, int32_t pass) {
  int out = 0;
  const bool mine = m.mark[t] >= pass;
  for (int i = 0; i < 3; ++i) {
    const int32_t u = across(m, i, t);
    if (u <= t) continue;  // boundary, or tested by u
    if (!mine && m.mark[u] < pass) continue;
    const Quad q = quad(m, t, i);
    const int r = pred::incircle_filter(q.a, q.b, q.c, q.d);
    if (r > 0) {
      mark_illegal(m, t, i, u);
      out |= 1 << i;
    } else if (r == 0) {
      out |= 16 << i;
    }
  }
  return out;
}

// Exact in-circle test of undecided edge k; w: kIncircleScratch doubles.
// Returns whether the edge is illegal.
DL_FN bool exact_body(const Mesh& m, int64_t k, double* w) {
  const int64_t key = m.undecided[k];
  const int64_t t = key / 3;
  const int i = (int)(key % 3);
  const Quad q = quad(m, t, i);
  if (pred::incircle_exact(q.a, q.b, q.c, q.d, w) <= 0) return false;
  mark_illegal(m, t, i, q.u);
  return true;
}

// Flip the illegal edge of t that holds the claims of both its triangles;
// returns whether it flipped. A triangle with an illegal edge, and both
// triangles of a flip, are marked for the next test pass.
DL_FN bool flip_body(const Mesh& m, int64_t t, int32_t round, int32_t pass) {
  const int32_t bits = m.cand[t];
  if (!bits) return false;
  m.mark[t] = pass + 1;
  const int64_t ts = m.ts;
  for (int i = 0; i < 3; ++i) {
    if (!(bits & (1 << i))) continue;
    const int32_t key = (int32_t)(3 * t + i);
    if (m.claim[t] != key) continue;  // t flips with a lower key, or not at all
    const int32_t u = across(m, i, t);
    if (m.claim[u] != key) continue;
    // t = (a, b, c) with the edge (b, c) opposite a; u holds (c, b) and d
    const int32_t a = corner(m, i, t), b = corner(m, (i + 1) % 3, t), c = corner(m, (i + 2) % 3, t);
    int j = 0;
    for (int k = 0; k < 3; ++k) {
      const int32_t w = corner(m, k, u);
      if (w != b && w != c) j = k;
    }
    const int32_t d = corner(m, j, u);
    // outer neighbours: across (a, b) and (c, a) in t; across (b, d) and (d, c) in u
    const int32_t n_ab = across(m, (i + 2) % 3, t), n_ca = across(m, (i + 1) % 3, t);
    int32_t n_bd = -1, n_dc = -1;
    for (int k = 0; k < 3; ++k) {
      const int32_t opp = corner(m, k, u);
      if (opp == c) n_bd = across(m, k, u);
      if (opp == b) n_dc = across(m, k, u);
    }
    // t becomes (a, b, d), u becomes (d, c, a)
    m.tri[0 * ts + t] = a;
    m.tri[1 * ts + t] = b;
    m.tri[2 * ts + t] = d;
    m.nbr[0 * ts + t] = n_bd;
    m.nbr[1 * ts + t] = u;
    m.nbr[2 * ts + t] = n_ab;
    m.tri[0 * ts + u] = d;
    m.tri[1 * ts + u] = c;
    m.tri[2 * ts + u] = a;
    m.nbr[0 * ts + u] = n_ca;
    m.nbr[1 * ts + u] = t;
    m.nbr[2 * ts + u] = n_dc;
    m.flipped[t] = round;
    m.flipped[u] = round;
    m.partner[t] = u;
    m.partner[u] = t;
    m.mark[t] = pass + 1;
    m.mark[u] = pass + 1;
    return true;
  }
  return false;
}

// Neighbour entries of w that point at a triangle flipped this round now
// point at whichever of the flipped pair holds the shared edge.
DL_FN void fix_body(const Mesh& m, int64_t w, int32_t round) {
  for (int k = 0; k < 3; ++k) {
    const int32_t x = across(m, k, w);
    if (x < 0 || m.flipped[x] != round) continue;
    const int32_t p = corner(m, (k + 1) % 3, w), q = corner(m, (k + 2) % 3, w);
    int has = 0;
    for (int r = 0; r < 3; ++r) {
      const int32_t v = corner(m, r, x);
      has += (v == p) + (v == q);
    }
    m.nbr[k * m.ts + w] = has == 2 ? x : m.partner[x];
  }
}

// ---------------------------------------------------------------------------
// Refinement (Section 2, one iteration; Section 4.1, parallel insertion set).

// Candidate priorities: unique per triangle, pseudo-random across the mesh
// (the high word is the 32-bit finaliser of MurmurHash3 applied to the
// triangle index and the iteration's seed; the low word the index + 1).
DL_FN uint32_t mix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

DL_FN unsigned long long priority(int64_t t, uint32_t seed) {
  return ((unsigned long long)mix32((uint32_t)t ^ seed) << 32) | (unsigned long long)(t + 1);
}

DL_FN void candidate_reset(const Refine& r, int64_t t) {
  r.prio[t] = 0;
  r.loc[t] = -1;
  r.where[t] = -1;
  r.lock[t] = 0;
  r.win[t] = 0;
  r.tnew[t] = 0;
}

// One axis of the size grid: node index i0, its neighbour i1 and the weight
// of i1 for coordinate v.
DL_FN void grid_axis(double v, double v0, double dv, int32_t n, double period, int32_t& i0, int32_t& i1, double& w) {
#pragma clang fp contract(off)
  double q = (v - v0) / dv;
  if (period > 0.0) {
    double fl = floor(q);
    w = q - fl;
    int64_t k = (int64_t)fl % n;
    if (k < 0) k += n;
    i0 = (int32_t)k;
    i1 = (int32_t)((k + 1) % n);
    return;
  }
  if (q < 0.0) q = 0.0;
  if (q > (double)(n - 1)) q = (double)(n - 1);
  double fl = floor(q);
  if (fl > (double)(n - 2)) fl = (double)(n - 2);
  if (fl < 0.0) fl = 0.0;
  i0 = (int32_t)fl;
  i1 = n > 1 ? i0 + 1 : i0;
  w = n > 1 ? q - fl : 0.0;
}

// s(x, y) of the size field (1 without a grid).
DL_FN double size_scale(const Mesh& m, const Refine& r, double x, double y) {
#pragma clang fp contract(off)
  if (!r.sgrid) return 1.0;
  int32_t x0, x1, y0, y1;
  double wx, wy;
  grid_axis(x, r.gx0, r.gdx, r.gnx, m.px, x0, x1, wx);
  grid_axis(y, r.gy0, r.gdy, r.gny, m.py, y0, y1, wy);
  const double a = r.sgrid[y0 * r.gnx + x0] * (1.0 - wx) + r.sgrid[y0 * r.gnx + x1] * wx;
  const double b = r.sgrid[y1 * r.gnx + x0] * (1.0 - wx) + r.sgrid[y1 * r.gnx + x1] * wx;
  return a * (1.0 - wy) + b * wy;
}

// Result of quality_body.
constexpr int kNone = 0, kCandidate = 1, kTooFar = 2;

// Does t need a new vertex: a boundary edge it encroaches (its opposite
// corner inside the edge's diametric circle: the edge is split at its
// midpoint), or a circumradius r > R s(centroid), or r / (shortest edge) > B
// (a vertex at the circumcentre). The circumradius is l_a l_b l_c / (2 |det|) with det the
// orientation determinant.
DL_FN int quality_body(const Mesh& m, const Refine& r, int64_t t) {
#pragma clang fp contract(off)
  candidate_reset(r, t);
  double v[3][2];
  const double o[2] = {m.x[corner(m, 0, t)], m.y[corner(m, 0, t)]};
  tri_near(m, t, o, v);
  for (int i = 0; i < 3; ++i) {
    if (across(m, i, t) >= 0) continue;
    const double* a = v[i];
    const double* b = v[(i + 1) % 3];
    const double* c = v[(i + 2) % 3];
    if ((b[0] - a[0]) * (c[0] - a[0]) + (b[1] - a[1]) * (c[1] - a[1]) < 0.0) {
      r.px[t] = wrap(0.5 * (b[0] + c[0]), m.px);
      r.py[t] = wrap(0.5 * (b[1] + c[1]), m.py);
      r.loc[t] = (int32_t)t;
      r.where[t] = 3 + i;
      r.prio[t] = priority(t, r.seed);
      return kCandidate;
    }
  }
  const double bx = v[1][0] - v[0][0], by = v[1][1] - v[0][1];
  const double cx = v[2][0] - v[0][0], cy = v[2][1] - v[0][1];
  const double ex = v[2][0] - v[1][0], ey = v[2][1] - v[1][1];
  const double lb2 = cx * cx + cy * cy, lc2 = bx * bx + by * by, la2 = ex * ex + ey * ey;
  const double det = bx * cy - by * cx;  // equal to the orientation determinant of (a, b, c)
  const double rad2 = la2 * lb2 * lc2 / (4.0 * det * det);
  double lmin2 = la2 < lb2 ? la2 : lb2;
  lmin2 = lmin2 < lc2 ? lmin2 : lc2;
  double rb2 = r.r2;
  if (r.sgrid && rb2 > 0.0) {  // the size field at the centroid
    const double sc = size_scale(m, r, wrap((v[0][0] + v[1][0] + v[2][0]) / 3.0, m.px),
                                 wrap((v[0][1] + v[1][1] + v[2][1]) / 3.0, m.py));
    rb2 = rb2 * (sc * sc);
  }
  const bool bad = (rb2 > 0.0 && rad2 > rb2) || (r.b2 > 0.0 && rad2 > r.b2 * lmin2);
  if (!bad) return kNone;
  // circumcentre, relative to corner 0
  const double ux = (cy * lc2 - by * lb2) / (2.0 * det);
  const double uy = (bx * lb2 - cx * lc2) / (2.0 * det);
  if ((m.px > 0.0 && fabs(ux) > 0.25 * m.px) || (m.py > 0.0 && fabs(uy) > 0.25 * m.py))
    return kTooFar;  // too far for one periodic image
  r.px[t] = wrap(v[0][0] + ux, m.px);
  r.py[t] = wrap(v[0][1] + uy, m.py);
  r.loc[t] = (int32_t)t;
  r.prio[t] = priority(t, r.seed);
  return kCandidate;
}

// Index of vertex v among the corners of t (or -1).
DL_FN int corner_of(const Mesh& m, int64_t t, int32_t v) {
  for (int k = 0; k < 3; ++k)
    if (corner(m, k, t) == v) return k;
  return -1;
}

// Boundary edge of x that p encroaches ((a - p).(b - p) < 0, plain FP64): its
// corner index, or -1.
DL_FN int encroached_edge(const Mesh& m, int64_t x, const double* p) {
#pragma clang fp contract(off)
  for (int i = 0; i < 3; ++i) {
    if (across(m, i, x) >= 0) continue;
    double a[2], b[2];
    vnear(m, corner(m, (i + 1) % 3, x), p[0], p[1], a);
    vnear(m, corner(m, (i + 2) % 3, x), p[0], p[1], b);
    if ((a[0] - p[0]) * (b[0] - p[0]) + (a[1] - p[1]) * (b[1] - p[1]) < 0.0) return i;
  }
  return -1;
}

// First triangle around vertex v (starting at s) with a boundary edge that p
// encroaches: returns 1 and sets (x, i); 0 when there is none; -1 when the
// ring is larger than kRing.
DL_FN int encroach_ring(const Mesh& m, int64_t s, int32_t v, const double* p, int32_t& ex, int& ei) {
  int64_t x = s;
  int n = 0;
  // one direction: across the edge (v, next corner)
  for (;;) {
    const int i = encroached_edge(m, x, p);
    if (i >= 0) {
      ex = (int32_t)x;
      ei = i;
      return 1;
    }
    if (++n > kRing) return -1;
    const int k = corner_of(m, x, v);
    const int32_t y = across(m, (k + 2) % 3, x);
    if (y < 0) break;
    if (y == s) return 0;  // the whole ring
    x = y;
  }
  // the other direction, from s, when the first one met the boundary
  x = s;
  for (;;) {
    const int k = corner_of(m, x, v);
    const int32_t y = across(m, (k + 1) % 3, x);
    if (y < 0) return 0;
    x = y;
    const int i = encroached_edge(m, x, p);
    if (i >= 0) {
      ex = (int32_t)x;
      ei = i;
      return 1;
    }
    if (++n > kRing) return -1;
  }
}

// Locate the candidate of t by walking from t towards it (exact orientation
// tests: step across the first edge that has the point strictly outside);
// a walk that leaves through a boundary edge splits that edge instead. Then
// the encroachment test over the triangles around the corners of the
// insertion triangle(s): the first encroached boundary edge is split at its
// midpoint instead.
DL_FN void locate_body(const Mesh& m, const Refine& r, int64_t t) {
#pragma clang fp contract(off)
  if (!r.prio[t] || r.where[t] >= 3) return;  // no candidate, or already a boundary split
  double p[2] = {r.px[t], r.py[t]};
  int64_t s = t;
  int where = -1;
  bool found = false;
  for (int step = 0; step < kWalk && !found; ++step) {
    double v[3][2];
    tri_near(m, s, p, v);
    int out = -1, zeros = 0, zi = -1;
    for (int i = 0; i < 3; ++i) {
      const int o = pred::orient(v[(i + 1) % 3], v[(i + 2) % 3], p);
      if (o < 0 && out < 0) out = i;
      if (o == 0) {
        ++zeros;
        zi = i;
      }
    }
    if (out >= 0) {
      const int32_t nb = across(m, out, s);
      if (nb >= 0) {
        s = nb;
        continue;
      }
      // outside the triangulation: split the boundary edge the walk met
      const double* b = v[(out + 1) % 3];
      const double* c = v[(out + 2) % 3];
      r.px[t] = wrap(0.5 * (b[0] + c[0]), m.px);
      r.py[t] = wrap(0.5 * (b[1] + c[1]), m.py);
      r.loc[t] = (int32_t)s;
      r.where[t] = 3 + out;
      return;
    }
    if (zeros >= 2) break;  // on a vertex: nothing to insert
    where = zeros == 1 ? (across(m, zi, s) < 0 ? 3 + zi : zi) : -1;
    found = true;
  }
  if (!found) {
    r.loc[t] = -1;
    atomicAdd(&r.count[1], 1);
    return;
  }
  r.loc[t] = (int32_t)s;
  r.where[t] = where;
  // corners whose surrounding triangles are checked
  int32_t vs[4];
  int64_t vt[4];
  int nvs = 0;
  for (int k = 0; k < 3; ++k) {
    vs[nvs] = corner(m, k, s);
    vt[nvs++] = s;
  }
  if (where >= 0 && where < 3) {
    const int32_t u = across(m, where, s);
    const int32_t b = corner(m, (where + 1) % 3, s), c = corner(m, (where + 2) % 3, s);
    for (int k = 0; k < 3; ++k) {
      const int32_t w = corner(m, k, u);
      if (w != b && w != c) {
        vs[nvs] = w;
        vt[nvs++] = u;
      }
    }
  }
  for (int q = 0; q < nvs; ++q) {
    int32_t ex = -1;
    int ei = -1;
    const int e = encroach_ring(m, vt[q], vs[q], p, ex, ei);
    if (e < 0) {
      r.loc[t] = -1;
      atomicAdd(&r.count[1], 1);
      return;
    }
    if (e > 0) {
      double b[2], c[2];
      const double o[2] = {m.x[corner(m, (ei + 1) % 3, ex)], m.y[corner(m, (ei + 1) % 3, ex)]};
      b[0] = o[0];
      b[1] = o[1];
      vnear(m, corner(m, (ei + 2) % 3, ex), o[0], o[1], c);
      r.px[t] = wrap(0.5 * (b[0] + c[0]), m.px);
      r.py[t] = wrap(0.5 * (b[1] + c[1]), m.py);
      r.loc[t] = ex;
      r.where[t] = 3 + ei;
      return;
    }
  }
}

// The candidate's cavity, conservatively: its insertion triangle(s) and,
// breadth first through neighbours, every triangle whose circumcircle the
// FP64 in-circle test does not place strictly outside of the point (a
// superset of the triangles whose circumcircle holds the point). Returns
// the size, or -1 beyond kCavity.
DL_FN int cavity(const Mesh& m, const Refine& r, int64_t t, int32_t* cav) {
  const double p[2] = {r.px[t], r.py[t]};
  const int32_t s = r.loc[t];
  const int where = r.where[t];
  int n = 0;
  cav[n++] = s;
  if (where >= 0 && where < 3) cav[n++] = across(m, where, s);
  for (int q = 0; q < n; ++q) {
    const int32_t x = cav[q];
    for (int k = 0; k < 3; ++k) {
      const int32_t y = across(m, k, x);
      if (y < 0) continue;
      bool seen = false;
      for (int z = 0; z < n; ++z) seen = seen || cav[z] == y;
      if (seen) continue;
      double v[3][2];
      tri_near(m, y, p, v);
      if (pred::incircle_filter(v[0], v[1], v[2], p) < 0) continue;
      if (n == kCavity) return -1;
      cav[n++] = y;
    }
  }
  return n;
}

// Lock every triangle of the candidate's cavity with its priority (highest
// priority holds a triangle).
DL_FN void lock_body(const Mesh& m, const Refine& r, int64_t t) {
  if (!r.prio[t] || r.loc[t] < 0) return;
  int32_t cav[kCavity];
  const int n = cavity(m, r, t, cav);
  if (n < 0) {
    r.loc[t] = -1;
    atomicAdd(&r.count[2], 1);
    return;
  }
  for (int q = 0; q < n; ++q) atomicMax(&r.lock[cav[q]], r.prio[t]);
}

// A candidate is inserted when it holds every triangle of its cavity.
DL_FN void check_body(const Mesh& m, const Refine& r, int64_t t) {
  if (!r.prio[t] || r.loc[t] < 0) return;
  int32_t cav[kCavity];
  const int n = cavity(m, r, t, cav);
  bool all = n > 0;
  for (int q = 0; q < n; ++q) all = all && r.lock[cav[q]] == r.prio[t];
  r.win[t] = all ? 1 : 0;
  r.tnew[t] = all ? (r.where[t] >= 3 ? 1 : 2) : 0;
}

DL_FN void set_tri(const Mesh& m, int64_t t, int32_t a, int32_t b, int32_t c, int32_t na, int32_t nb, int32_t nc) {
  m.tri[0 * m.ts + t] = a;
  m.tri[1 * m.ts + t] = b;
  m.tri[2 * m.ts + t] = c;
  m.nbr[0 * m.ts + t] = na;
  m.nbr[1 * m.ts + t] = nb;
  m.nbr[2 * m.ts + t] = nc;
}

// Insert the winning candidate of t as vertex nv + wpos[t]: inside its
// triangle s = (a, b, c) (s becomes three triangles), on the interior edge
// shared by s and u (each becomes two), or on a boundary edge of s (s
// becomes two). New triangles are numbered from m.nt + tpos[t]; the
// neighbour entries of the split triangles' outer neighbours are repaired by
// fixsplit_body. The split triangles and their children are marked for the
// next edge-test pass `pass`.
DL_FN void insert_body(const Mesh& m, const Refine& r, int64_t t, int32_t it, int32_t pass) {
  if (!r.win[t]) return;
  const int32_t pv = (int32_t)(r.nv + r.wpos[t]);
  m.x[pv] = r.px[t];
  m.y[pv] = r.py[t];
  const int32_t t1 = (int32_t)(m.nt + r.tpos[t]);
  const int32_t s = r.loc[t];
  const int where = r.where[t];
  const int64_t ts = m.ts;
  if (where < 0) {
    const int32_t a = corner(m, 0, s), b = corner(m, 1, s), c = corner(m, 2, s);
    const int32_t n0 = across(m, 0, s), n1 = across(m, 1, s), n2 = across(m, 2, s);
    const int32_t t2 = t1 + 1;
    set_tri(m, s, a, b, pv, t1, t2, n2);
    set_tri(m, t1, b, c, pv, t2, s, n0);
    set_tri(m, t2, c, a, pv, s, t1, n1);
    m.mark[s] = m.mark[t1] = m.mark[t2] = pass;
    r.split[s] = it;
    r.child[0 * ts + s] = t1;
    r.child[1 * ts + s] = t2;
    return;
  }
  const int i = where % 3;
  const int32_t a = corner(m, i, s), b = corner(m, (i + 1) % 3, s), c = corner(m, (i + 2) % 3, s);
  const int32_t n_ab = across(m, (i + 2) % 3, s), n_ca = across(m, (i + 1) % 3, s);
  if (where >= 3) {
    set_tri(m, s, a, b, pv, -1, t1, n_ab);
    set_tri(m, t1, a, pv, c, -1, n_ca, s);
    m.mark[s] = m.mark[t1] = pass;
    r.split[s] = it;
    r.child[0 * ts + s] = t1;
    r.child[1 * ts + s] = -1;
    return;
  }
  const int32_t u = across(m, i, s);
  const int32_t t2 = t1 + 1;
  int32_t d = -1, n_bd = -1, n_dc = -1;
  for (int k = 0; k < 3; ++k) {
    const int32_t w = corner(m, k, u);
    if (w != b && w != c) d = w;
    if (w == c) n_bd = across(m, k, u);
    if (w == b) n_dc = across(m, k, u);
  }
  set_tri(m, s, a, b, pv, u, t1, n_ab);
  set_tri(m, t1, a, pv, c, t2, n_ca, s);
  set_tri(m, u, pv, b, d, n_bd, t2, s);
  set_tri(m, t2, c, pv, d, u, n_dc, t1);
  m.mark[s] = m.mark[t1] = m.mark[u] = m.mark[t2] = pass;
  r.split[s] = it;
  r.child[0 * ts + s] = t1;
  r.child[1 * ts + s] = -1;
  r.split[u] = it;
  r.child[0 * ts + u] = t2;
  r.child[1 * ts + u] = -1;
}

DL_FN bool has_edge(const Mesh& m, int64_t x, int32_t p, int32_t q) {
  int h = 0;
  for (int k = 0; k < 3; ++k) {
    const int32_t v = corner(m, k, x);
    h += (v == p) + (v == q);
  }
  return h == 2;
}

// Neighbour entries of w that point at a triangle split this iteration now
// point at whichever of it and its children (w excepted) holds the shared
// edge.
DL_FN void fixsplit_body(const Mesh& m, const Refine& r, int64_t w, int32_t it) {
  for (int k = 0; k < 3; ++k) {
    const int32_t x = across(m, k, w);
    if (x < 0 || r.split[x] != it) continue;
    const int32_t p = corner(m, (k + 1) % 3, w), q = corner(m, (k + 2) % 3, w);
    const int32_t opts[3] = {x, r.child[0 * m.ts + x], r.child[1 * m.ts + x]};
    for (int z = 0; z < 3; ++z) {
      const int32_t y = opts[z];
      if (y < 0 || y == w) continue;
      if (has_edge(m, y, p, q)) {
        m.nbr[k * m.ts + w] = y;
        break;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Morton ordering (Section 4.1: vertices and triangles renumbered along a
// Z-order curve as the mesh grows, for locality). A key interleaves the
// 32-bit quantised coordinates, x in the even bits:
// q(x) = min(2^32 - 1, floor(max(0, (x - x0) * sx))), likewise for y; a
// triangle's key is that of its centroid (corners at their images nearest
// to corner 0, the mean wrapped into the period). Elements are ordered by
// the top 32 bits of the key (a 2^16 x 2^16 grid of cells), which is what
// is stored and sorted; the sort is stable, so elements in one cell keep
// their order.

struct Order {
  double x0 = 0.0, y0 = 0.0, sx = 0.0, sy = 0.0;
  uint32_t* key = nullptr;             // [n] top 32 bits of the keys
  uint32_t* skey = nullptr;            // [n] sorted
  int32_t* idx = nullptr;              // [n] 0, 1, ..., n - 1
  int32_t* perm = nullptr;             // [n] new -> old
  int32_t* inv = nullptr;              // [n] old -> new
  double* xt = nullptr;                // [vertex capacity] reordered coordinates
  double* yt = nullptr;
  int32_t* tt = nullptr;               // [3][ts] reordered corners
  int32_t* nb = nullptr;               // [3][ts] reordered neighbours
};

DL_FN unsigned long long spread_bits(uint32_t v) {
  unsigned long long x = v;
  x = (x | (x << 16)) & 0x0000ffff0000ffffull;
  x = (x | (x << 8)) & 0x00ff00ff00ff00ffull;
  x = (x | (x << 4)) & 0x0f0f0f0f0f0f0f0full;
  x = (x | (x << 2)) & 0x3333333333333333ull;
  x = (x | (x << 1)) & 0x5555555555555555ull;
  return x;
}

DL_FN uint32_t quantise(double v, double v0, double s) {
#pragma clang fp contract(off)
  double q = (v - v0) * s;
  if (!(q > 0.0)) q = 0.0;
  if (q > 4294967295.0) q = 4294967295.0;
  return (uint32_t)q;
}

DL_FN unsigned long long morton_key(const Order& o, double x, double y) {
  return spread_bits(quantise(x, o.x0, o.sx)) | (spread_bits(quantise(y, o.y0, o.sy)) << 1);
}

DL_FN void vkey_body(const Mesh& m, const Order& o, int64_t v) {
  o.key[v] = (uint32_t)(morton_key(o, m.x[v], m.y[v]) >> 32);
  o.idx[v] = (int32_t)v;
}

DL_FN void tkey_body(const Mesh& m, const Order& o, int64_t t) {
#pragma clang fp contract(off)
  double v[3][2];
  const double a[2] = {m.x[corner(m, 0, t)], m.y[corner(m, 0, t)]};
  tri_near(m, t, a, v);
  const double cx = wrap((v[0][0] + v[1][0] + v[2][0]) / 3.0, m.px);
  const double cy = wrap((v[0][1] + v[1][1] + v[2][1]) / 3.0, m.py);
  o.key[t] = (uint32_t)(morton_key(o, cx, cy) >> 32);
  o.idx[t] = (int32_t)t;
}

DL_FN void invert_body(const Order& o, int64_t i) { o.inv[o.perm[i]] = (int32_t)i; }

// Coordinates in the new vertex order (to o.xt, o.yt) and every corner
// renamed (in place: each triangle its own).
DL_FN void vapply_body(const Mesh& m, const Order& o, int64_t i) {
  o.xt[i] = m.x[o.perm[i]];
  o.yt[i] = m.y[o.perm[i]];
}
DL_FN void vrename_body(const Mesh& m, const Order& o, int64_t t) {
  for (int k = 0; k < 3; ++k) m.tri[k * m.ts + t] = o.inv[m.tri[k * m.ts + t]];
}

// Triangles in the new order (to o.tt, o.nb), neighbours renamed.
DL_FN void tapply_body(const Mesh& m, const Order& o, int64_t i) {
  const int32_t old = o.perm[i];
  for (int k = 0; k < 3; ++k) {
    o.tt[k * m.ts + i] = m.tri[k * m.ts + old];
    const int32_t n = m.nbr[k * m.ts + old];
    o.nb[k * m.ts + i] = n < 0 ? -1 : o.inv[n];
  }
}

}  // namespace dl
}  // namespace rd
