// Exact in-circle predicate for the Delaunay flips of mesh generation
// (Section 2: the flip test must be exact, or flipping can cycle or create
// inverted triangles).
//
// Method: floating-point expansion arithmetic (Shewchuk 1997, the paper's
// reference for its predicates). A number is held exactly as a sum of
// doubles of increasing magnitude that do not overlap; sums and products of
// doubles are made exact with an error-free transformation (the rounding
// error of a + b and of a * b is itself a double). The in-circle
// determinant is first evaluated in plain FP64 with a bound on its rounding
// error; only when the result is within that bound of zero is it recomputed
// exactly (every coordinate difference carried as a two-term expansion).
//
// Everything here must be evaluated exactly as written: each function
// switches off multiply-add contraction. Like all expansion arithmetic it is
// exact as long as no product underflows or overflows: every nonzero
// coordinate difference between about 2^-200 and 2^250 in magnitude.
#pragma once

#include <cmath>
#include <cstdint>

#ifndef __HIP_DEVICE_COMPILE__
#ifndef __host__
#define __host__
#define __device__
#define RD_PRED_HOST_ONLY 1
#endif
#endif

namespace rd {
namespace pred {

// x + y = a + b exactly (x = fl(a + b)).
__host__ __device__ inline void two_sum(double a, double b, double& x, double& y) {
#pragma clang fp contract(off)
  x = a + b;
  const double bv = x - a;
  const double av = x - bv;
  y = (a - av) + (b - bv);
}

// x + y = a + b exactly, for |a| >= |b| or a = 0.
__host__ __device__ inline void fast_two_sum(double a, double b, double& x, double& y) {
#pragma clang fp contract(off)
  x = a + b;
  y = b - (x - a);
}

// x + y = a * b exactly (the fused multiply-add gives the rounding error).
__host__ __device__ inline void two_product(double a, double b, double& x, double& y) {
#pragma clang fp contract(off)
  x = a * b;
  y = fma(a, b, -x);
}

// h = e + b for an expansion e of n terms (increasing magnitude, no zero
// terms kept); returns the length of h (at most n + 1). h may not alias e.
__host__ __device__ inline int grow(int n, const double* e, double b, double* h) {
#pragma clang fp contract(off)
  double q = b;
  int m = 0;
  for (int i = 0; i < n; ++i) {
    double s, err;
    two_sum(q, e[i], s, err);
    q = s;
    if (err != 0.0) h[m++] = err;
  }
  if (q != 0.0 || m == 0) h[m++] = q;
  return m;
}

// h = e + f by growing e by every term of f in turn (lengths add);
// tmp holds at least ne + nf terms. h may alias neither e nor f.
__host__ __device__ inline int sum(int ne, const double* e, int nf, const double* f, double* h, double* tmp) {
  int n = ne;
  double* src = h;
  double* dst = tmp;
  for (int i = 0; i < ne; ++i) src[i] = e[i];
  for (int j = 0; j < nf; ++j) {
    n = grow(n, src, f[j], dst);
    double* t = src;
    src = dst;
    dst = t;
  }
  if (src != h)
    for (int i = 0; i < n; ++i) h[i] = src[i];
  return n;
}

// h = e * b (at most 2n terms).
__host__ __device__ inline int scale(int n, const double* e, double b, double* h) {
#pragma clang fp contract(off)
  double q, lo;
  two_product(e[0], b, q, lo);
  int m = 0;
  if (lo != 0.0) h[m++] = lo;
  for (int i = 1; i < n; ++i) {
    double p1, p0, s, err;
    two_product(e[i], b, p1, p0);
    two_sum(q, p0, s, err);
    if (err != 0.0) h[m++] = err;
    fast_two_sum(p1, s, q, err);
    if (err != 0.0) h[m++] = err;
  }
  if (q != 0.0 || m == 0) h[m++] = q;
  return m;
}

// h = e * f (at most 2 ne nf terms); tmp holds at least 2 (2 ne nf) + 2 ne terms.
__host__ __device__ inline int mul(int ne, const double* e, int nf, const double* f, double* h, double* tmp) {
  double* part = tmp;              // one scaled copy: <= 2 ne
  double* acc = tmp + 2 * ne;      // running product
  double* work = acc + 2 * ne * nf;
  int na = 0;
  for (int j = 0; j < nf; ++j) {
    const int np = scale(ne, e, f[j], part);
    if (j == 0) {
      for (int i = 0; i < np; ++i) acc[i] = part[i];
      na = np;
    } else {
      na = sum(na, acc, np, part, h, work);
      for (int i = 0; i < na; ++i) acc[i] = h[i];
    }
  }
  for (int i = 0; i < na; ++i) h[i] = acc[i];
  return na;
}

__host__ __device__ inline void negate(int n, double* e) {
  for (int i = 0; i < n; ++i) e[i] = -e[i];
}

// Sign of an expansion: that of its largest (last) term.
__host__ __device__ inline int sign(int n, const double* e) {
  const double x = e[n - 1];
  return (x > 0.0) - (x < 0.0);
}

// Scratch terms the exact in-circle evaluation needs.
constexpr int kIncircleScratch = 5184;

// Exact sign of the in-circle determinant of (a, b, c, d): the 3x3
// determinant with rows (p_x - d_x, p_y - d_y, (p_x - d_x)^2 + (p_y - d_y)^2)
// for p = a, b, c; positive when d lies inside the circle through a, b, c
// (counter-clockwise), zero on it. w: kIncircleScratch doubles.
__host__ __device__ inline int incircle_exact(const double* a, const double* b, const double* c, const double* d,
                                              double* w) {
#pragma clang fp contract(off)
  // coordinate differences as exact two-term expansions
  double dx[3][2], dy[3][2];
  int nx[3], ny[3];
  const double* p[3] = {a, b, c};
  for (int i = 0; i < 3; ++i) {
    double hi, lo;
    two_sum(p[i][0], -d[0], hi, lo);
    nx[i] = 0;
    if (lo != 0.0) dx[i][nx[i]++] = lo;
    if (hi != 0.0 || nx[i] == 0) dx[i][nx[i]++] = hi;
    two_sum(p[i][1], -d[1], hi, lo);
    ny[i] = 0;
    if (lo != 0.0) dy[i][ny[i]++] = lo;
    if (hi != 0.0 || ny[i] == 0) dy[i][ny[i]++] = hi;
  }
  // buffers (sizes for two-term inputs): products <= 8, cross <= 16,
  // lift <= 16, lift * cross <= 512, total <= 1536
  double* t1 = w;            // 8
  double* t2 = w + 8;        // 8
  double* cross = w + 16;    // 16
  double* lift = w + 32;     // 16
  double* term = w + 48;     // 512
  double* total = w + 560;   // 1536
  double* tot2 = w + 2096;   // 1536
  double* tmp = w + 3632;    // scratch for mul / sum (1552: a sum of up to 1536 terms, or 1088 for mul)
  int ntot = 0;
  for (int k = 0; k < 3; ++k) {
    const int i = (k + 1) % 3, j = (k + 2) % 3;
    // cross_k = dx_i dy_j - dx_j dy_i
    const int n1 = mul(nx[i], dx[i], ny[j], dy[j], t1, tmp);
    const int n2 = mul(nx[j], dx[j], ny[i], dy[i], t2, tmp);
    negate(n2, t2);
    const int nc = sum(n1, t1, n2, t2, cross, tmp);
    // lift_k = dx_k^2 + dy_k^2
    const int l1 = mul(nx[k], dx[k], nx[k], dx[k], t1, tmp);
    const int l2 = mul(ny[k], dy[k], ny[k], dy[k], t2, tmp);
    const int nl = sum(l1, t1, l2, t2, lift, tmp);
    const int nt = mul(nl, lift, nc, cross, term, tmp);
    if (k == 0) {
      for (int q = 0; q < nt; ++q) total[q] = term[q];
      ntot = nt;
    } else {
      ntot = sum(ntot, total, nt, term, tot2, tmp);
      for (int q = 0; q < ntot; ++q) total[q] = tot2[q];
    }
  }
  return sign(ntot, total);
}

// The same determinant in plain FP64 with a bound on its rounding error:
// returns +1 / -1 when the sign is certain, 0 when the exact evaluation is
// needed. The bound (11 + 100 eps) eps * permanent exceeds the forward error
// of this evaluation order (differences, products and sums of the
// expansion along the third column).
__host__ __device__ inline int incircle_filter(const double* a, const double* b, const double* c, const double* d) {
#pragma clang fp contract(off)
  const double adx = a[0] - d[0], ady = a[1] - d[1];
  const double bdx = b[0] - d[0], bdy = b[1] - d[1];
  const double cdx = c[0] - d[0], cdy = c[1] - d[1];
  const double bc = bdx * cdy - cdx * bdy, ca = cdx * ady - adx * cdy, ab = adx * bdy - bdx * ady;
  const double al = adx * adx + ady * ady, bl = bdx * bdx + bdy * bdy, cl = cdx * cdx + cdy * cdy;
  const double det = al * bc + bl * ca + cl * ab;
  const double perm = (fabs(bdx * cdy) + fabs(cdx * bdy)) * al + (fabs(cdx * ady) + fabs(adx * cdy)) * bl +
                      (fabs(adx * bdy) + fabs(bdx * ady)) * cl;
  const double eps = 1.1102230246251565e-16;  // 2^-53
  const double bound = (11.0 + 100.0 * eps) * eps * perm;
  if (det > bound) return 1;
  if (-det > bound) return -1;
  return 0;
}

// Exact sign of the orientation determinant of (a, b, c): (a - c) x (b - c),
// positive when a, b, c are counter-clockwise, zero when collinear. FP64 with
// the error bound (3 + 16 eps) eps (|l| + |r|) of the two products first; when
// that cannot decide, the coordinate differences as two-term expansions and
// the determinant as an exact expansion (at most 16 terms).
__host__ __device__ inline int orient(const double* a, const double* b, const double* c) {
#pragma clang fp contract(off)
  const double l = (a[0] - c[0]) * (b[1] - c[1]), r = (a[1] - c[1]) * (b[0] - c[0]);
  const double det = l - r;
  const double eps = 1.1102230246251565e-16;
  const double bound = (3.0 + 16.0 * eps) * eps * (fabs(l) + fabs(r));
  if (det > bound) return 1;
  if (-det > bound) return -1;
  double d[4][2];
  int n[4];
  const double v[4][2] = {{a[0], c[0]}, {b[1], c[1]}, {a[1], c[1]}, {b[0], c[0]}};
  for (int k = 0; k < 4; ++k) {
    double hi, lo;
    two_sum(v[k][0], -v[k][1], hi, lo);
    n[k] = 0;
    if (lo != 0.0) d[k][n[k]++] = lo;
    if (hi != 0.0 || n[k] == 0) d[k][n[k]++] = hi;
  }
  double t1[8], t2[8], out[16], tmp[40];
  const int n1 = mul(n[0], d[0], n[1], d[1], t1, tmp);
  const int n2 = mul(n[2], d[2], n[3], d[3], t2, tmp);
  negate(n2, t2);
  const int no = sum(n1, t1, n2, t2, out, tmp);
  return sign(no, out);
}

}  // namespace pred
}  // namespace rd

#ifdef RD_PRED_HOST_ONLY
#undef __host__
#undef __device__
#undef RD_PRED_HOST_ONLY
#endif
