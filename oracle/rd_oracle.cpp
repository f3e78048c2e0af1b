// Plain CPU oracle for the residual-distribution step of the two-dimensional
// Euler equations on triangular meshes (Paardekooper 2017, Section 3 and
// Appendix A).
//
// TEST INFRASTRUCTURE ONLY. This file is the independent reference the GPU
// library is checked against. It shares no code, header or table with the
// GPU path; only the tests, the smoke check and the benchmark's CPU-baseline
// leg load it. It is written for readability, not speed: every step follows
// the paper's order and notation, in IEEE FP64, built without FMA
// contraction (-ffp-contract=off) and without fast-math.
//
// The scalar type is a template parameter. `double` gives the oracle itself;
// `Dual` (value + tangent) runs the very same code in forward mode and gives
// the exact Jacobian-vector product of a step, used to pin the hand-written
// adjoint of the GPU library. Branches (max/min of eigenvalues, pivot choice,
// |.|, the 0/0 and clamp cases of the blend) are taken on the value part, so
// derivatives follow the branch the value takes; d|x|/dx at x = 0 is 0.
//
// Readings of points the paper leaves open (each also listed in the design
// notes of the repository):
//  * Parameter vector in two dimensions: Z = sqrt(rho) (1, u, v, h), the
//    multidimensional analogue named in Section 3.2.
//  * K_i = (|n_i|/2) K(n_i/|n_i|): n_i is the inward normal scaled by the
//    edge length (the gradient formula of Section 3.2 needs that), 1/d = 1/2,
//    and Appendix A's entries are for a unit normal (eigenvalues w +- c).
//  * K_i^{+-} are Appendix A's explicit entries with l = lambda^{+-}; K_i is
//    the same formula with l = lambda.
//  * The state differences the K matrices act on are dW_i = M(Zbar)(Z_i-Z_0),
//    M = dW/dZ at the Roe average, which is the Z-form of Section 3.2 written
//    with the W-form matrices of Appendix A (equal in exact arithmetic).
//  * N-hat = (sum K^-)^{-1} = -A^{-1} with A = sum K^+; the N and LDA parts
//    solve A x = b by Gaussian elimination with partial pivoting; a column
//    whose best pivot is at most 2^-45 max|A| is skipped (its unknown is 0).
//    At stagnation A is singular but K_i^+ x does not depend on the choice.
//  * Blend (Section 3.3.3): Theta_k = |phi^T_k| / sum_i |phi^N_{i,k}|, 0 when
//    the denominator is 0, and at most 1 (exact arithmetic gives <= 1).
//  * Vertex volume V_i = sum of |T|/3 over the triangles of i (median dual),
//    the global lumping of Section 3.4.
//  * RK2 (Section 3.4): phi(n) terms are the stage-1 values; Phi^T is the
//    total residual of the triangle; the LDA coefficients of stage 2 are
//    taken at W*; the wall term of stage 2 is the mean of its values at W^n
//    and W*. Ghost vertices keep their value.
//  * Vertex sums run over the triangles of a vertex in ascending triangle
//    order, then add the wall term.
//  * Bx (Section 3.3.3, after Dobes): one scalar theta per triangle,
//    theta = min(1, s^2 h / L) with s = max(0, -L div(v) / (|v|max - |v|min)).
//    As printed theta = s^2 h has the dimension of a length; h is read in
//    units of the domain size L (on the unit square this is the printed
//    formula) and theta is clamped to 1 so that the blend stays convex.
//    h = sqrt(2|T|) (the leg of a right isosceles triangle of that area);
//    div(v) is the divergence of the linear interpolant of the vertex
//    velocities, sum_i v_i . n_i / (2|T|) with the inward scaled normals;
//    |v|max and |v|min are taken over all vertices of the mesh at the
//    stage's state (W^n in stage 1, W* in stage 2); s = 0 when they are
//    equal. L is the larger side of the domain: the period on a periodic
//    axis, else the extent of the vertex coordinates.
//  * Selective lumping (Section 3.4): in stage 2 both the N and the LDA
//    total parts get sum_j (|T| delta_ij / 3 - m^G_ij)(W*_j - W^n_j)/dt
//    with the Galerkin mass m^G_ij = |T| (1 + delta_ij) / 12, before the
//    blend (so the B coefficients see the lumped N parts). Off by default
//    (global lumping); it does nothing in a forward Euler step.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ------------------------------------------------------------ scalars -----

struct Dual {
  double v, d;
  Dual() : v(0.0), d(0.0) {}
  Dual(double a) : v(a), d(0.0) {}  // NOLINT: constants promote
  Dual(double a, double b) : v(a), d(b) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
  double q = a.v / b.v;
  return Dual(q, (a.d - q * b.d) / b.v);
}
inline Dual operator+(Dual a, double b) { return Dual(a.v + b, a.d); }
inline Dual operator+(double a, Dual b) { return Dual(a + b.v, b.d); }
inline Dual operator-(Dual a, double b) { return Dual(a.v - b, a.d); }
inline Dual operator-(double a, Dual b) { return Dual(a - b.v, -b.d); }
inline Dual operator*(Dual a, double b) { return Dual(a.v * b, a.d * b); }
inline Dual operator*(double a, Dual b) { return Dual(a * b.v, a * b.d); }
inline Dual operator/(Dual a, double b) { return Dual(a.v / b, a.d / b); }
inline Dual operator/(double a, Dual b) {
  double q = a / b.v;
  return Dual(q, -q * b.d / b.v);
}
inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
inline Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }

inline double val(double x) { return x; }
inline double val(Dual x) { return x.v; }
inline double sq_root(double x) { return std::sqrt(x); }
inline Dual sq_root(Dual x) {
  double s = std::sqrt(x.v);
  return Dual(s, x.d / (2.0 * s));
}
template <class T> inline T absval(T x) {
  if (val(x) > 0.0) return x;
  if (val(x) < 0.0) return -x;
  return T(0.0);
}
template <class T> inline T pos_part(T x) { return val(x) > 0.0 ? x : T(0.0); }
template <class T> inline T neg_part(T x) { return val(x) < 0.0 ? x : T(0.0); }

enum { SCHEME_N = 0, SCHEME_LDA = 1, SCHEME_B = 2, SCHEME_BMAX = 3, SCHEME_BMIN = 4, SCHEME_BX = 5 };

// ---------------------------------------------------------------- mesh ----

struct Mesh {
  int64_t nv = 0, nt = 0;
  std::vector<double> x, y;
  std::vector<int32_t> tri;  // [nt][3]
  double px = 0.0, py = 0.0;
  std::vector<uint8_t> ghost;
  std::vector<int32_t> wall;  // [nw][2]
  double gamma = 1.4;
  // geometry (Section 3.2, 3.3)
  std::vector<double> area;   // |T|
  std::vector<double> nrm;    // inward normals scaled by edge length, [nt][3][2]
  std::vector<double> lmax;   // longest edge
  std::vector<double> V;      // vertex volume
  std::vector<double> wlen, wnx, wny;  // wall edge length and outward unit normal
  double L = 0.0;           // domain size (Bx sensor)
  bool selective = false;   // selective lumping in stage 2
};

// Minimum-image difference of two coordinates on a periodic axis.
double unwrap(double d, double period) {
  if (period > 0.0) {
    if (d > 0.5 * period) d -= period;
    else if (d < -0.5 * period) d += period;
  }
  return d;
}

bool build_geometry(Mesh& m, std::string& err) {
  m.area.assign(m.nt, 0.0);
  m.nrm.assign(m.nt * 6, 0.0);
  m.lmax.assign(m.nt, 0.0);
  m.V.assign(m.nv, 0.0);
  for (int64_t t = 0; t < m.nt; ++t) {
    int32_t v[3] = {m.tri[3 * t], m.tri[3 * t + 1], m.tri[3 * t + 2]};
    for (int k = 0; k < 3; ++k) {
      if (v[k] < 0 || v[k] >= m.nv) {
        err = "triangle " + std::to_string(t) + " has a vertex index out of range";
        return false;
      }
    }
    // corner positions relative to corner 0, unwrapped to the minimum image
    double p[3][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    for (int k = 1; k < 3; ++k) {
      p[k][0] = unwrap(m.x[v[k]] - m.x[v[0]], m.px);
      p[k][1] = unwrap(m.y[v[k]] - m.y[v[0]], m.py);
    }
    double a = 0.5 * (p[1][0] * p[2][1] - p[1][1] * p[2][0]);
    if (!(a > 0.0)) {
      err = "triangle " + std::to_string(t) + " is not counter-clockwise with positive area";
      return false;
    }
    m.area[t] = a;
    double lm = 0.0;
    for (int i = 0; i < 3; ++i) {
      // inward normal of the edge opposite corner i: rotate (p_{i+2} - p_{i+1}) by +90 degrees
      const double* pa = p[(i + 1) % 3];
      const double* pb = p[(i + 2) % 3];
      double ex = pb[0] - pa[0], ey = pb[1] - pa[1];
      m.nrm[6 * t + 2 * i] = -ey;
      m.nrm[6 * t + 2 * i + 1] = ex;
      lm = std::max(lm, std::sqrt(ex * ex + ey * ey));
    }
    m.lmax[t] = lm;
  }
  for (int64_t t = 0; t < m.nt; ++t)
    for (int k = 0; k < 3; ++k) m.V[m.tri[3 * t + k]] += m.area[t] / 3.0;
  {
    double x0 = m.x[0], x1 = m.x[0], y0 = m.y[0], y1 = m.y[0];
    for (int64_t i = 0; i < m.nv; ++i) {
      x0 = std::min(x0, m.x[i]);
      x1 = std::max(x1, m.x[i]);
      y0 = std::min(y0, m.y[i]);
      y1 = std::max(y1, m.y[i]);
    }
    const double lx = m.px > 0.0 ? m.px : x1 - x0, ly = m.py > 0.0 ? m.py : y1 - y0;
    m.L = std::max(lx, ly);
  }
  for (int64_t i = 0; i < m.nv; ++i) {
    if (!(m.V[i] > 0.0)) {
      err = "vertex " + std::to_string(i) + " belongs to no triangle";
      return false;
    }
  }
  int64_t nw = (int64_t)m.wall.size() / 2;
  m.wlen.assign(nw, 0.0);
  m.wnx.assign(nw, 0.0);
  m.wny.assign(nw, 0.0);
  for (int64_t e = 0; e < nw; ++e) {
    int32_t a = m.wall[2 * e], b = m.wall[2 * e + 1];
    if (a < 0 || a >= m.nv || b < 0 || b >= m.nv || a == b) {
      err = "wall edge " + std::to_string(e) + " is invalid";
      return false;
    }
    double dx = unwrap(m.x[b] - m.x[a], m.px), dy = unwrap(m.y[b] - m.y[a], m.py);
    double len = std::sqrt(dx * dx + dy * dy);
    m.wlen[e] = len;
    m.wnx[e] = dy / len;   // the domain lies to the left of a->b, so the
    m.wny[e] = -dx / len;  // outward normal is the right-hand normal
  }
  return true;
}

// ------------------------------------------------------ per-vertex maps ---

// Z = sqrt(rho) (1, u, v, h) from W = (rho, rho u, rho v, e).
template <class T> void w_to_z(const T W[4], double gamma, T Z[4]) {
  T rho = W[0];
  T u = W[1] / rho, v = W[2] / rho;
  T p = (gamma - 1.0) * (W[3] - 0.5 * rho * (u * u + v * v));
  T h = (W[3] + p) / rho;
  T s = sq_root(rho);
  Z[0] = s;
  Z[1] = s * u;
  Z[2] = s * v;
  Z[3] = s * h;
}

// --------------------------------------------------- Appendix A entries ---

// K(l1, l2, l3) for unit normal (nx, ny) at state (u, v, h, c); l = lambda
// gives K = A nx + B ny, l = lambda^{+-} gives K^{+-}.
template <class T>
void k_entries(T u, T v, T h, T c, double gamma, T nx, T ny, T l1, T l2, T l3, T K[4][4]) {
  const double g1 = gamma - 1.0, g2 = gamma - 2.0;
  T w = u * nx + v * ny;
  T alpha = g1 * (u * u + v * v) / 2.0;
  T ac = alpha / c, uc = u / c, vc = v / c, hc = h / c;
  T l123 = (l1 + l2 - 2.0 * l3) / 2.0;
  T l12 = (l1 - l2) / 2.0;
  K[0][0] = ac / c * l123 - w / c * l12 + l3;
  K[0][1] = -g1 * uc / c * l123 + nx / c * l12;
  K[0][2] = -g1 * vc / c * l123 + ny / c * l12;
  K[0][3] = g1 / (c * c) * l123;
  K[1][0] = (ac * uc - w * nx) * l123 + (ac * nx - uc * w) * l12;
  K[1][1] = (nx * nx - g1 * uc * uc) * l123 - g2 * uc * nx * l12 + l3;
  K[1][2] = (nx * ny - g1 * uc * vc) * l123 + (uc * ny - g1 * vc * nx) * l12;
  K[1][3] = g1 * uc / c * l123 + g1 * nx / c * l12;
  K[2][0] = (ac * vc - w * ny) * l123 + (ac * ny - vc * w) * l12;
  K[2][1] = (nx * ny - g1 * uc * vc) * l123 + (vc * nx - g1 * uc * ny) * l12;
  K[2][2] = (ny * ny - g1 * vc * vc) * l123 - g2 * vc * ny * l12 + l3;
  K[2][3] = g1 * vc / c * l123 + g1 * ny / c * l12;
  K[3][0] = (ac * hc - w * w) * l123 + w * (ac - hc) * l12;
  K[3][1] = (w * nx - u - ac * uc) * l123 + (hc * nx - g1 * uc * w) * l12;
  K[3][2] = (w * ny - v - ac * vc) * l123 + (hc * ny - g1 * vc * w) * l12;
  K[3][3] = g1 * hc / c * l123 + g1 * w / c * l12 + l3;
}

template <class T> void matvec(const T M[4][4], const T x[4], T y[4]) {
  for (int r = 0; r < 4; ++r) y[r] = M[r][0] * x[0] + M[r][1] * x[1] + M[r][2] * x[2] + M[r][3] * x[3];
}

// A x = b for one right-hand side, partial pivoting with the skip rule.
template <class T> void solve4(const T Ain[4][4], const T b_in[4], T x[4]) {
  T A[4][4], b[4];
  double amax = 0.0;
  for (int r = 0; r < 4; ++r) {
    b[r] = b_in[r];
    for (int c = 0; c < 4; ++c) {
      A[r][c] = Ain[r][c];
      amax = std::max(amax, std::fabs(val(Ain[r][c])));
    }
  }
  const double tol = std::ldexp(amax, -45);
  bool used[4] = {false, false, false, false};
  int prow[4] = {-1, -1, -1, -1};
  for (int k = 0; k < 4; ++k) {
    int r = -1;
    double best = -1.0;
    for (int i = 0; i < 4; ++i) {
      if (used[i]) continue;
      double a = std::fabs(val(A[i][k]));
      if (a > best) { best = a; r = i; }
    }
    if (r < 0 || !(best > tol)) continue;  // column skipped: unknown k is 0
    used[r] = true;
    prow[k] = r;
    for (int i = 0; i < 4; ++i) {
      if (used[i]) continue;
      T f = A[i][k] / A[r][k];
      for (int j = k; j < 4; ++j) A[i][j] = A[i][j] - f * A[r][j];
      b[i] = b[i] - f * b[r];
    }
  }
  for (int k = 3; k >= 0; --k) {
    if (prow[k] < 0) { x[k] = T(0.0); continue; }
    int r = prow[k];
    T s = b[r];
    for (int j = k + 1; j < 4; ++j) s = s - A[r][j] * x[j];
    x[k] = s / A[r][k];
  }
}

// Everything one triangle needs at one state.
template <class T> struct TriState {
  T dW[3][4];       // M(Zbar)(Z_i - Z_0); dW[0] = 0
  T K[3][4][4];     // K_i
  T Kp[3][4][4];    // K_i^+
  T Km[3][4][4];    // K_i^-
  T A[4][4];        // sum_i K_i^+
  T phiT[4];        // triangle residual
  T phiN[3][4];     // N scheme
  T xL[4];          // A^{-1} phi^T
};

// Section 3.2-3.3 for one triangle: Roe average, K matrices, residual, N.
template <class T>
void eval_triangle(const T Zc[3][4], const double n[3][2], double gamma, TriState<T>& s) {
  const double g1 = gamma - 1.0;
  T zb[4];
  for (int k = 0; k < 4; ++k) zb[k] = (Zc[0][k] + Zc[1][k] + Zc[2][k]) / 3.0;
  T u = zb[1] / zb[0], v = zb[2] / zb[0], h = zb[3] / zb[0];
  T c = sq_root(g1 * (h - 0.5 * (u * u + v * v)));
  for (int k = 0; k < 4; ++k) s.dW[0][k] = T(0.0);
  for (int i = 1; i < 3; ++i) {
    T dz[4];
    for (int k = 0; k < 4; ++k) dz[k] = Zc[i][k] - Zc[0][k];
    s.dW[i][0] = 2.0 * zb[0] * dz[0];
    s.dW[i][1] = zb[1] * dz[0] + zb[0] * dz[1];
    s.dW[i][2] = zb[2] * dz[0] + zb[0] * dz[2];
    s.dW[i][3] = (zb[3] * dz[0] + g1 * zb[1] * dz[1] + g1 * zb[2] * dz[2] + zb[0] * dz[3]) / gamma;
  }
  for (int i = 0; i < 3; ++i) {
    double len = std::sqrt(n[i][0] * n[i][0] + n[i][1] * n[i][1]);
    T nx = T(n[i][0] / len), ny = T(n[i][1] / len);
    T w = u * nx + v * ny;
    T lam[3] = {w + c, w - c, w};
    T lp[3], lm[3];
    for (int k = 0; k < 3; ++k) { lp[k] = pos_part(lam[k]); lm[k] = neg_part(lam[k]); }
    k_entries(u, v, h, c, gamma, nx, ny, lam[0], lam[1], lam[2], s.K[i]);
    k_entries(u, v, h, c, gamma, nx, ny, lp[0], lp[1], lp[2], s.Kp[i]);
    k_entries(u, v, h, c, gamma, nx, ny, lm[0], lm[1], lm[2], s.Km[i]);
    const double half = len / 2.0;
    for (int r = 0; r < 4; ++r)
      for (int q = 0; q < 4; ++q) {
        s.K[i][r][q] = half * s.K[i][r][q];
        s.Kp[i][r][q] = half * s.Kp[i][r][q];
        s.Km[i][r][q] = half * s.Km[i][r][q];
      }
  }
  T t1[4], t2[4];
  matvec(s.K[1], s.dW[1], t1);
  matvec(s.K[2], s.dW[2], t2);
  for (int k = 0; k < 4; ++k) s.phiT[k] = t1[k] + t2[k];
  for (int r = 0; r < 4; ++r)
    for (int q = 0; q < 4; ++q) s.A[r][q] = s.Kp[0][r][q] + s.Kp[1][r][q] + s.Kp[2][r][q];
  T bN[4];
  matvec(s.Km[1], s.dW[1], t1);
  matvec(s.Km[2], s.dW[2], t2);
  for (int k = 0; k < 4; ++k) bN[k] = t1[k] + t2[k];
  T xN[4];
  solve4(s.A, bN, xN);
  solve4(s.A, s.phiT, s.xL);
  for (int i = 0; i < 3; ++i) {
    T y[4];
    for (int k = 0; k < 4; ++k) y[k] = s.dW[i][k] + xN[k];
    matvec(s.Kp[i], y, s.phiN[i]);
  }
}

// Blend coefficients of the B family from a residual and its N parts.
template <class T> void blend_theta(const T res[4], const T pn[3][4], int scheme, T theta[4]) {
  for (int k = 0; k < 4; ++k) {
    T den = absval(pn[0][k]) + absval(pn[1][k]) + absval(pn[2][k]);
    if (val(den) == 0.0) {
      theta[k] = T(0.0);
    } else {
      T q = absval(res[k]) / den;
      theta[k] = val(q) > 1.0 ? T(1.0) : q;
    }
  }
  if (scheme == SCHEME_BMAX || scheme == SCHEME_BMIN) {
    int pick = 0;
    for (int k = 1; k < 4; ++k) {
      bool better = scheme == SCHEME_BMAX ? val(theta[k]) > val(theta[pick]) : val(theta[k]) < val(theta[pick]);
      if (better) pick = k;
    }
    T t = theta[pick];
    for (int k = 0; k < 4; ++k) theta[k] = t;
  }
}

// Distributed parts of one triangle for a scheme, given N and LDA parts and
// the residual they split.
template <class T>
void distribute(int scheme, const T res[4], const T pn[3][4], const T pl[3][4], T out[3][4], T theta_out[4],
                T bx = T(0.0)) {
  T theta[4] = {T(0.0), T(0.0), T(0.0), T(0.0)};
  if (scheme == SCHEME_BX) {
    for (int k = 0; k < 4; ++k) theta[k] = bx;
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 4; ++k) out[i][k] = pl[i][k] + bx * (pn[i][k] - pl[i][k]);
  } else if (scheme == SCHEME_N) {
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 4; ++k) out[i][k] = pn[i][k];
  } else if (scheme == SCHEME_LDA) {
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 4; ++k) out[i][k] = pl[i][k];
  } else {
    blend_theta(res, pn, scheme, theta);
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 4; ++k) out[i][k] = pl[i][k] + theta[k] * (pn[i][k] - pl[i][k]);
  }
  if (theta_out)
    for (int k = 0; k < 4; ++k) theta_out[k] = theta[k];
}

template <class T> void corner_z(const Mesh& m, const std::vector<T>& Z, int64_t t, T Zc[3][4]) {
  for (int i = 0; i < 3; ++i) {
    int64_t v = m.tri[3 * t + i];
    for (int k = 0; k < 4; ++k) Zc[i][k] = Z[4 * v + k];
  }
}

template <class T> void corner_normals(const Mesh& m, int64_t t, double n[3][2]) {
  for (int i = 0; i < 3; ++i) {
    n[i][0] = m.nrm[6 * t + 2 * i];
    n[i][1] = m.nrm[6 * t + 2 * i + 1];
  }
}

// Wall correction residual (Section 3.5), per vertex, AoS [nv][4].
template <class T> void wall_term(const Mesh& m, const std::vector<T>& W, std::vector<T>& out) {
  const double alpha = 0.75, g1 = m.gamma - 1.0;
  out.assign(4 * m.nv, T(0.0));
  int64_t nw = (int64_t)m.wall.size() / 2;
  for (int64_t e = 0; e < nw; ++e) {
    int64_t ab[2] = {m.wall[2 * e], m.wall[2 * e + 1]};
    T F[2][4];
    for (int s = 0; s < 2; ++s) {
      const T* w = &W[4 * ab[s]];
      T u = w[1] / w[0], v = w[2] / w[0];
      T p = g1 * (w[3] - 0.5 * w[0] * (u * u + v * v));
      T vn = u * m.wnx[e] + v * m.wny[e];
      F[s][0] = -vn * w[0];
      F[s][1] = -vn * w[1];
      F[s][2] = -vn * w[2];
      F[s][3] = -vn * (w[3] + p);
    }
    const double hl = m.wlen[e] / 2.0;
    for (int k = 0; k < 4; ++k) {
      out[4 * ab[0] + k] += hl * (alpha * F[0][k] + (1.0 - alpha) * F[1][k]);
      out[4 * ab[1] + k] += hl * ((1.0 - alpha) * F[0][k] + alpha * F[1][k]);
    }
  }
}

// Sum per-triangle corner parts into vertices, ascending triangle order.
template <class T> void gather(const Mesh& m, const std::vector<T>& part, std::vector<T>& R) {
  R.assign(4 * m.nv, T(0.0));
  for (int64_t t = 0; t < m.nt; ++t)
    for (int i = 0; i < 3; ++i) {
      int64_t v = m.tri[3 * t + i];
      for (int k = 0; k < 4; ++k) R[4 * v + k] += part[12 * t + 4 * i + k];
    }
}

template <class T> void all_z(const Mesh& m, const std::vector<T>& W, std::vector<T>& Z) {
  Z.assign(4 * m.nv, T(0.0));
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m.nv; ++i) w_to_z(&W[4 * i], m.gamma, &Z[4 * i]);
}

// Smallest and largest flow speed |v| over the vertices of a state (Bx).
template <class T> void speed_range(const Mesh& m, const std::vector<T>& W, T& vmin, T& vmax) {
  for (int64_t i = 0; i < m.nv; ++i) {
    T u = W[4 * i + 1] / W[4 * i], v = W[4 * i + 2] / W[4 * i];
    T sp = sq_root(u * u + v * v);
    if (i == 0 || val(sp) < val(vmin)) vmin = sp;
    if (i == 0 || val(sp) > val(vmax)) vmax = sp;
  }
}

// Blend coefficient of the Bx scheme for triangle t at state W (Section
// 3.3.3): theta = min(1, s^2 h / L), s = (-L div v / (|v|max - |v|min))^+.
template <class T> T bx_theta(const Mesh& m, const std::vector<T>& W, int64_t t, T vmin, T vmax) {
  T div = T(0.0);
  for (int i = 0; i < 3; ++i) {
    int64_t v = m.tri[3 * t + i];
    T u = W[4 * v + 1] / W[4 * v], w = W[4 * v + 2] / W[4 * v];
    div = div + u * m.nrm[6 * t + 2 * i] + w * m.nrm[6 * t + 2 * i + 1];
  }
  div = div / (2.0 * m.area[t]);
  T range = vmax - vmin;
  T s = val(range) > 0.0 ? pos_part(-m.L * div / range) : T(0.0);
  const double h = std::sqrt(2.0 * m.area[t]);
  T theta = s * s * h / m.L;
  return val(theta) > 1.0 ? T(1.0) : theta;
}

// Stage-1 spatial parts of every triangle; optionally keeps phi^N and phi^T.
template <class T>
void spatial_parts(const Mesh& m, const std::vector<T>& W, const std::vector<T>& Z, int scheme,
                   std::vector<T>& part, std::vector<T>* keepN, std::vector<T>* keepT) {
  T vmin = T(0.0), vmax = T(0.0);
  if (scheme == SCHEME_BX) speed_range(m, W, vmin, vmax);
  part.assign(12 * m.nt, T(0.0));
  if (keepN) keepN->assign(12 * m.nt, T(0.0));
  if (keepT) keepT->assign(4 * m.nt, T(0.0));
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < m.nt; ++t) {
    T Zc[3][4];
    double n[3][2];
    corner_z(m, Z, t, Zc);
    corner_normals<T>(m, t, n);
    TriState<T> s;
    eval_triangle(Zc, n, m.gamma, s);
    T pl[3][4];
    for (int i = 0; i < 3; ++i) matvec(s.Kp[i], s.xL, pl[i]);
    T out[3][4];
    const T bx = scheme == SCHEME_BX ? bx_theta(m, W, t, vmin, vmax) : T(0.0);
    distribute(scheme, s.phiT, s.phiN, pl, out, (T*)nullptr, bx);
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 4; ++k) part[12 * t + 4 * i + k] = out[i][k];
    if (keepN)
      for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 4; ++k) (*keepN)[12 * t + 4 * i + k] = s.phiN[i][k];
    if (keepT)
      for (int k = 0; k < 4; ++k) (*keepT)[4 * t + k] = s.phiT[k];
  }
}

// One step of Section 3.4: forward Euler (time_order 1) or the two-stage RK
// scheme (time_order 2). W is AoS [nv][4] in and out.
template <class T> void step(const Mesh& m, std::vector<T>& W, double dt, int scheme, int time_order) {
  std::vector<T> Z, part, keepN, keepT, R, Wc_n;
  all_z(m, W, Z);
  spatial_parts<T>(m, W, Z, scheme, part, time_order == 2 ? &keepN : nullptr, time_order == 2 ? &keepT : nullptr);
  gather(m, part, R);
  wall_term(m, W, Wc_n);
  std::vector<T> Ws(W);
  for (int64_t i = 0; i < m.nv; ++i) {
    if (m.ghost[i]) continue;
    for (int k = 0; k < 4; ++k) {
      T r = R[4 * i + k] + Wc_n[4 * i + k];
      Ws[4 * i + k] = W[4 * i + k] - (dt / m.V[i]) * r;
    }
  }
  if (time_order == 1) {
    W.swap(Ws);
    return;
  }
  std::vector<T> Zs;
  all_z(m, Ws, Zs);
  T vmin = T(0.0), vmax = T(0.0);
  if (scheme == SCHEME_BX) speed_range(m, Ws, vmin, vmax);
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < m.nt; ++t) {
    T Zc[3][4];
    double n[3][2];
    corner_z(m, Zs, t, Zc);
    corner_normals<T>(m, t, n);
    TriState<T> s;
    eval_triangle(Zc, n, m.gamma, s);
    const double mass = m.area[t] / 3.0;
    T rate[3][4];
    for (int i = 0; i < 3; ++i) {
      int64_t v = m.tri[3 * t + i];
      for (int k = 0; k < 4; ++k) rate[i][k] = (Ws[4 * v + k] - W[4 * v + k]) / dt;
    }
    T PN[3][4], PT[4];
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 4; ++k)
        PN[i][k] = mass * rate[i][k] + 0.5 * (keepN[12 * t + 4 * i + k] + s.phiN[i][k]);
    for (int k = 0; k < 4; ++k)
      PT[k] = mass * (rate[0][k] + rate[1][k] + rate[2][k]) + 0.5 * (keepT[4 * t + k] + s.phiT[k]);
    T x[4];
    solve4(s.A, PT, x);
    T PL[3][4];
    for (int i = 0; i < 3; ++i) matvec(s.Kp[i], x, PL[i]);
    if (m.selective) {
      // selective lumping: + sum_j (|T| delta_ij / 3 - m^G_ij) (W*_j - W^n_j) / dt
      for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 4; ++k) {
          T sl = T(0.0);
          for (int j = 0; j < 3; ++j) {
            const double mg = m.area[t] * ((i == j ? 1.0 : 0.0) + 1.0) / 12.0;
            const double ml = i == j ? m.area[t] / 3.0 : 0.0;
            sl = sl + (ml - mg) * rate[j][k];
          }
          PN[i][k] = PN[i][k] + sl;
          PL[i][k] = PL[i][k] + sl;
        }
    }
    T out[3][4];
    const T bx = scheme == SCHEME_BX ? bx_theta(m, Ws, t, vmin, vmax) : T(0.0);
    distribute(scheme, PT, PN, PL, out, (T*)nullptr, bx);
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 4; ++k) part[12 * t + 4 * i + k] = out[i][k];
  }
  gather(m, part, R);
  std::vector<T> Wc_s;
  wall_term(m, Ws, Wc_s);
  for (int64_t i = 0; i < m.nv; ++i) {
    if (m.ghost[i]) continue;
    for (int k = 0; k < 4; ++k) {
      T r = R[4 * i + k] + 0.5 * (Wc_n[4 * i + k] + Wc_s[4 * i + k]);
      W[4 * i + k] = Ws[4 * i + k] - (dt / m.V[i]) * r;
    }
  }
}

void soa_to_aos(const Mesh& m, const double* soa, std::vector<double>& aos) {
  aos.resize(4 * m.nv);
  for (int64_t i = 0; i < m.nv; ++i)
    for (int k = 0; k < 4; ++k) aos[4 * i + k] = soa[k * m.nv + i];
}
void aos_to_soa(const Mesh& m, const std::vector<double>& aos, double* soa) {
  for (int64_t i = 0; i < m.nv; ++i)
    for (int k = 0; k < 4; ++k) soa[k * m.nv + i] = aos[4 * i + k];
}

}  // namespace

// ------------------------------------------------------------- C API ------
// Arrays of states are structure-of-arrays [4][nv] (rho, rho u, rho v, e).
extern "C" {

void* rdo_mesh_new(int64_t nv, int64_t nt, const double* x, const double* y, const int32_t* tri,
                   double px, double py, const uint8_t* ghost, int64_t n_wall, const int32_t* wall,
                   double gamma, char* err, int errlen) {
  Mesh* m = new Mesh();
  m->nv = nv;
  m->nt = nt;
  m->x.assign(x, x + nv);
  m->y.assign(y, y + nv);
  m->tri.assign(tri, tri + 3 * nt);
  m->px = px;
  m->py = py;
  m->ghost.assign(nv, 0);
  if (ghost) m->ghost.assign(ghost, ghost + nv);
  if (n_wall > 0) m->wall.assign(wall, wall + 2 * n_wall);
  m->gamma = gamma;
  std::string e;
  if (nv <= 0 || nt <= 0) e = "empty mesh";
  if (e.empty() && !(gamma > 1.0)) e = "gamma must exceed 1";
  if (e.empty()) build_geometry(*m, e);
  if (!e.empty()) {
    if (err && errlen > 0) std::snprintf(err, errlen, "%s", e.c_str());
    delete m;
    return nullptr;
  }
  return m;
}

void rdo_mesh_free(void* h) { delete static_cast<Mesh*>(h); }

// Lumping of the stage-2 mass term: 0 global (default), 1 selective.
void rdo_set_lumping(void* h, int selective) { static_cast<Mesh*>(h)->selective = selective != 0; }

// Domain size L of the Bx sensor.
double rdo_domain_size(void* h) { return static_cast<Mesh*>(h)->L; }

void rdo_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int rdo_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// area [nt], normals [nt][3][2], longest edge [nt], vertex volume [nv]
void rdo_geometry(void* h, double* area, double* nrm, double* lmax, double* V) {
  const Mesh& m = *static_cast<Mesh*>(h);
  std::memcpy(area, m.area.data(), sizeof(double) * m.nt);
  std::memcpy(nrm, m.nrm.data(), sizeof(double) * 6 * m.nt);
  std::memcpy(lmax, m.lmax.data(), sizeof(double) * m.nt);
  std::memcpy(V, m.V.data(), sizeof(double) * m.nv);
}

// Spatial residual of every vertex: sum of the scheme's parts over its
// triangles plus the wall term, R [4][nv]; triangle residuals phiT [4][nt]
// (may be NULL).
int rdo_residual(void* h, const double* W_soa, int scheme, double* R_soa, double* phiT_soa) {
  const Mesh& m = *static_cast<Mesh*>(h);
  if (scheme < 0 || scheme > 5) return 1;
  std::vector<double> W, Z, part, keepT, R, Wc;
  soa_to_aos(m, W_soa, W);
  all_z(m, W, Z);
  spatial_parts<double>(m, W, Z, scheme, part, nullptr, &keepT);
  gather(m, part, R);
  wall_term(m, W, Wc);
  for (int64_t i = 0; i < 4 * m.nv; ++i) R[i] = R[i] + Wc[i];
  aos_to_soa(m, R, R_soa);
  if (phiT_soa)
    for (int64_t t = 0; t < m.nt; ++t)
      for (int k = 0; k < 4; ++k) phiT_soa[k * m.nt + t] = keepT[4 * t + k];
  return 0;
}

// Per-triangle corner parts of a scheme at a state, [nt][3][4].
int rdo_parts(void* h, const double* W_soa, int scheme, double* parts) {
  const Mesh& m = *static_cast<Mesh*>(h);
  if (scheme < 0 || scheme > 5) return 1;
  std::vector<double> W, Z, part;
  soa_to_aos(m, W_soa, W);
  all_z(m, W, Z);
  spatial_parts<double>(m, W, Z, scheme, part, nullptr, nullptr);
  std::memcpy(parts, part.data(), sizeof(double) * 12 * m.nt);
  return 0;
}

int rdo_step(void* h, double* W_soa, double dt, int scheme, int time_order) {
  const Mesh& m = *static_cast<Mesh*>(h);
  if (scheme < 0 || scheme > 5 || (time_order != 1 && time_order != 2) || !(dt > 0.0)) return 1;
  std::vector<double> W;
  soa_to_aos(m, W_soa, W);
  step(m, W, dt, scheme, time_order);
  aos_to_soa(m, W, W_soa);
  return 0;
}

// Forward-mode derivative of one step: on return W holds the new state and
// dW the Jacobian of the step applied to the incoming dW (dt held fixed).
int rdo_step_jvp(void* h, double* W_soa, double* dW_soa, double dt, int scheme, int time_order) {
  const Mesh& m = *static_cast<Mesh*>(h);
  if (scheme < 0 || scheme > 5 || (time_order != 1 && time_order != 2) || !(dt > 0.0)) return 1;
  std::vector<Dual> W(4 * m.nv);
  for (int64_t i = 0; i < m.nv; ++i)
    for (int k = 0; k < 4; ++k) W[4 * i + k] = Dual(W_soa[k * m.nv + i], dW_soa[k * m.nv + i]);
  step(m, W, dt, scheme, time_order);
  for (int64_t i = 0; i < m.nv; ++i)
    for (int k = 0; k < 4; ++k) {
      W_soa[k * m.nv + i] = W[4 * i + k].v;
      dW_soa[k * m.nv + i] = W[4 * i + k].d;
    }
  return 0;
}

// CFL limit of Section 3.2 times `cfl`.
double rdo_max_dt(void* h, const double* W_soa, double cfl) {
  const Mesh& m = *static_cast<Mesh*>(h);
  std::vector<double> sig(m.nv), acc(m.nv, 0.0);
  for (int64_t i = 0; i < m.nv; ++i) {
    double rho = W_soa[i], u = W_soa[m.nv + i] / rho, v = W_soa[2 * m.nv + i] / rho;
    double p = (m.gamma - 1.0) * (W_soa[3 * m.nv + i] - 0.5 * rho * (u * u + v * v));
    sig[i] = std::sqrt(u * u + v * v) + std::sqrt(m.gamma * p / rho);
  }
  for (int64_t t = 0; t < m.nt; ++t) {
    double lam = 0.0;
    for (int i = 0; i < 3; ++i) lam = std::max(lam, sig[m.tri[3 * t + i]]);
    for (int i = 0; i < 3; ++i) acc[m.tri[3 * t + i]] += m.lmax[t] * lam;
  }
  double best = INFINITY;
  for (int64_t i = 0; i < m.nv; ++i) best = std::min(best, 2.0 * m.V[i] / acc[i]);
  return cfl * best;
}

// One triangle in isolation, for unit checks. W3: corner states [3][4]
// (conserved); xy: corner positions [3][2] (already unwrapped, CCW).
// out: phiT[4], phiN[3][4], phiLDA[3][4], phiB[3][4], Theta[4] (52 values).
int rdo_triangle(const double* W3, const double* xy, double gamma, int scheme, double* out) {
  double Zc[3][4];
  for (int i = 0; i < 3; ++i) w_to_z(&W3[4 * i], gamma, Zc[i]);
  double n[3][2];
  for (int i = 0; i < 3; ++i) {
    const double* pa = &xy[2 * ((i + 1) % 3)];
    const double* pb = &xy[2 * ((i + 2) % 3)];
    n[i][0] = -(pb[1] - pa[1]);
    n[i][1] = pb[0] - pa[0];
  }
  TriState<double> s;
  eval_triangle(Zc, n, gamma, s);
  double pl[3][4], pb[3][4], theta[4];
  for (int i = 0; i < 3; ++i) matvec(s.Kp[i], s.xL, pl[i]);
  int sch = (scheme >= SCHEME_B && scheme <= SCHEME_BMIN) ? scheme : SCHEME_B;
  distribute(sch, s.phiT, s.phiN, pl, pb, theta);
  double* o = out;
  for (int k = 0; k < 4; ++k) *o++ = s.phiT[k];
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 4; ++k) *o++ = s.phiN[i][k];
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 4; ++k) *o++ = pl[i][k];
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 4; ++k) *o++ = pb[i][k];
  for (int k = 0; k < 4; ++k) *o++ = theta[k];
  return 0;
}

// K, K^+, K^- (row-major 4x4) for the state W (conserved) and a normal n
// scaled by the edge length, with the factor 1/2 of Section 3.2 included.
void rdo_kmat(const double* W, double nx, double ny, double gamma, double* K, double* Kp, double* Km) {
  double u = W[1] / W[0], v = W[2] / W[0];
  double p = (gamma - 1.0) * (W[3] - 0.5 * W[0] * (u * u + v * v));
  double h = (W[3] + p) / W[0];
  double c = std::sqrt(gamma * p / W[0]);
  double len = std::sqrt(nx * nx + ny * ny);
  double ux = nx / len, uy = ny / len;
  double w = u * ux + v * uy;
  double lam[3] = {w + c, w - c, w}, lp[3], lm[3];
  for (int k = 0; k < 3; ++k) { lp[k] = pos_part(lam[k]); lm[k] = neg_part(lam[k]); }
  double M[4][4];
  double* outs[3] = {K, Kp, Km};
  const double* ls[3] = {lam, lp, lm};
  for (int q = 0; q < 3; ++q) {
    k_entries(u, v, h, c, gamma, ux, uy, ls[q][0], ls[q][1], ls[q][2], M);
    for (int r = 0; r < 4; ++r)
      for (int s = 0; s < 4; ++s) outs[q][4 * r + s] = (len / 2.0) * M[r][s];
  }
}

// The pivoted solve on its own, for unit checks: x = A^{-1} b, row-major A.
void rdo_solve4(const double* A, const double* b, double* x) {
  double M[4][4];
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) M[r][c] = A[4 * r + c];
  solve4(M, b, x);
}

}  // extern "C"
