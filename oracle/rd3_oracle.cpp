// Plain CPU oracle for the residual-distribution step generalised to three
// dimensions on tetrahedral meshes (Paardekooper 2017: Section 3 gives the
// method in two dimensions; its closing discussion states that it extends to
// three by adding a row and a column to every matrix).
//
// TEST INFRASTRUCTURE ONLY. This file is the independent reference the GPU
// library's three-dimensional path is checked against. It shares no code,
// header or table with the GPU path (nor with the two-dimensional oracle);
// only the tests and the benchmark's CPU-baseline leg load it. It follows the
// method step by step in IEEE FP64, built without FMA contraction.
//
// Readings (each also listed in the design notes of the repository):
//  * State W = (rho, rho u, rho v, rho w, e); parameter vector
//    Z = sqrt(rho) (1, u, v, w, h).
//  * K_i = (|n_i| / 3) K(n_i / |n_i|): n_i is the inward normal of the face
//    opposite corner i scaled by the face's area (the gradient of a linear
//    function on a tetrahedron is sum_i f_i n_i / (3 |T|)), so 1/d = 1/3.
//  * K(n) for a unit normal is R diag(l) R^{-1} with the eigenvectors of the
//    Euler flux Jacobian along n: the acoustic waves (1, u -+ c n, H -+ c u.n)
//    with l = u.n -+ c, the entropy wave (1, u, |u|^2 / 2) and two shear
//    waves (0, t, u.t) for an orthonormal pair of tangents t, all with
//    l = u.n. l = lambda gives K, l = lambda^{+-} gives K^{+-}; R^{-1} is
//    computed by Gaussian elimination.
//  * The state differences the K matrices act on are dW_i = M(Zbar)(Z_i-Z_0),
//    M = dW/dZ at the mean Zbar of the four corners.
//  * N, LDA and the B blends as in two dimensions with four corners and five
//    components: A = sum K^+, A x = b solved by Gaussian elimination with
//    partial pivoting, a column whose best pivot is at most 2^-45 max|A|
//    skipped (its unknown is 0); Theta_k = |phi^T_k| / sum_i |phi^N_{i,k}|
//    (0 for a zero denominator, at most 1).
//  * Vertex volume V_i = sum of |T| / 4 over the tetrahedra of i (median
//    dual, global lumping); RK2 with the mass |T| / 4 per corner, stage-1
//    phi^N and phi^T kept, the LDA coefficients of stage 2 at W*.
//  * CFL limit dt_i = 3 V_i / sum_T (S_T lambda_T) with S_T the largest face
//    area of T and lambda_T the largest |u| + c at its corners (the bound of
//    the two-dimensional case with the edge length replaced by a face area
//    and 1/2 by 1/3).
//  * Periodic boxes only (every axis periodic or not, no wall or ghost
//    vertices); coordinates are unwrapped to the minimum image of corner 0.
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

enum { SCHEME_N = 0, SCHEME_LDA = 1, SCHEME_B = 2, SCHEME_BMAX = 3, SCHEME_BMIN = 4 };

struct Mesh {
  int64_t nv = 0, nt = 0;
  std::vector<double> x, y, z;
  std::vector<int32_t> tet;  // [nt][4]
  double px = 0.0, py = 0.0, pz = 0.0;
  double gamma = 1.4;
  std::vector<double> vol;   // |T|
  std::vector<double> nrm;   // inward face normals scaled by face area, [nt][4][3]
  std::vector<double> smax;  // largest face area
  std::vector<double> V;     // vertex volume
};

double unwrap(double d, double period) {
  if (period > 0.0) {
    if (d > 0.5 * period) d -= period;
    else if (d < -0.5 * period) d += period;
  }
  return d;
}

void cross(const double a[3], const double b[3], double c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

bool build_geometry(Mesh& m, std::string& err) {
  m.vol.assign(m.nt, 0.0);
  m.nrm.assign(12 * m.nt, 0.0);
  m.smax.assign(m.nt, 0.0);
  m.V.assign(m.nv, 0.0);
  for (int64_t t = 0; t < m.nt; ++t) {
    int32_t v[4];
    for (int k = 0; k < 4; ++k) {
      v[k] = m.tet[4 * t + k];
      if (v[k] < 0 || v[k] >= m.nv) {
        err = "tetrahedron " + std::to_string(t) + " has a vertex index out of range";
        return false;
      }
    }
    double p[4][3] = {};
    for (int k = 1; k < 4; ++k) {
      p[k][0] = unwrap(m.x[v[k]] - m.x[v[0]], m.px);
      p[k][1] = unwrap(m.y[v[k]] - m.y[v[0]], m.py);
      p[k][2] = unwrap(m.z[v[k]] - m.z[v[0]], m.pz);
    }
    double c[3];
    cross(p[2], p[3], c);
    const double vol = dot3(p[1], c) / 6.0;
    if (!(vol > 0.0)) {
      err = "tetrahedron " + std::to_string(t) + " is not positively oriented";
      return false;
    }
    m.vol[t] = vol;
    double smax = 0.0;
    for (int i = 0; i < 4; ++i) {
      const double* a = p[(i + 1) % 4];
      const double* b = p[(i + 2) % 4];
      const double* d = p[(i + 3) % 4];
      double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
      double e2[3] = {d[0] - a[0], d[1] - a[1], d[2] - a[2]};
      double n[3];
      cross(e1, e2, n);
      for (int k = 0; k < 3; ++k) n[k] *= 0.5;  // |n| = face area
      double toward[3] = {p[i][0] - a[0], p[i][1] - a[1], p[i][2] - a[2]};
      if (dot3(n, toward) < 0.0)
        for (int k = 0; k < 3; ++k) n[k] = -n[k];
      for (int k = 0; k < 3; ++k) m.nrm[12 * t + 3 * i + k] = n[k];
      smax = std::max(smax, std::sqrt(dot3(n, n)));
    }
    m.smax[t] = smax;
  }
  for (int64_t t = 0; t < m.nt; ++t)
    for (int k = 0; k < 4; ++k) m.V[m.tet[4 * t + k]] += m.vol[t] / 4.0;
  for (int64_t i = 0; i < m.nv; ++i)
    if (!(m.V[i] > 0.0)) {
      err = "vertex " + std::to_string(i) + " belongs to no tetrahedron";
      return false;
    }
  return true;
}

// Z = sqrt(rho) (1, u, v, w, h).
void w_to_z(const double W[5], double gamma, double Z[5]) {
  const double rho = W[0], u = W[1] / rho, v = W[2] / rho, w = W[3] / rho;
  const double p = (gamma - 1.0) * (W[4] - 0.5 * rho * (u * u + v * v + w * w));
  const double h = (W[4] + p) / rho;
  const double s = std::sqrt(rho);
  Z[0] = s;
  Z[1] = s * u;
  Z[2] = s * v;
  Z[3] = s * w;
  Z[4] = s * h;
}

// Gaussian elimination with partial pivoting; the skip rule of the
// two-dimensional oracle for (near-)singular columns.
void solve5(const double Ain[5][5], const double b_in[5], double x[5]) {
  double A[5][5], b[5], amax = 0.0;
  for (int r = 0; r < 5; ++r) {
    b[r] = b_in[r];
    for (int c = 0; c < 5; ++c) {
      A[r][c] = Ain[r][c];
      amax = std::max(amax, std::fabs(A[r][c]));
    }
  }
  const double tol = std::ldexp(amax, -45);
  bool used[5] = {false, false, false, false, false};
  int prow[5] = {-1, -1, -1, -1, -1};
  for (int k = 0; k < 5; ++k) {
    int r = -1;
    double best = -1.0;
    for (int i = 0; i < 5; ++i) {
      if (used[i]) continue;
      if (std::fabs(A[i][k]) > best) {
        best = std::fabs(A[i][k]);
        r = i;
      }
    }
    if (r < 0 || !(best > tol)) continue;
    used[r] = true;
    prow[k] = r;
    for (int i = 0; i < 5; ++i) {
      if (used[i]) continue;
      const double f = A[i][k] / A[r][k];
      for (int j = k; j < 5; ++j) A[i][j] -= f * A[r][j];
      b[i] -= f * b[r];
    }
  }
  for (int k = 4; k >= 0; --k) {
    if (prow[k] < 0) {
      x[k] = 0.0;
      continue;
    }
    const int r = prow[k];
    double s = b[r];
    for (int j = k + 1; j < 5; ++j) s -= A[r][j] * x[j];
    x[k] = s / A[r][k];
  }
}

// Inverse of a 5x5 matrix by Gauss-Jordan elimination with partial pivoting.
void invert5(const double Ain[5][5], double inv[5][5]) {
  double A[5][10];
  for (int r = 0; r < 5; ++r)
    for (int c = 0; c < 10; ++c) A[r][c] = c < 5 ? Ain[r][c] : (c - 5 == r ? 1.0 : 0.0);
  for (int k = 0; k < 5; ++k) {
    int p = k;
    for (int i = k + 1; i < 5; ++i)
      if (std::fabs(A[i][k]) > std::fabs(A[p][k])) p = i;
    for (int c = 0; c < 10; ++c) std::swap(A[k][c], A[p][c]);
    const double d = A[k][k];
    for (int c = 0; c < 10; ++c) A[k][c] /= d;
    for (int i = 0; i < 5; ++i) {
      if (i == k) continue;
      const double f = A[i][k];
      for (int c = 0; c < 10; ++c) A[i][c] -= f * A[k][c];
    }
  }
  for (int r = 0; r < 5; ++r)
    for (int c = 0; c < 5; ++c) inv[r][c] = A[r][c + 5];
}

// Right eigenvectors (columns) of the Euler flux Jacobian along the unit
// normal n at (u, H, c), in the order of the eigenvalues
// (u.n - c, u.n, u.n, u.n, u.n + c).
void eigenvectors(const double u[3], double H, double c, const double n[3], double R[5][5]) {
  // tangents: t1 perpendicular to n and to the axis n is least aligned with
  int axis = 0;
  for (int k = 1; k < 3; ++k)
    if (std::fabs(n[k]) < std::fabs(n[axis])) axis = k;
  double e[3] = {0.0, 0.0, 0.0};
  e[axis] = 1.0;
  double t1[3], t2[3];
  cross(n, e, t1);
  const double l1 = std::sqrt(dot3(t1, t1));
  for (int k = 0; k < 3; ++k) t1[k] /= l1;
  cross(n, t1, t2);
  const double un = dot3(u, n), q2 = dot3(u, u);
  double col[5][5];
  col[0][0] = 1.0;
  col[4][0] = 1.0;
  col[1][0] = 1.0;
  for (int k = 0; k < 3; ++k) {
    col[0][1 + k] = u[k] - c * n[k];
    col[4][1 + k] = u[k] + c * n[k];
    col[1][1 + k] = u[k];
    col[2][1 + k] = t1[k];
    col[3][1 + k] = t2[k];
  }
  col[0][4] = H - c * un;
  col[4][4] = H + c * un;
  col[1][4] = 0.5 * q2;
  col[2][0] = 0.0;
  col[3][0] = 0.0;
  col[2][4] = dot3(u, t1);
  col[3][4] = dot3(u, t2);
  for (int r = 0; r < 5; ++r)
    for (int j = 0; j < 5; ++j) R[r][j] = col[j][r];
}

// K = R diag(l) R^{-1}.
void kmat(const double R[5][5], const double L[5][5], const double l[5], double K[5][5]) {
  for (int r = 0; r < 5; ++r)
    for (int q = 0; q < 5; ++q) {
      double s = 0.0;
      for (int j = 0; j < 5; ++j) s += R[r][j] * l[j] * L[j][q];
      K[r][q] = s;
    }
}

void matvec(const double M[5][5], const double x[5], double y[5]) {
  for (int r = 0; r < 5; ++r) {
    double s = 0.0;
    for (int q = 0; q < 5; ++q) s += M[r][q] * x[q];
    y[r] = s;
  }
}

struct TetState {
  double dW[4][5];
  double K[4][5][5], Kp[4][5][5], Km[4][5][5];
  double A[5][5];
  double phiT[5];
  double phiN[4][5];
  double xL[5];
};

// Section 3.2-3.3 for one tetrahedron.
void eval_tet(const double Zc[4][5], const double n[4][3], double gamma, TetState& s) {
  const double g1 = gamma - 1.0;
  double zb[5];
  for (int k = 0; k < 5; ++k) zb[k] = (Zc[0][k] + Zc[1][k] + Zc[2][k] + Zc[3][k]) / 4.0;
  const double u[3] = {zb[1] / zb[0], zb[2] / zb[0], zb[3] / zb[0]};
  const double H = zb[4] / zb[0];
  const double c = std::sqrt(g1 * (H - 0.5 * dot3(u, u)));
  for (int k = 0; k < 5; ++k) s.dW[0][k] = 0.0;
  for (int i = 1; i < 4; ++i) {
    double dz[5];
    for (int k = 0; k < 5; ++k) dz[k] = Zc[i][k] - Zc[0][k];
    s.dW[i][0] = 2.0 * zb[0] * dz[0];
    for (int k = 1; k < 4; ++k) s.dW[i][k] = zb[k] * dz[0] + zb[0] * dz[k];
    s.dW[i][4] = (zb[4] * dz[0] + g1 * (zb[1] * dz[1] + zb[2] * dz[2] + zb[3] * dz[3]) + zb[0] * dz[4]) / gamma;
  }
  for (int i = 0; i < 4; ++i) {
    const double area = std::sqrt(dot3(n[i], n[i]));
    const double nh[3] = {n[i][0] / area, n[i][1] / area, n[i][2] / area};
    const double un = dot3(u, nh);
    const double lam[5] = {un - c, un, un, un, un + c};
    double lp[5], lm[5];
    for (int k = 0; k < 5; ++k) {
      lp[k] = lam[k] > 0.0 ? lam[k] : 0.0;
      lm[k] = lam[k] < 0.0 ? lam[k] : 0.0;
    }
    double R[5][5], L[5][5];
    eigenvectors(u, H, c, nh, R);
    invert5(R, L);
    kmat(R, L, lam, s.K[i]);
    kmat(R, L, lp, s.Kp[i]);
    kmat(R, L, lm, s.Km[i]);
    const double third = area / 3.0;
    for (int r = 0; r < 5; ++r)
      for (int q = 0; q < 5; ++q) {
        s.K[i][r][q] *= third;
        s.Kp[i][r][q] *= third;
        s.Km[i][r][q] *= third;
      }
  }
  for (int k = 0; k < 5; ++k) s.phiT[k] = 0.0;
  double bN[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int i = 1; i < 4; ++i) {
    double t1[5], t2[5];
    matvec(s.K[i], s.dW[i], t1);
    matvec(s.Km[i], s.dW[i], t2);
    for (int k = 0; k < 5; ++k) {
      s.phiT[k] += t1[k];
      bN[k] += t2[k];
    }
  }
  for (int r = 0; r < 5; ++r)
    for (int q = 0; q < 5; ++q) s.A[r][q] = s.Kp[0][r][q] + s.Kp[1][r][q] + s.Kp[2][r][q] + s.Kp[3][r][q];
  double xN[5];
  solve5(s.A, bN, xN);
  solve5(s.A, s.phiT, s.xL);
  for (int i = 0; i < 4; ++i) {
    double y[5];
    for (int k = 0; k < 5; ++k) y[k] = s.dW[i][k] + xN[k];
    matvec(s.Kp[i], y, s.phiN[i]);
  }
}

void blend_theta(const double res[5], const double pn[4][5], int scheme, double theta[5]) {
  for (int k = 0; k < 5; ++k) {
    const double den = std::fabs(pn[0][k]) + std::fabs(pn[1][k]) + std::fabs(pn[2][k]) + std::fabs(pn[3][k]);
    if (den == 0.0) {
      theta[k] = 0.0;
    } else {
      const double q = std::fabs(res[k]) / den;
      theta[k] = q > 1.0 ? 1.0 : q;
    }
  }
  if (scheme == SCHEME_BMAX || scheme == SCHEME_BMIN) {
    int pick = 0;
    for (int k = 1; k < 5; ++k) {
      const bool better = scheme == SCHEME_BMAX ? theta[k] > theta[pick] : theta[k] < theta[pick];
      if (better) pick = k;
    }
    for (int k = 0; k < 5; ++k) theta[k] = theta[pick];
  }
}

void distribute(int scheme, const double res[5], const double pn[4][5], const double pl[4][5], double out[4][5],
                double theta_out[5]) {
  double theta[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (scheme == SCHEME_N) {
    for (int k = 0; k < 5; ++k) theta[k] = 1.0;
  } else if (scheme != SCHEME_LDA) {
    blend_theta(res, pn, scheme, theta);
  }
  for (int i = 0; i < 4; ++i)
    for (int k = 0; k < 5; ++k) out[i][k] = pl[i][k] + theta[k] * (pn[i][k] - pl[i][k]);
  if (scheme == SCHEME_N)
    for (int i = 0; i < 4; ++i)
      for (int k = 0; k < 5; ++k) out[i][k] = pn[i][k];
  if (theta_out)
    for (int k = 0; k < 5; ++k) theta_out[k] = theta[k];
}

void corner_data(const Mesh& m, const std::vector<double>& Z, int64_t t, double Zc[4][5], double n[4][3]) {
  for (int i = 0; i < 4; ++i) {
    const int64_t v = m.tet[4 * t + i];
    for (int k = 0; k < 5; ++k) Zc[i][k] = Z[5 * v + k];
    for (int k = 0; k < 3; ++k) n[i][k] = m.nrm[12 * t + 3 * i + k];
  }
}

void all_z(const Mesh& m, const std::vector<double>& W, std::vector<double>& Z) {
  Z.assign(5 * m.nv, 0.0);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m.nv; ++i) w_to_z(&W[5 * i], m.gamma, &Z[5 * i]);
}

// Sum corner parts into vertices in ascending tetrahedron order.
void gather(const Mesh& m, const std::vector<double>& part, std::vector<double>& R) {
  R.assign(5 * m.nv, 0.0);
  for (int64_t t = 0; t < m.nt; ++t)
    for (int i = 0; i < 4; ++i) {
      const int64_t v = m.tet[4 * t + i];
      for (int k = 0; k < 5; ++k) R[5 * v + k] += part[20 * t + 5 * i + k];
    }
}

void spatial_parts(const Mesh& m, const std::vector<double>& Z, int scheme, std::vector<double>& part,
                   std::vector<double>* keepN, std::vector<double>* keepT) {
  part.assign(20 * m.nt, 0.0);
  if (keepN) keepN->assign(20 * m.nt, 0.0);
  if (keepT) keepT->assign(5 * m.nt, 0.0);
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < m.nt; ++t) {
    double Zc[4][5], n[4][3];
    corner_data(m, Z, t, Zc, n);
    TetState s;
    eval_tet(Zc, n, m.gamma, s);
    double pl[4][5], out[4][5];
    for (int i = 0; i < 4; ++i) matvec(s.Kp[i], s.xL, pl[i]);
    distribute(scheme, s.phiT, s.phiN, pl, out, nullptr);
    for (int i = 0; i < 4; ++i)
      for (int k = 0; k < 5; ++k) part[20 * t + 5 * i + k] = out[i][k];
    if (keepN)
      for (int i = 0; i < 4; ++i)
        for (int k = 0; k < 5; ++k) (*keepN)[20 * t + 5 * i + k] = s.phiN[i][k];
    if (keepT)
      for (int k = 0; k < 5; ++k) (*keepT)[5 * t + k] = s.phiT[k];
  }
}

// One step: forward Euler (order 1) or the two-stage scheme (order 2). W is
// AoS [nv][5].
void step(const Mesh& m, std::vector<double>& W, double dt, int scheme, int order) {
  std::vector<double> Z, part, keepN, keepT, R;
  all_z(m, W, Z);
  spatial_parts(m, Z, scheme, part, order == 2 ? &keepN : nullptr, order == 2 ? &keepT : nullptr);
  gather(m, part, R);
  std::vector<double> Ws(W);
  for (int64_t i = 0; i < m.nv; ++i)
    for (int k = 0; k < 5; ++k) Ws[5 * i + k] = W[5 * i + k] - (dt / m.V[i]) * R[5 * i + k];
  if (order == 1) {
    W.swap(Ws);
    return;
  }
  std::vector<double> Zs;
  all_z(m, Ws, Zs);
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < m.nt; ++t) {
    double Zc[4][5], n[4][3];
    corner_data(m, Zs, t, Zc, n);
    TetState s;
    eval_tet(Zc, n, m.gamma, s);
    const double mass = m.vol[t] / 4.0;
    double rate[4][5];
    for (int i = 0; i < 4; ++i) {
      const int64_t v = m.tet[4 * t + i];
      for (int k = 0; k < 5; ++k) rate[i][k] = (Ws[5 * v + k] - W[5 * v + k]) / dt;
    }
    double PN[4][5], PT[5];
    for (int i = 0; i < 4; ++i)
      for (int k = 0; k < 5; ++k) PN[i][k] = mass * rate[i][k] + 0.5 * (keepN[20 * t + 5 * i + k] + s.phiN[i][k]);
    for (int k = 0; k < 5; ++k)
      PT[k] = mass * (rate[0][k] + rate[1][k] + rate[2][k] + rate[3][k]) + 0.5 * (keepT[5 * t + k] + s.phiT[k]);
    double x[5];
    solve5(s.A, PT, x);
    double PL[4][5], out[4][5];
    for (int i = 0; i < 4; ++i) matvec(s.Kp[i], x, PL[i]);
    distribute(scheme, PT, PN, PL, out, nullptr);
    for (int i = 0; i < 4; ++i)
      for (int k = 0; k < 5; ++k) part[20 * t + 5 * i + k] = out[i][k];
  }
  gather(m, part, R);
  for (int64_t i = 0; i < m.nv; ++i)
    for (int k = 0; k < 5; ++k) W[5 * i + k] = Ws[5 * i + k] - (dt / m.V[i]) * R[5 * i + k];
}

void soa_to_aos(const Mesh& m, const double* soa, std::vector<double>& aos) {
  aos.resize(5 * m.nv);
  for (int64_t i = 0; i < m.nv; ++i)
    for (int k = 0; k < 5; ++k) aos[5 * i + k] = soa[k * m.nv + i];
}
void aos_to_soa(const Mesh& m, const std::vector<double>& aos, double* soa) {
  for (int64_t i = 0; i < m.nv; ++i)
    for (int k = 0; k < 5; ++k) soa[k * m.nv + i] = aos[5 * i + k];
}

}  // namespace

// ------------------------------------------------------------- C API ------
// States are structure-of-arrays [5][nv] (rho, rho u, rho v, rho w, e).
extern "C" {

void* rdo3_mesh_new(int64_t nv, int64_t nt, const double* x, const double* y, const double* z, const int32_t* tet,
                    double px, double py, double pz, double gamma, char* err, int errlen) {
  Mesh* m = new Mesh();
  m->nv = nv;
  m->nt = nt;
  m->x.assign(x, x + nv);
  m->y.assign(y, y + nv);
  m->z.assign(z, z + nv);
  m->tet.assign(tet, tet + 4 * nt);
  m->px = px;
  m->py = py;
  m->pz = pz;
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

void rdo3_mesh_free(void* h) { delete static_cast<Mesh*>(h); }

// vol [nt], normals [nt][4][3], largest face area [nt], vertex volume [nv]
void rdo3_geometry(void* h, double* vol, double* nrm, double* smax, double* V) {
  const Mesh& m = *static_cast<Mesh*>(h);
  std::memcpy(vol, m.vol.data(), sizeof(double) * m.nt);
  std::memcpy(nrm, m.nrm.data(), sizeof(double) * 12 * m.nt);
  std::memcpy(smax, m.smax.data(), sizeof(double) * m.nt);
  std::memcpy(V, m.V.data(), sizeof(double) * m.nv);
}

// Vertex sums of the stage-1 parts of a scheme (the spatial residual).
void rdo3_residual(void* h, const double* W_soa, int scheme, double* R_soa) {
  const Mesh& m = *static_cast<Mesh*>(h);
  std::vector<double> W, Z, part, R;
  soa_to_aos(m, W_soa, W);
  all_z(m, W, Z);
  spatial_parts(m, Z, scheme, part, nullptr, nullptr);
  gather(m, part, R);
  aos_to_soa(m, R, R_soa);
}

void rdo3_step(void* h, double* W_soa, double dt, int scheme, int order) {
  const Mesh& m = *static_cast<Mesh*>(h);
  std::vector<double> W;
  soa_to_aos(m, W_soa, W);
  step(m, W, dt, scheme, order);
  aos_to_soa(m, W, W_soa);
}

double rdo3_max_dt(void* h, const double* W_soa, double cfl) {
  const Mesh& m = *static_cast<Mesh*>(h);
  std::vector<double> sig(m.nv), acc(m.nv, 0.0);
  for (int64_t i = 0; i < m.nv; ++i) {
    const double rho = W_soa[i];
    const double u = W_soa[m.nv + i] / rho, v = W_soa[2 * m.nv + i] / rho, w = W_soa[3 * m.nv + i] / rho;
    const double p = (m.gamma - 1.0) * (W_soa[4 * m.nv + i] - 0.5 * rho * (u * u + v * v + w * w));
    sig[i] = std::sqrt(u * u + v * v + w * w) + std::sqrt(m.gamma * p / rho);
  }
  for (int64_t t = 0; t < m.nt; ++t) {
    double lam = 0.0;
    for (int i = 0; i < 4; ++i) lam = std::max(lam, sig[m.tet[4 * t + i]]);
    for (int i = 0; i < 4; ++i) acc[m.tet[4 * t + i]] += m.smax[t] * lam;
  }
  double best = INFINITY;
  for (int64_t i = 0; i < m.nv; ++i) best = std::min(best, 3.0 * m.V[i] / acc[i]);
  return cfl * best;
}

// One tetrahedron in isolation. W4: corner states [4][5]; xyz: corner
// positions [4][3] (positively oriented). out: phiT[5], phiN[4][5],
// phiLDA[4][5], phi(scheme)[4][5], Theta[5] (70 values).
void rdo3_tet(const double* W4, const double* xyz, double gamma, int scheme, double* out) {
  double Zc[4][5], p[4][3], n[4][3];
  for (int i = 0; i < 4; ++i) {
    w_to_z(&W4[5 * i], gamma, Zc[i]);
    for (int k = 0; k < 3; ++k) p[i][k] = xyz[3 * i + k];
  }
  for (int i = 0; i < 4; ++i) {
    const double* a = p[(i + 1) % 4];
    const double* b = p[(i + 2) % 4];
    const double* d = p[(i + 3) % 4];
    double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    double e2[3] = {d[0] - a[0], d[1] - a[1], d[2] - a[2]};
    cross(e1, e2, n[i]);
    for (int k = 0; k < 3; ++k) n[i][k] *= 0.5;
    double toward[3] = {p[i][0] - a[0], p[i][1] - a[1], p[i][2] - a[2]};
    if (dot3(n[i], toward) < 0.0)
      for (int k = 0; k < 3; ++k) n[i][k] = -n[i][k];
  }
  TetState s;
  eval_tet(Zc, n, gamma, s);
  double pl[4][5], pb[4][5], theta[5];
  for (int i = 0; i < 4; ++i) matvec(s.Kp[i], s.xL, pl[i]);
  distribute(scheme, s.phiT, s.phiN, pl, pb, theta);
  double* o = out;
  for (int k = 0; k < 5; ++k) *o++ = s.phiT[k];
  for (int i = 0; i < 4; ++i)
    for (int k = 0; k < 5; ++k) *o++ = s.phiN[i][k];
  for (int i = 0; i < 4; ++i)
    for (int k = 0; k < 5; ++k) *o++ = pl[i][k];
  for (int i = 0; i < 4; ++i)
    for (int k = 0; k < 5; ++k) *o++ = pb[i][k];
  for (int k = 0; k < 5; ++k) *o++ = theta[k];
}

// K, K^+, K^- (each [5][5], row-major) for the state W and the normal n
// (not necessarily unit: the result is |n| K(n / |n|), without the 1/3).
void rdo3_kmat(const double* W, const double* n, double gamma, double* K, double* Kp, double* Km) {
  double Z[5];
  w_to_z(W, gamma, Z);
  const double u[3] = {Z[1] / Z[0], Z[2] / Z[0], Z[3] / Z[0]};
  const double H = Z[4] / Z[0];
  const double c = std::sqrt((gamma - 1.0) * (H - 0.5 * dot3(u, u)));
  const double area = std::sqrt(dot3(n, n));
  const double nh[3] = {n[0] / area, n[1] / area, n[2] / area};
  const double un = dot3(u, nh);
  const double lam[5] = {un - c, un, un, un, un + c};
  double lp[5], lm[5];
  for (int k = 0; k < 5; ++k) {
    lp[k] = lam[k] > 0.0 ? lam[k] : 0.0;
    lm[k] = lam[k] < 0.0 ? lam[k] : 0.0;
  }
  double R[5][5], L[5][5], A[5][5];
  eigenvectors(u, H, c, nh, R);
  invert5(R, L);
  double* outs[3] = {K, Kp, Km};
  const double* ls[3] = {lam, lp, lm};
  for (int q = 0; q < 3; ++q) {
    kmat(R, L, ls[q], A);
    for (int r = 0; r < 5; ++r)
      for (int j = 0; j < 5; ++j) outs[q][5 * r + j] = area * A[r][j];
  }
}

void rdo3_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
}
