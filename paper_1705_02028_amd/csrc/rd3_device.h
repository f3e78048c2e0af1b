// Three-dimensional residual distribution on tetrahedra (the method of
// Section 3 with a row and a column added to every matrix, as the paper's
// closing discussion describes): per-tetrahedron and per-vertex bodies of the
// gfx950 kernels in rd3_kernels.hip. FP64 throughout.
//
// For a unit normal n the flux Jacobian K(n) = R diag(l) R^{-1} of the Euler
// equations is applied in its rank-two form: with the pressure gradient
// g = (g1 |u|^2 / 2, -g1 u, g1) (dp = g . dW), the normal-velocity row
// m = (-u.n, n, 0) (rho du.n = m . dW), r0 = (1, u, H) and s = (0, n, u.n),
// K x = l3 x + r0 ((l123 / c^2) g.x + (l12 / c) m.x) + s ((l12 / c) g.x + l123 m.x)
// with l123 = (l1 + l2) / 2 - l3 and l12 = (l1 - l2) / 2 for the eigenvalues
// l1 = u.n + c, l2 = u.n - c, l3 = u.n (or their positive or negative parts
// for K^+ and K^-). This is the three-dimensional form of the entries of
// Appendix A. K_i = (|n_i| / 3) K(n_i / |n_i|) with n_i the inward normal of
// the face opposite corner i scaled by the face's area.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rd3 {

constexpr int kBlock = 256;

enum { S_N = 0, S_LDA = 1, S_B = 2, S_BMAX = 3, S_BMIN = 4 };

// Device view of a tetrahedral mesh and its state.
struct Dev3 {
  int64_t nv = 0, nt = 0, ns = 0;  // vertices, tetrahedra, slots (4 nt plus slice padding)
  double gamma = 1.4;
  const int32_t* tet = nullptr;    // [4][nt] corners
  const int32_t* slot = nullptr;   // [4][nt] slot of each corner's part
  // Slots in sliced-ELL order: vertices in slices of 64; slice q owns
  // [sbase[q], sbase[q] + 64 w_q) with w_q its largest degree; the j-th
  // tetrahedron (ascending) of vertex v has slot sbase[v / 64] + 64 j + v % 64,
  // so a wave summing its 64 vertices reads consecutive slots.
  const int32_t* deg = nullptr;    // [nv] tetrahedra of vertex v
  const int32_t* sbase = nullptr;  // [ceil(nv / 64)]
  const double* nrm = nullptr;     // [12][nt] inward face normals scaled by area: component k of corner i at 3 i + k
  const double* vol = nullptr;     // [nt] volume
  const double* smax = nullptr;    // [nt] largest face area
  const double* V = nullptr;       // [nv] vertex volume (sum of |T| / 4)
  double* W = nullptr;             // [5][nv] state
  double* Ws = nullptr;            // [5][nv] first-stage state
  double* Z = nullptr;             // [5][nv] parameter vector of the state the next tetrahedron pass reads
  double* rate = nullptr;          // [5][nv] (W* - W^n) / dt, written by the first vertex pass
  double* sig = nullptr;           // [nv] |u| + c of W
  double* part = nullptr;          // [5][ns] distributed parts by slot
  double* keepN = nullptr;         // [15][nt] stage-1 N parts of corners 0-2 (component k of corner i at 5 i + k);
                                   // corner 3's is the kept residual minus those three
  double* keepT = nullptr;         // [5][nt] stage-1 residual
  double* cpart = nullptr;         // [ns] CFL parts by slot
  double* dt = nullptr;            // device scalar: the step's time step
  double* bmin = nullptr;          // [blocks] partial minima of the CFL limit
  int* flag = nullptr;             // non-physical state latch (rho <= 0, p <= 0 or not finite)
};

// Z and |u| + c of a state; returns whether it is physical (rho > 0, p > 0,
// finite).
__device__ inline bool to_z(const double w[5], double gamma, double z[5], double& sig) {
  const double rho = w[0], iu = 1.0 / rho;
  const double u = w[1] * iu, v = w[2] * iu, ww = w[3] * iu;
  const double q2 = u * u + v * v + ww * ww;
  const double p = (gamma - 1.0) * (w[4] - 0.5 * rho * q2);
  const double s = sqrt(rho);
  z[0] = s;
  z[1] = s * u;
  z[2] = s * v;
  z[3] = s * ww;
  z[4] = s * (w[4] + p) * iu;
  sig = sqrt(q2) + sqrt(gamma * p * iu);
  return rho > 0.0 && p > 0.0 && isfinite(sig) && isfinite(z[4]) && isfinite(z[1] + z[2] + z[3]);
}

// Rank-two application y = scale * K(l1, l2, l3) x at one corner.
struct Corner {
  double n[3];   // unit normal
  double un;     // u . n
  double scale;  // |n_i| / 3
};

struct Flow {
  double u[3], H, c, g[5], r0[5];
};

__device__ inline void kapply(const Flow& f, const Corner& q, double l1, double l2, double l3, const double x[5],
                              double y[5]) {
  const double l123 = 0.5 * (l1 + l2) - l3, l12 = 0.5 * (l1 - l2);
  const double gx = f.g[0] * x[0] + f.g[1] * x[1] + f.g[2] * x[2] + f.g[3] * x[3] + f.g[4] * x[4];
  const double mx = -q.un * x[0] + q.n[0] * x[1] + q.n[1] * x[2] + q.n[2] * x[3];
  const double ic = 1.0 / f.c;
  const double a = (l123 * ic * ic) * gx + (l12 * ic) * mx;
  const double b = (l12 * ic) * gx + l123 * mx;
  const double s[5] = {0.0, q.n[0], q.n[1], q.n[2], q.un};
  for (int k = 0; k < 5; ++k) y[k] = q.scale * (l3 * x[k] + f.r0[k] * a + s[k] * b);
}

__device__ inline double pos(double x) { return x > 0.0 ? x : 0.0; }
__device__ inline double neg(double x) { return x < 0.0 ? x : 0.0; }

// A x = b for two right-hand sides, Gaussian elimination with partial
// pivoting (the largest magnitude among the rows not yet used, first such
// row on ties); a column whose best pivot is at most 2^-45 max|A| is skipped
// (its unknowns are 0). Every array index is a compile-time constant (the
// pivot row is picked with selects and copied into U, its diagonal replaced
// by the pivot's reciprocal), so nothing goes to scratch memory.
__device__ inline void solve5x2(double A[5][5], double b1[5], double b2[5], double x1[5], double x2[5]) {
  double amax = 0.0;
#pragma unroll
  for (int r = 0; r < 5; ++r)
#pragma unroll
    for (int q = 0; q < 5; ++q) amax = fmax(amax, fabs(A[r][q]));
  const double tol = ldexp(amax, -45);
  int used = 0;
  bool skip[5];
  double U[5][5], c1[5], c2[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    int r = -1;
    double best = -1.0;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      const double a = fabs(A[i][k]);
      if (!(used & (1 << i)) && a > best) {
        best = a;
        r = i;
      }
    }
    skip[k] = r < 0 || !(best > tol);
    double pr[5], pb1 = b1[0], pb2 = b2[0];
#pragma unroll
    for (int j = 0; j < 5; ++j) pr[j] = A[0][j];
#pragma unroll
    for (int i = 1; i < 5; ++i) {
      const bool sel = r == i;
#pragma unroll
      for (int j = 0; j < 5; ++j) pr[j] = sel ? A[i][j] : pr[j];
      pb1 = sel ? b1[i] : pb1;
      pb2 = sel ? b2[i] : pb2;
    }
#pragma unroll
    for (int j = 0; j < 5; ++j) U[k][j] = pr[j];
    c1[k] = pb1;
    c2[k] = pb2;
    if (skip[k]) continue;
    used |= 1 << r;
    const double ip = 1.0 / pr[k];
    U[k][k] = ip;  // the back substitution multiplies by it
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      if (used & (1 << i)) continue;
      const double fct = A[i][k] * ip;
#pragma unroll
      for (int j = k; j < 5; ++j) A[i][j] -= fct * pr[j];
      b1[i] -= fct * pb1;
      b2[i] -= fct * pb2;
    }
  }
#pragma unroll
  for (int k = 4; k >= 0; --k) {
    double s1 = c1[k], s2 = c2[k];
#pragma unroll
    for (int j = k + 1; j < 5; ++j) {
      s1 -= U[k][j] * x1[j];
      s2 -= U[k][j] * x2[j];
    }
    x1[k] = skip[k] ? 0.0 : s1 * U[k][k];
    x2[k] = skip[k] ? 0.0 : s2 * U[k][k];
  }
}

// Blend coefficients of the B family from the residual `res` and the N
// parts pn: Theta_k = min(1, |res_k| / sum_i |pn_ik|) (0 for a zero sum),
// one common value for Bmax / Bmin; unused by N and LDA.
__device__ inline void blend_theta(int scheme, const double res[5], const double pn[4][5], double th[5]) {
  for (int k = 0; k < 5; ++k) {
    const double den = fabs(pn[0][k]) + fabs(pn[1][k]) + fabs(pn[2][k]) + fabs(pn[3][k]);
    const double q = den == 0.0 ? 0.0 : fabs(res[k]) / den;
    th[k] = q > 1.0 ? 1.0 : q;
  }
  if (scheme == S_BMAX || scheme == S_BMIN) {
    int pick = 0;
    for (int k = 1; k < 5; ++k)
      if (scheme == S_BMAX ? th[k] > th[pick] : th[k] < th[pick]) pick = k;
    double t = th[0];
    for (int k = 1; k < 5; ++k) t = pick == k ? th[k] : t;
    for (int k = 0; k < 5; ++k) th[k] = t;
  }
}

// One tetrahedron: stage 1 (or Euler) at the Z in d.Z; stage 2 adds the
// mass term of the first-stage increment and the kept stage-1 parts.
template <int STAGE, int SCHEME>
__device__ inline void tet_body(const Dev3& d, int64_t t, bool keep) {
  constexpr int scheme = SCHEME;
  const int64_t nt = d.nt, nv = d.nv;
  const double g1 = d.gamma - 1.0;
  int32_t vid[4];
  double Zc[4][5];
  for (int i = 0; i < 4; ++i) {
    vid[i] = d.tet[i * nt + t];
    for (int k = 0; k < 5; ++k) Zc[i][k] = d.Z[k * nv + vid[i]];
  }
  double zb[5];
  for (int k = 0; k < 5; ++k) zb[k] = 0.25 * (Zc[0][k] + Zc[1][k] + Zc[2][k] + Zc[3][k]);
  Flow f;
  const double iz = 1.0 / zb[0];
  f.u[0] = zb[1] * iz;
  f.u[1] = zb[2] * iz;
  f.u[2] = zb[3] * iz;
  f.H = zb[4] * iz;
  const double q2 = f.u[0] * f.u[0] + f.u[1] * f.u[1] + f.u[2] * f.u[2];
  f.c = sqrt(g1 * (f.H - 0.5 * q2));
  f.g[0] = 0.5 * g1 * q2;
  f.g[1] = -g1 * f.u[0];
  f.g[2] = -g1 * f.u[1];
  f.g[3] = -g1 * f.u[2];
  f.g[4] = g1;
  f.r0[0] = 1.0;
  f.r0[1] = f.u[0];
  f.r0[2] = f.u[1];
  f.r0[3] = f.u[2];
  f.r0[4] = f.H;
  // state differences M(zbar)(Z_i - Z_0)
  double dW[4][5];
  const double igam = 1.0 / d.gamma;
  for (int k = 0; k < 5; ++k) dW[0][k] = 0.0;
  for (int i = 1; i < 4; ++i) {
    double dz[5];
    for (int k = 0; k < 5; ++k) dz[k] = Zc[i][k] - Zc[0][k];
    dW[i][0] = 2.0 * zb[0] * dz[0];
    for (int k = 1; k < 4; ++k) dW[i][k] = zb[k] * dz[0] + zb[0] * dz[k];
    dW[i][4] = (zb[4] * dz[0] + g1 * (zb[1] * dz[1] + zb[2] * dz[2] + zb[3] * dz[3]) + zb[0] * dz[4]) * igam;
  }
  Corner cn[4];
  for (int i = 0; i < 4; ++i) {
    double n[3];
    for (int k = 0; k < 3; ++k) n[k] = d.nrm[(3 * i + k) * nt + t];
    const double area = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    const double ia = 1.0 / area;
    for (int k = 0; k < 3; ++k) cn[i].n[k] = n[k] * ia;
    cn[i].un = f.u[0] * cn[i].n[0] + f.u[1] * cn[i].n[1] + f.u[2] * cn[i].n[2];
    cn[i].scale = area * (1.0 / 3.0);
  }
  // residual and the N right-hand side
  double phiT[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, bN[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int i = 1; i < 4; ++i) {
    const double un = cn[i].un;
    double y[5];
    kapply(f, cn[i], un + f.c, un - f.c, un, dW[i], y);
    for (int k = 0; k < 5; ++k) phiT[k] += y[k];
    kapply(f, cn[i], neg(un + f.c), neg(un - f.c), neg(un), dW[i], y);
    for (int k = 0; k < 5; ++k) bN[k] += y[k];
  }
  // A = sum_i K_i^+ from the rank-two form: sum_i sc_i l3_i I + r0 (sum_i a_i)^T
  // + sum_i s_i b_i^T, with s_i = (0, n_i, u.n_i) (its first entry is zero)
  double A[5][5], abar[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, dsum = 0.0;
  for (int r = 0; r < 5; ++r)
    for (int q = 0; q < 5; ++q) A[r][q] = 0.0;
  {
    const double ic = 1.0 / f.c;
    for (int i = 0; i < 4; ++i) {
      const double un = cn[i].un;
      const double l1 = pos(un + f.c), l2 = pos(un - f.c), l3 = pos(un);
      const double sc = cn[i].scale;
      const double l123 = sc * (0.5 * (l1 + l2) - l3), l12 = sc * (0.5 * (l1 - l2));
      const double m[5] = {-un, cn[i].n[0], cn[i].n[1], cn[i].n[2], 0.0};
      const double s[4] = {cn[i].n[0], cn[i].n[1], cn[i].n[2], un};
      dsum += sc * l3;
      for (int q = 0; q < 5; ++q) {
        abar[q] += (l123 * ic * ic) * f.g[q] + (l12 * ic) * m[q];
        const double b = (l12 * ic) * f.g[q] + l123 * m[q];
        for (int r = 1; r < 5; ++r) A[r][q] += s[r - 1] * b;
      }
    }
  }
  for (int r = 0; r < 5; ++r) {
    A[r][r] += dsum;
    for (int q = 0; q < 5; ++q) A[r][q] += f.r0[r] * abar[q];
  }
  double PT[5];
  if (STAGE == 1) {
    for (int k = 0; k < 5; ++k) PT[k] = phiT[k];
  } else {
    // stage 2: the mass |T| / 4 times the first-stage rate, plus the mean of
    // the kept and the current residual
    const double mass = 0.25 * d.vol[t];
    double rate_sum[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int i = 0; i < 4; ++i)
      for (int k = 0; k < 5; ++k) rate_sum[k] += d.rate[k * nv + vid[i]];
    for (int k = 0; k < 5; ++k) PT[k] = mass * rate_sum[k] + 0.5 * (d.keepT[k * nt + t] + phiT[k]);
  }
  double rhsT[5];
  for (int k = 0; k < 5; ++k) rhsT[k] = PT[k];
  double xN[5], xT[5];
  solve5x2(A, bN, rhsT, xN, xT);
  // N parts of every corner (the blend needs all of them), then each
  // corner's LDA part and output. The parts of a distribution add up to the
  // residual they split (sum_i K_i^+ (dW_i + xN) = phi^T, sum_i K_i^+ xT =
  // PT), so corner 3's are that residual minus those of corners 0-2.
  double pn[4][5];
  for (int i = 0; i < 3; ++i) {
    const double un = cn[i].un;
    double y[5];
    for (int k = 0; k < 5; ++k) y[k] = (i == 0 ? 0.0 : dW[i][k]) + xN[k];
    kapply(f, cn[i], pos(un + f.c), pos(un - f.c), pos(un), y, pn[i]);
  }
  for (int k = 0; k < 5; ++k) pn[3][k] = phiT[k] - pn[0][k] - pn[1][k] - pn[2][k];
  if (STAGE == 1 && keep) {
    // read back only by the stage-2 pass after the gather: stored with the
    // non-temporal hint so they do not evict what the gather reads next;
    // corner 3's part is formed again from the residual in stage 2
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 5; ++k) __builtin_nontemporal_store(pn[i][k], &d.keepN[(5 * i + k) * nt + t]);
    for (int k = 0; k < 5; ++k) __builtin_nontemporal_store(phiT[k], &d.keepT[k * nt + t]);
  }
  if (STAGE == 2) {
    const double mass = 0.25 * d.vol[t];
    for (int k = 0; k < 5; ++k) {
      double kn[4];
      for (int i = 0; i < 3; ++i) kn[i] = d.keepN[(5 * i + k) * nt + t];
      kn[3] = d.keepT[k * nt + t] - kn[0] - kn[1] - kn[2];
      for (int i = 0; i < 4; ++i) pn[i][k] = mass * d.rate[k * nv + vid[i]] + 0.5 * (kn[i] + pn[i][k]);
    }
  }
  double th[5];
  blend_theta(scheme, PT, pn, th);
  double lsum[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int i = 0; i < 4; ++i) {
    double pl[5];
    if (i < 3) {
      const double un = cn[i].un;
      kapply(f, cn[i], pos(un + f.c), pos(un - f.c), pos(un), xT, pl);
      for (int k = 0; k < 5; ++k) lsum[k] += pl[k];
    } else {
      for (int k = 0; k < 5; ++k) pl[k] = PT[k] - lsum[k];
    }
    const int64_t sl = d.slot[i * nt + t];
    for (int k = 0; k < 5; ++k) {
      const double o = scheme == S_N ? pn[i][k] : scheme == S_LDA ? pl[k] : pl[k] + th[k] * (pn[i][k] - pl[k]);
      d.part[k * d.ns + sl] = o;
    }
  }
}

}  // namespace rd3
