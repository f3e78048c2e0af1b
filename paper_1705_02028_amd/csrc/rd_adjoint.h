// Reverse mode of one residual-distribution step (FP64, time step fixed).
//
// The step of Sections 3.2-3.4 is, per triangle, a function of the three
// corner parameter vectors (stage 1), or of the stage-1 state W*, of
// W* - W^n and of the kept stage-1 N parts and residual (stage 2), followed
// by per-vertex sums and updates. Its adjoint runs the same structure
// backwards: per triangle, the forward arithmetic is recomputed in registers
// and then differentiated line by line in reverse order (each block below
// is the transpose of the matching block of the forward pass in
// rd_device.h); per vertex, the corner cotangents are summed over the vertex
// CSR in fixed order and mapped through dZ/dW. Branches follow the forward
// values: max/min of eigenvalues, pivot order, |.| (derivative 0 at 0), the
// 0/0 and clamped cases of the blend, the component Bmax/Bmin selects.
// The pivoted solve is differentiated as x = A^{-1} b, which needs every
// column of A to have its pivot; a triangle whose solve skips a column (an
// exactly stagnant triangle, Section 3.3.1) is reported through the
// adjoint's flag instead (flag[1]), and the call's result is not used.
#pragma once

#include "rd_device.h"

namespace rd {

// Stage-2 corner cotangents of one slot: of Z* and of W* - W^n, side by side
// so the reverse gather reads one 64-byte record per slot.
struct alignas(64) ZW {
  D4 z, w;
};

// A field of cotangents, one 4-vector per vertex: records (AoS) or the
// caller's structure-of-arrays layout [4][n].
struct LamAoS {
  const D4* p = nullptr;
  __host__ __device__ D4 at(int64_t v) const { return p[v]; }
};
struct LamSoA {
  const double* p = nullptr;
  int64_t n = 0;
  __host__ __device__ D4 at(int64_t v) const { return D4{{p[v], p[n + v], p[2 * n + v], p[3 * n + v]}}; }
};

// Per-vertex inputs of the reverse triangle passes, packed so that a pass
// reads each corner's inputs as one contiguous record: for stage 2 the
// parameter vector at W* (at W^n on ghosts), W* - W^n and mu2 = -(dt/V)
// dL/dW^{n+1}; for stage 1 the parameter vector at W^n and mu1 = -(dt/V)
// dL/dW* (mu is 0 on ghosts, whose update ignores their residual).
struct alignas(32) AdjRec2 {
  D4 zc, dw, mu;
};
struct alignas(32) AdjRec1 {
  D4 zn, mu;
};

struct AdjDev {
  LamSoA lam;                // dL/dW^{n+1}, the caller's [4][nv]
  AdjRec2* r2 = nullptr;     // [nv] stage-2 reverse inputs
  AdjRec1* r1 = nullptr;     // [nv] stage-1 reverse inputs
  D4* lamS = nullptr;        // [nv] dL/dW*
  D4* lamN = nullptr;        // [nv] running dL/dW^n (output)
  D4* Zn = nullptr;          // [nv] parameter vectors at W^n
  // per-slot and per-triangle records below are stored in 16-byte planes
  // (plane_store / plane_load: chunk c of record j of item i at (2 j + c) n + i)
  D4* cZ = nullptr;          // [ns] stage-1 corner cotangent of Z (sliced part layout)
  ZW* cZW = nullptr;         // [ns] stage-2 corner cotangents of Z* (record 0) and W* - W^n (record 1)
  D4* kN = nullptr;          // [2nt] cotangent of the kept stage-1 N parts of corners 0 and 1 (records 0, 1)
  D4* kT = nullptr;          // [nt] cotangent of kept stage-1 residual
  D4* wcbar = nullptr;       // [nwv] cotangent of the wall term at W^n (stage 1 + half of stage 2)
  int* flag = nullptr;       // [2]: [0] the recomputed step went non-physical, [1] a solve skipped a column
  double idt = 0.0;          // 1 / dt of the step being reversed
  int32_t waves = 0;         // workgroups of the reverse triangle passes (one per SIMD)
};

// The staged reverse triangle passes keep one wavefront per SIMD resident.
constexpr int kAdjWavesPerCu = 4;

// Cotangents of the quantities shared by all corners of a triangle.
struct RoeBar {
  double u = 0, v = 0, h = 0, c = 0, ic = 0, ac = 0, uc = 0, vc = 0;
};
struct CornerBar {
  double w = 0, l3p = 0, h1p = 0, h2p = 0, l3m = 0, h1m = 0, h2m = 0;
};

__host__ __device__ inline double sgn(double x) { return x > 0.0 ? 1.0 : (x < 0.0 ? -1.0 : 0.0); }

// Transpose of the tail shared by both K applications:
// g = ac y0 - g1 (uc y1 + vc y2 - ic y3), d = -w y0 + nx y1 + ny y2.
__host__ __device__ inline void gd_bar(const Roe<double>& q, const Corner<double>& k, const double y[4], double gb,
                                       double db, double yb[4], RoeBar& qb, CornerBar& kb) {
  yb[0] += q.ac * gb - k.w * db;
  yb[1] += -q.g1 * q.uc * gb + k.nx * db;
  yb[2] += -q.g1 * q.vc * gb + k.ny * db;
  yb[3] += q.g1 * q.ic * gb;
  qb.ac += y[0] * gb;
  qb.uc += -q.g1 * y[1] * gb;
  qb.vc += -q.g1 * y[2] * gb;
  qb.ic += q.g1 * y[3] * gb;
  kb.w += -y[0] * db;
}

// Transpose of apply_split (out = sl3 y + sp E + sm N).
__host__ __device__ inline void apply_split_bar(const Roe<double>& q, const Corner<double>& k, double sl3, double h1,
                                                double h2, const double y[4], const double ob[4], double yb[4],
                                                RoeBar& qb, CornerBar& kb, double& sl3b, double& h1b, double& h2b) {
  const double g = q.ac * y[0] - q.g1 * (q.uc * y[1] + q.vc * y[2] - q.ic * y[3]);
  const double d = -k.w * y[0] + k.nx * y[1] + k.ny * y[2];
  const double a1 = h1 * (g + d), a2 = h2 * (g - d);
  const double sp = a1 + a2, sm = (a1 - a2) * q.c;
  sl3b += ob[0] * y[0] + ob[1] * y[1] + ob[2] * y[2] + ob[3] * y[3];
  for (int r = 0; r < 4; ++r) yb[r] += sl3 * ob[r];
  const double spb = ob[0] + ob[1] * q.u + ob[2] * q.v + ob[3] * q.h;
  qb.u += ob[1] * sp;
  qb.v += ob[2] * sp;
  qb.h += ob[3] * sp;
  const double smb = ob[1] * k.nx + ob[2] * k.ny + ob[3] * k.w;
  kb.w += ob[3] * sm;
  const double a1b = spb + smb * q.c, a2b = spb - smb * q.c;
  qb.c += smb * (a1 - a2);
  h1b += a1b * (g + d);
  h2b += a2b * (g - d);
  const double gb = a1b * h1 + a2b * h2, db = a1b * h1 - a2b * h2;
  gd_bar(q, k, y, gb, db, yb, qb, kb);
}

// Transpose of apply_full (out = s (w y + d E + c g N)).
__host__ __device__ inline void apply_full_bar(const Roe<double>& q, const Corner<double>& k, const double y[4],
                                               const double ob[4], double yb[4], RoeBar& qb, CornerBar& kb) {
  const double g = q.ac * y[0] - q.g1 * (q.uc * y[1] + q.vc * y[2] - q.ic * y[3]);
  const double d = -k.w * y[0] + k.nx * y[1] + k.ny * y[2];
  double o[4];
  for (int r = 0; r < 4; ++r) o[r] = k.s * ob[r];
  kb.w += o[0] * y[0] + o[1] * y[1] + o[2] * y[2] + o[3] * y[3] + o[3] * q.c * g;
  for (int r = 0; r < 4; ++r) yb[r] += k.w * o[r];
  const double db = o[0] + o[1] * q.u + o[2] * q.v + o[3] * q.h;
  qb.u += o[1] * d;
  qb.v += o[2] * d;
  qb.h += o[3] * d;
  const double cgb = o[1] * k.nx + o[2] * k.ny + o[3] * k.w;
  qb.c += g * cgb;
  gd_bar(q, k, y, q.c * cgb, db, yb, qb, kb);
}

// Transpose of build_A for the rank-2 cotangent A_bar = -(a b^T + c d^T)
// (the cotangent of A in x = A^{-1} rhs for two right-hand sides): every
// contraction of A_bar is formed from dot products with a, b, c, d.
__host__ __device__ inline void build_A_bar(const Roe<double>& q, const Corner<double> k[3], const double a[4],
                                            const double b[4], const double c[4], const double dd[4], RoeBar& qb,
                                            CornerBar kb[3]) {
  auto dot = [](const double* x, const double* y) { return x[0] * y[0] + x[1] * y[1] + x[2] * y[2] + x[3] * y[3]; };
  const double G[4] = {q.ac, -q.g1 * q.uc, -q.g1 * q.vc, q.g1 * q.ic};
  const double E[4] = {1.0, q.u, q.v, q.h};
  double P[3], Qv[3];
  for (int i = 0; i < 3; ++i) {
    P[i] = k[i].h1p + k[i].h2p;
    Qv[i] = k[i].h1p - k[i].h2p;
  }
  const double sP = P[0] + P[1] + P[2];
  double ev[4];
  ev[0] = sP * G[0] - (Qv[0] * k[0].w + Qv[1] * k[1].w + Qv[2] * k[2].w);
  ev[1] = sP * G[1] + (Qv[0] * k[0].nx + Qv[1] * k[1].nx + Qv[2] * k[2].nx);
  ev[2] = sP * G[2] + (Qv[0] * k[0].ny + Qv[1] * k[1].ny + Qv[2] * k[2].ny);
  ev[3] = sP * G[3];
  double sQN[4];
  sQN[0] = 0.0;
  sQN[1] = Qv[0] * k[0].nx + Qv[1] * k[1].nx + Qv[2] * k[2].nx;
  sQN[2] = Qv[0] * k[0].ny + Qv[1] * k[1].ny + Qv[2] * k[2].ny;
  sQN[3] = Qv[0] * k[0].w + Qv[1] * k[1].w + Qv[2] * k[2].w;
  double nvv[4];
  for (int r = 0; r < 4; ++r) nvv[r] = q.c * sQN[r];
  // A = L3 I + E ev^T + nvv G^T + S
  const double L3b = -(dot(a, b) + dot(c, dd));
  const double bev = dot(b, ev), dev = dot(dd, ev), bG = dot(b, G), dG = dot(dd, G);
  const double aE = dot(a, E), cE = dot(c, E), an = dot(a, nvv), cn = dot(c, nvv);
  double Eb[4], evb[4], nvvb[4], Gb[4];
  for (int r = 0; r < 4; ++r) {
    Eb[r] = -(a[r] * bev + c[r] * dev);
    evb[r] = -(b[r] * aE + dd[r] * cE);
    nvvb[r] = -(a[r] * bG + c[r] * dG);
    Gb[r] = -(b[r] * an + dd[r] * cn);
  }
  // S[r][j] = c sum_i P_i N_ir D_ij  (r = 1..3, j = 0..2)
  double Pb[3] = {0, 0, 0}, Qb[3] = {0, 0, 0};
  for (int i = 0; i < 3; ++i) {
    const double Nr[4] = {0.0, k[i].nx, k[i].ny, k[i].w};
    const double Dc[4] = {-k[i].w, k[i].nx, k[i].ny, 0.0};
    const double aN = dot(a, Nr), cN = dot(c, Nr), bD = dot(b, Dc), dD = dot(dd, Dc);
    const double acc = -(aN * bD + cN * dD);
    Pb[i] += q.c * acc;
    qb.c += P[i] * acc;
    // w appears as N_i3 (row 3) and as -D_i0 (column 0)
    const double wb = -(a[3] * bD + c[3] * dD) + (b[0] * aN + dd[0] * cN);
    kb[i].w += q.c * P[i] * wb;
  }
  // nvv = c sQN
  for (int r = 0; r < 4; ++r) qb.c += nvvb[r] * sQN[r];
  for (int i = 0; i < 3; ++i) {
    Qb[i] += q.c * (nvvb[1] * k[i].nx + nvvb[2] * k[i].ny + nvvb[3] * k[i].w);
    kb[i].w += q.c * Qv[i] * nvvb[3];
  }
  // ev = sP G + sum_i Q_i D_i
  double sPb = 0.0;
  for (int j = 0; j < 4; ++j) {
    sPb += evb[j] * G[j];
    Gb[j] += sP * evb[j];
  }
  for (int i = 0; i < 3; ++i) {
    Qb[i] += -evb[0] * k[i].w + evb[1] * k[i].nx + evb[2] * k[i].ny;
    kb[i].w += -Qv[i] * evb[0];
  }
  for (int i = 0; i < 3; ++i) {
    Pb[i] += sPb;
    kb[i].h1p += Pb[i] + Qb[i];
    kb[i].h2p += Pb[i] - Qb[i];
    kb[i].l3p += L3b;
  }
  qb.u += Eb[1];
  qb.v += Eb[2];
  qb.h += Eb[3];
  qb.ac += Gb[0];
  qb.uc += -q.g1 * Gb[1];
  qb.vc += -q.g1 * Gb[2];
  qb.ic += q.g1 * Gb[3];
}

// A D4 in the staging buffer of the reverse triangle passes: 16-byte units
// laid out [unit][lane], so a record's two halves sit 64 units apart.
struct D4Lds {
  const double2* p = nullptr;
  __host__ __device__ D4 operator*() const {
    const double2 lo = p[0], hi = p[64];
    return D4{{lo.x, lo.y, hi.x, hi.y}};
  }
  __host__ __device__ explicit operator bool() const { return p != nullptr; }
};

// Inputs of the stage-2 function of one triangle besides its parameter
// vectors, read where they are used (not held in registers across the
// triangle's forward recomputation) through P: a pointer-like type whose
// operator* gives the D4 and whose bool conversion says whether it is there.
template <class P>
struct Stage2In {
  double mass = 0.0, idt = 0.0;
  P dw[3];  // W*_i - W^n_i
  P kn[2];  // stage-1 N parts of corners 0 and 1
  P kt;     // stage-1 residual
};
struct Stage2Bar {
  double dw[3][4];
  double keepN[3][4];
  double keepT[4];
};

// Reverse of one triangle. Zc: corner parameter vectors; geometry from the
// unwrapped normals (nxd, nyd). mu.get(i): cotangent of the scheme's part of
// corner i. Stage 1 also takes the cotangents of the kept N parts of corners
// 0 and 1 (kN0, kN1) and of the kept residual (kT), or null for a
// forward Euler step; stage 2 takes its extra inputs in s2 and returns theirs in
// s2b. Returns the corner cotangents of Z in Zb.
// Returns true when the pivoted solve skipped a column (A singular), where
// the cotangents are not the derivative.
template <int SCHEME, int STAGE, class P, class MU>
__host__ __device__ inline bool tri_adjoint(const D4 Zc[3], const double nxd[3], const double nyd[3], double gamma,
                                            double igamma, const MU& mu, P kN0, P kN1, P kT,
                                            const Stage2In<P>* s2, Stage2Bar* s2b, double Zb[3][4]) {
  // ---------------- forward (recomputed, as in tri_compute) ----------------
  Roe<double> q;
  q.g1 = gamma - 1.0;
  const double third = 1.0 / 3.0, igam = igamma;
  double zb[4];
  for (int k = 0; k < 4; ++k) zb[k] = (Zc[0].v[k] + Zc[1].v[k] + Zc[2].v[k]) * third;
  const double iz = 1.0 / zb[0];
  q.u = zb[1] * iz;
  q.v = zb[2] * iz;
  q.h = zb[3] * iz;
  const double q2 = q.u * q.u + q.v * q.v;
  q.c = sqrt(q.g1 * (q.h - 0.5 * q2));
  q.ic = 1.0 / q.c;
  q.ac = 0.5 * q.g1 * q2 * q.ic;
  q.uc = q.u * q.ic;
  q.vc = q.v * q.ic;
  double dz[3][4], dWh[3][4];
  for (int k = 0; k < 4; ++k) dz[0][k] = dWh[0][k] = 0.0;
  for (int i = 1; i < 3; ++i) {
    for (int k = 0; k < 4; ++k) dz[i][k] = Zc[i].v[k] - Zc[0].v[k];
    dWh[i][0] = 2.0 * zb[0] * dz[i][0];
    dWh[i][1] = zb[1] * dz[i][0] + zb[0] * dz[i][1];
    dWh[i][2] = zb[2] * dz[i][0] + zb[0] * dz[i][2];
    dWh[i][3] = (zb[3] * dz[i][0] + q.g1 * (zb[1] * dz[i][1] + zb[2] * dz[i][2]) + zb[0] * dz[i][3]) * igam;
  }
  Corner<double> kc[3];
  const double hic = 0.5 * q.ic;
  for (int i = 0; i < 3; ++i) {
    const double L = sqrt(nxd[i] * nxd[i] + nyd[i] * nyd[i]);
    const double iL = 1.0 / L;
    Corner<double>& k = kc[i];
    k.nx = nxd[i] * iL;
    k.ny = nyd[i] * iL;
    k.s = 0.5 * L;
    k.w = q.u * k.nx + q.v * k.ny;
    const double l1 = k.w + q.c, l2 = k.w - q.c, l3 = k.w;
    const double p1 = rmax(l1, 0.0), p2 = rmax(l2, 0.0), p3 = rmax(l3, 0.0);
    const double m1 = rmin(l1, 0.0), m2 = rmin(l2, 0.0), m3 = rmin(l3, 0.0);
    const double sh = k.s * hic;
    k.l3p = k.s * p3;
    k.h1p = sh * (p1 - p3);
    k.h2p = sh * (p2 - p3);
    k.l3m = k.s * m3;
    k.h1m = sh * (m1 - m3);
    k.h2m = sh * (m2 - m3);
  }
  double phiT[4], bN[4], t1[4], t2[4];
  apply_full(q, kc[1], dWh[1], t1);
  apply_full(q, kc[2], dWh[2], t2);
  for (int k = 0; k < 4; ++k) phiT[k] = t1[k] + t2[k];
  double A[4][4];
  build_A(q, kc, A);
  apply_split(q, kc[1], kc[1].l3m, kc[1].h1m, kc[1].h2m, dWh[1], t1);
  apply_split(q, kc[2], kc[2].l3m, kc[2].h1m, kc[2].h2m, dWh[2], t2);
  for (int k = 0; k < 4; ++k) bN[k] = t1[k] + t2[k];
  // A^{-1} (columns from unit right-hand sides) and the two solutions
  double Ai[4][4];
  bool singular = false;
  {
    double e0[4], e1[4], x0[4], x1[4], Aw[4][4];
    for (int c2 = 0; c2 < 4; c2 += 2) {
      for (int r = 0; r < 4; ++r) {
        e0[r] = r == c2 ? 1.0 : 0.0;
        e1[r] = r == c2 + 1 ? 1.0 : 0.0;
        for (int c = 0; c < 4; ++c) Aw[r][c] = A[r][c];
      }
      bool skipped;
      solve2<double, false>(Aw, e0, e1, x0, x1, skipped);  // IEEE division: the fast one spills here
      singular = singular || skipped;
      for (int r = 0; r < 4; ++r) {
        Ai[r][c2] = x0[r];
        Ai[r][c2 + 1] = x1[r];
      }
    }
  }
  // the LDA right-hand side (stage 2: with the rate of W* - W^n and the kept
  // stage-1 residual), formed after the inverse: its inputs are read late
  double rhs1[4], srate[4] = {0, 0, 0, 0};
  if (STAGE == 1) {
    for (int k = 0; k < 4; ++k) rhs1[k] = phiT[k];
  } else {
    for (int i = 0; i < 3; ++i) {
      const D4 w = *s2->dw[i];
      for (int k = 0; k < 4; ++k) srate[k] += w.v[k] * s2->idt;
    }
    const D4 kt = SCHEME == SCH_N ? D4{{0.0, 0.0, 0.0, 0.0}} : *s2->kt;
    for (int k = 0; k < 4; ++k) rhs1[k] = s2->mass * srate[k] + 0.5 * (kt.v[k] + phiT[k]);
  }
  double xN[4], xL[4];
  for (int r = 0; r < 4; ++r) {
    xN[r] = Ai[r][0] * bN[0] + Ai[r][1] * bN[1] + Ai[r][2] * bN[2] + Ai[r][3] * bN[3];
    xL[r] = Ai[r][0] * rhs1[0] + Ai[r][1] * rhs1[1] + Ai[r][2] * rhs1[2] + Ai[r][3] * rhs1[3];
  }
  // per corner: N part pN (stage 2: total PN), LDA part pl. As in the
  // forward pass, corner 2's parts are the residual being split minus those
  // of corners 0 and 1 (sum_i K_i^+ (dW_i + xN) = phi^T and
  // sum_i K_i^+ xL = rhs1), so the reverse differentiates two K^+ products
  // per corner fewer. Kept are the blend's sums and the signs of PN (the
  // reverse recomputes the rest).
  double th[4] = {0, 0, 0, 0}, den[4] = {0, 0, 0, 0}, thb[4] = {0, 0, 0, 0};
  unsigned spos = 0, sneg = 0;  // bit 4 i + k: PN_ik > 0, PN_ik < 0
  {
    double pN[3][4], pl[3][4];
    for (int i = 0; i < 2; ++i) {
      double yN[4];
      for (int k = 0; k < 4; ++k) yN[k] = dWh[i][k] + xN[k];
      apply_split(q, kc[i], kc[i].l3p, kc[i].h1p, kc[i].h2p, yN, pN[i]);
      apply_split(q, kc[i], kc[i].l3p, kc[i].h1p, kc[i].h2p, xL, pl[i]);
    }
    for (int k = 0; k < 4; ++k) {
      pN[2][k] = phiT[k] - pN[0][k] - pN[1][k];
      pl[2][k] = rhs1[k] - pl[0][k] - pl[1][k];
    }
    // stage 2: the kept stage-1 N parts (corner 2's formed as the forward
    // pass forms it, phi^T(n) minus corners 0 and 1) and W* - W^n
    double kn[3][4], dw[3][4];
    if (STAGE == 2) {
      const D4 z = {{0.0, 0.0, 0.0, 0.0}};
      const bool keep = SCHEME != SCH_LDA;
      const D4 k0 = keep ? *s2->kn[0] : z, k1 = keep ? *s2->kn[1] : z, kt = keep ? *s2->kt : z;
      for (int k = 0; k < 4; ++k) {
        kn[0][k] = k0.v[k];
        kn[1][k] = k1.v[k];
        kn[2][k] = kt.v[k] - k0.v[k] - k1.v[k];
      }
      for (int i = 0; i < 3; ++i) {
        const D4 w = *s2->dw[i];
        for (int k = 0; k < 4; ++k) dw[i][k] = w.v[k];
      }
    }
    for (int i = 0; i < 3; ++i) {
      const D4 ob = mu.get(i);
      for (int k = 0; k < 4; ++k) {
        const double PN = STAGE == 1 ? pN[i][k] : s2->mass * (dw[i][k] * s2->idt) + 0.5 * (kn[i][k] + pN[i][k]);
        den[k] = den[k] + fabs(PN);
        thb[k] = thb[k] + ob.v[k] * (PN - pl[i][k]);
        spos |= (PN > 0.0 ? 1u : 0u) << (4 * i + k);
        sneg |= (PN < 0.0 ? 1u : 0u) << (4 * i + k);
      }
    }
  }
  bool active[4] = {false, false, false, false};  // Theta_k = |r_k| / den_k, not 0/0, not clamped
  double idn[4] = {0, 0, 0, 0};                    // 1 / den_k (0 where den_k = 0)
  double ratio[4] = {0, 0, 0, 0};                    // |r_k| / den_k before the clamp and the Bmax/Bmin pick
  int pick = 0;
  if (SCHEME >= SCH_B) {
    for (int k = 0; k < 4; ++k) {
      // the forward pass's quotient: |r_k| times the reciprocal of den_k
      // (the reciprocal is kept for the reverse)
      idn[k] = den[k] == 0.0 ? 0.0 : 1.0 / den[k];
      const double qq = fabs(rhs1[k]) * idn[k];
      active[k] = den[k] != 0.0 && !(qq > 1.0);
      ratio[k] = qq;
      th[k] = qq > 1.0 ? 1.0 : qq;
    }
    if (SCHEME == SCH_BMAX || SCHEME == SCH_BMIN) {
      double t = th[0];
      for (int k = 1; k < 4; ++k) {
        const bool better = SCHEME == SCH_BMAX ? th[k] > t : th[k] < t;
        t = better ? th[k] : t;
        pick = better ? k : pick;
      }
      for (int k = 0; k < 4; ++k) th[k] = t;
    }
  }

  // ---------------- reverse ----------------
  RoeBar qb;
  CornerBar kb[3];
  double rhs1b[4] = {0, 0, 0, 0}, denb[4] = {0, 0, 0, 0};
  if (SCHEME >= SCH_B) {
    if (SCHEME == SCH_BMAX || SCHEME == SCH_BMIN) {
      const double s = thb[0] + thb[1] + thb[2] + thb[3];
      for (int k = 0; k < 4; ++k) thb[k] = k == pick ? s : 0.0;
    }
    for (int k = 0; k < 4; ++k) {
      if (!active[k]) continue;
      rhs1b[k] += thb[k] * sgn(rhs1[k]) * idn[k];
      denb[k] = -thb[k] * ratio[k] * idn[k];
    }
  }
  double xLb[4] = {0, 0, 0, 0}, xNb[4] = {0, 0, 0, 0}, dWhb[3][4];
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 4; ++k) dWhb[i][k] = 0.0;
  double plb[3][4], pNb[3][4];
  for (int i = 0; i < 3; ++i) {
    const D4 ob = mu.get(i);
    for (int k = 0; k < 4; ++k) {
      double PNb;
      if (SCHEME == SCH_N) {
        PNb = ob.v[k];
        plb[i][k] = 0.0;
      } else if (SCHEME == SCH_LDA) {
        PNb = 0.0;
        plb[i][k] = ob.v[k];
      } else {
        const unsigned bit = 1u << (4 * i + k);
        const double sg = (spos & bit) ? 1.0 : ((sneg & bit) ? -1.0 : 0.0);
        PNb = ob.v[k] * th[k] + denb[k] * sg;
        plb[i][k] = ob.v[k] * (1.0 - th[k]);
      }
      if (STAGE == 1) {
        pNb[i][k] = PNb;
      } else {
        pNb[i][k] = 0.5 * PNb;
        s2b->keepN[i][k] = 0.5 * PNb;
        s2b->dw[i][k] = s2->mass * s2->idt * PNb;
      }
    }
  }
  if (STAGE == 1 && kN0) {
    // cotangents of the kept stage-1 N parts of corners 0 and 1
    const D4 c0 = *kN0, c1 = *kN1;
    for (int k = 0; k < 4; ++k) {
      pNb[0][k] += c0.v[k];
      pNb[1][k] += c1.v[k];
    }
  }
  // corner 2's parts: rhs1 and phi^T minus those of corners 0 and 1
  double phiTb[4];
  for (int k = 0; k < 4; ++k) {
    rhs1b[k] += plb[2][k];
    phiTb[k] = pNb[2][k];
    for (int i = 0; i < 2; ++i) {
      plb[i][k] -= plb[2][k];
      pNb[i][k] -= pNb[2][k];
    }
  }
  for (int i = 0; i < 2; ++i) {
    double yN[4], yb[4] = {0, 0, 0, 0};
    for (int k = 0; k < 4; ++k) yN[k] = dWh[i][k] + xN[k];
    apply_split_bar(q, kc[i], kc[i].l3p, kc[i].h1p, kc[i].h2p, xL, plb[i], xLb, qb, kb[i], kb[i].l3p, kb[i].h1p,
                    kb[i].h2p);
    apply_split_bar(q, kc[i], kc[i].l3p, kc[i].h1p, kc[i].h2p, yN, pNb[i], yb, qb, kb[i], kb[i].l3p, kb[i].h1p,
                    kb[i].h2p);
    for (int k = 0; k < 4; ++k) {
      dWhb[i][k] += yb[k];
      xNb[k] += yb[k];
    }
  }
  // x = A^{-1} b: b_bar = A^{-T} x_bar, A_bar = -(bN_bar xN^T + rhs_bar xL^T)
  double bNb[4], rb[4];
  for (int c = 0; c < 4; ++c) {
    bNb[c] = Ai[0][c] * xNb[0] + Ai[1][c] * xNb[1] + Ai[2][c] * xNb[2] + Ai[3][c] * xNb[3];
    rb[c] = Ai[0][c] * xLb[0] + Ai[1][c] * xLb[1] + Ai[2][c] * xLb[2] + Ai[3][c] * xLb[3];
  }
  for (int k = 0; k < 4; ++k) rhs1b[k] += rb[k];
  if (STAGE == 1) {
    const D4 ct = kT ? *kT : D4{{0.0, 0.0, 0.0, 0.0}};
    for (int k = 0; k < 4; ++k) phiTb[k] += rhs1b[k] + ct.v[k];
  } else {
    for (int k = 0; k < 4; ++k) {
      phiTb[k] += 0.5 * rhs1b[k];
      s2b->keepT[k] = 0.5 * rhs1b[k];
      const double rateb = s2->mass * rhs1b[k] * s2->idt;
      for (int i = 0; i < 3; ++i) s2b->dw[i][k] += rateb;
    }
  }
  // corners: (l3, h1, h2)^{+-} from the eigenvalues, w = u nx + v ny; a
  // corner's coefficients are reversed as soon as its cotangents are complete
  // (corner 0 after the matrix A, corners 1 and 2 after their K^- and K
  // products), which ends their live ranges early
  auto corner_bar = [&](int i) {
    const Corner<double>& k = kc[i];
    // the eigenvalues again, as the forward part forms them
    const double l[3] = {k.w + q.c, k.w - q.c, k.w};
    const double p[3] = {rmax(l[0], 0.0), rmax(l[1], 0.0), rmax(l[2], 0.0)};
    const double m[3] = {rmin(l[0], 0.0), rmin(l[1], 0.0), rmin(l[2], 0.0)};
    const double sh = k.s * hic;
    double pb[3] = {0, 0, 0}, mb[3] = {0, 0, 0};
    pb[2] += k.s * kb[i].l3p;
    mb[2] += k.s * kb[i].l3m;
    pb[0] += sh * kb[i].h1p;
    pb[2] -= sh * kb[i].h1p;
    pb[1] += sh * kb[i].h2p;
    pb[2] -= sh * kb[i].h2p;
    mb[0] += sh * kb[i].h1m;
    mb[2] -= sh * kb[i].h1m;
    mb[1] += sh * kb[i].h2m;
    mb[2] -= sh * kb[i].h2m;
    const double shb = kb[i].h1p * (p[0] - p[2]) + kb[i].h2p * (p[1] - p[2]) + kb[i].h1m * (m[0] - m[2]) +
                       kb[i].h2m * (m[1] - m[2]);
    qb.ic += 0.5 * k.s * shb;
    double lb[3];
    for (int j = 0; j < 3; ++j) lb[j] = (l[j] > 0.0 ? pb[j] : 0.0) + (l[j] < 0.0 ? mb[j] : 0.0);
    const double wb = kb[i].w + lb[0] + lb[1] + lb[2];
    qb.c += lb[0] - lb[1];
    qb.u += wb * k.nx;
    qb.v += wb * k.ny;
  };
  build_A_bar(q, kc, bNb, xN, rb, xL, qb, kb);
  corner_bar(0);
  for (int i = 1; i < 3; ++i) {
    apply_split_bar(q, kc[i], kc[i].l3m, kc[i].h1m, kc[i].h2m, dWh[i], bNb, dWhb[i], qb, kb[i], kb[i].l3m, kb[i].h1m,
                    kb[i].h2m);
    apply_full_bar(q, kc[i], dWh[i], phiTb, dWhb[i], qb, kb[i]);
    corner_bar(i);
  }
  // Roe average and dW = M(zbar)(Z_i - Z_0)
  double zbb[4] = {0, 0, 0, 0}, dzb[3][4];
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 4; ++k) dzb[i][k] = 0.0;
  for (int i = 1; i < 3; ++i) {
    const double* g = dWhb[i];
    const double* z = dz[i];
    zbb[0] += 2.0 * z[0] * g[0];
    dzb[i][0] += 2.0 * zb[0] * g[0];
    zbb[1] += z[0] * g[1];
    dzb[i][0] += zb[1] * g[1];
    zbb[0] += z[1] * g[1];
    dzb[i][1] += zb[0] * g[1];
    zbb[2] += z[0] * g[2];
    dzb[i][0] += zb[2] * g[2];
    zbb[0] += z[2] * g[2];
    dzb[i][2] += zb[0] * g[2];
    const double t3 = g[3] * igam;
    zbb[3] += z[0] * t3;
    dzb[i][0] += zb[3] * t3;
    zbb[1] += q.g1 * z[1] * t3;
    dzb[i][1] += q.g1 * zb[1] * t3;
    zbb[2] += q.g1 * z[2] * t3;
    dzb[i][2] += q.g1 * zb[2] * t3;
    zbb[0] += z[3] * t3;
    dzb[i][3] += zb[0] * t3;
  }
  // ac = g1 q2 ic / 2, uc = u ic, vc = v ic, ic = 1/c, c = sqrt(g1 (h - q2/2)), q2 = u^2 + v^2
  double q2b = 0.5 * q.g1 * q.ic * qb.ac;
  qb.ic += 0.5 * q.g1 * q2 * qb.ac;
  qb.u += q.ic * qb.uc;
  qb.ic += q.u * qb.uc;
  qb.v += q.ic * qb.vc;
  qb.ic += q.v * qb.vc;
  qb.c += -q.ic * q.ic * qb.ic;
  const double c2b = 0.5 * qb.c * q.ic;
  qb.h += q.g1 * c2b;
  q2b += -0.5 * q.g1 * c2b;
  qb.u += 2.0 * q.u * q2b;
  qb.v += 2.0 * q.v * q2b;
  // u = zb1/zb0, v = zb2/zb0, h = zb3/zb0
  zbb[1] += iz * qb.u;
  zbb[2] += iz * qb.v;
  zbb[3] += iz * qb.h;
  const double izb = zb[1] * qb.u + zb[2] * qb.v + zb[3] * qb.h;
  zbb[0] += -iz * iz * izb;
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 4; ++k) Zb[i][k] = zbb[k] * third;
  for (int i = 1; i < 3; ++i)
    for (int k = 0; k < 4; ++k) {
      Zb[i][k] += dzb[i][k];
      Zb[0][k] -= dzb[i][k];
    }
  return singular;
}

// Transpose of W -> Z at one state: Wb += (dZ/dW)^T Zb.
__host__ __device__ inline void z_of_w_bar(const double w[4], double gamma, const double Zb[4], double Wb[4]) {
  const double g1 = gamma - 1.0;
  const double rho = w[0], u = w[1] / rho, v = w[2] / rho;
  const double s = sqrt(rho);
  const double p = g1 * (w[3] - 0.5 * rho * (u * u + v * v));
  const double Z3 = (w[3] + p) / s;
  const double is = 1.0 / s;
  // Z0 = s, Z1 = m/s, Z2 = n/s, Z3 = (gamma e - g1 (m^2+n^2)/(2 rho)) / s
  Wb[0] += Zb[0] * 0.5 * is - Zb[1] * 0.5 * u * is - Zb[2] * 0.5 * v * is +
           Zb[3] * (0.5 * g1 * (u * u + v * v) * is - 0.5 * Z3 / rho);
  Wb[1] += Zb[1] * is - Zb[3] * g1 * u * is;
  Wb[2] += Zb[2] * is - Zb[3] * g1 * v * is;
  Wb[3] += Zb[3] * gamma * is;
}

// Transpose of one wall flux F = -v_n (rho, rho u, rho v, rho h) at state w:
// Wb += (dF/dW)^T Fb.
__host__ __device__ inline void wall_flux_bar(const double w[4], double gamma, double nx, double ny, const double Fb[4],
                                              double Wb[4]) {
  const double g1 = gamma - 1.0;
  const double rho = w[0], u = w[1] / rho, v = w[2] / rho;
  const double p = g1 * (w[3] - 0.5 * rho * (u * u + v * v));
  const double vn = u * nx + v * ny;
  const double G[4] = {w[0], w[1], w[2], w[3] + p};
  const double GtF = G[0] * Fb[0] + G[1] * Fb[1] + G[2] * Fb[2] + G[3] * Fb[3];
  // dvn/dW = (-vn/rho, nx/rho, ny/rho, 0); dG/dW = I + e3 (g1 q^2/2, -g1 u, -g1 v, g1)
  Wb[0] += -GtF * (-vn / rho) - vn * (Fb[0] + Fb[3] * 0.5 * g1 * (u * u + v * v));
  Wb[1] += -GtF * (nx / rho) - vn * (Fb[1] - Fb[3] * g1 * u);
  Wb[2] += -GtF * (ny / rho) - vn * (Fb[2] - Fb[3] * g1 * v);
  Wb[3] += -vn * (Fb[3] * (1.0 + g1));
}

}  // namespace rd

namespace rd {

// mu = -(dt / V) lam at a vertex whose update uses its residual (0 at ghosts).
template <class L>
__host__ __device__ inline void mu_of(const Dev& d, const L& lam, int64_t v, double mu[4]) {
  const bool ghost = d.bc && is_ghost(d.bc[v]);
  const double f = ghost ? 0.0 : -d.dt[0] / d.V[v];
  const D4 l = lam.at(v);
  for (int k = 0; k < 4; ++k) mu[k] = f * l.v[k];
}

// Unwrapped inward normals (scaled by edge length) and area of a triangle
// from its corner coordinates.
__host__ __device__ inline void tri_normals_p(const Dev& d, const double2 p[3], double nxd[3], double nyd[3],
                                              double* area) {
  const double d1x = unwrap(p[1].x - p[0].x, d.px, d.hpx), d1y = unwrap(p[1].y - p[0].y, d.py, d.hpy);
  const double d2x = unwrap(p[2].x - p[0].x, d.px, d.hpx), d2y = unwrap(p[2].y - p[0].y, d.py, d.hpy);
  nxd[0] = -(d2y - d1y);
  nxd[1] = d2y;
  nxd[2] = -d1y;
  nyd[0] = d2x - d1x;
  nyd[1] = -d2x;
  nyd[2] = d1x;
  if (area) *area = 0.5 * (d1x * d2y - d1y * d2x);
}

// Inputs of one triangle's reverse: the corners' part slots, corner
// coordinates, parameter vectors and mu; for stage 2 the records W* - W^n
// and the kept stage-1 N parts of corners 0, 1 and residual; for stage 1
// (after a stage 2) the cotangents of those kept values. mu (through MU's
// get(i)) and the records (through P) are read where the reverse uses them.
template <class P, class MU>
struct AdjTriIn {
  int32_t slot[3];  // part slots of the corners
  double2 p[3];
  D4 z[3];
  MU mu;
  P dw[3];
  P kn[2];
  P kt;
};

// Stage-2 reverse of one triangle: cotangents of Z*, W* - W^n (CSR order) and
// of the kept stage-1 parts (triangle order), from mu2 = -(dt/V) dL/dW^{n+1}.
template <int SCHEME, class P, class MU>
__host__ __device__ inline void adj_tri2_compute(int64_t t, const Dev& d, const AdjDev& a, const AdjTriIn<P, MU>& in) {
  double nxd[3], nyd[3], area;
  tri_normals_p(d, in.p, nxd, nyd, &area);
  Stage2In<P> s2;
  s2.mass = area * (1.0 / 3.0);
  s2.idt = a.idt;
  s2.kn[0] = in.kn[0];
  s2.kn[1] = in.kn[1];
  s2.kt = in.kt;
  for (int i = 0; i < 3; ++i) s2.dw[i] = in.dw[i];
  Stage2Bar s2b;
  double Zb[3][4];
  if (tri_adjoint<SCHEME, 2, P, MU>(in.z, nxd, nyd, d.gamma, d.igamma, in.mu, P{}, P{}, P{}, &s2, &s2b, Zb))
    a.flag[1] = 1;
  for (int i = 0; i < 3; ++i) {
    plane_store<double, false>(a.cZW, d.ns, in.slot[i], 0, Zb[i]);
    plane_store<double, false>(a.cZW, d.ns, in.slot[i], 1, s2b.dw[i]);
  }
  // the kept stage-1 values are corners 0 and 1 and phi^T (corner 2 = phi^T
  // minus the other two), so corner 2's cotangent moves onto those three
  double b[3][4];
  for (int k = 0; k < 4; ++k) {
    b[0][k] = s2b.keepN[0][k] - s2b.keepN[2][k];
    b[1][k] = s2b.keepN[1][k] - s2b.keepN[2][k];
    b[2][k] = s2b.keepT[k] + s2b.keepN[2][k];
  }
  plane_store<double, false>(a.kN, d.nt, t, 0, b[0]);
  plane_store<double, false>(a.kN, d.nt, t, 1, b[1]);
  plane_store<double, false>(a.kT, d.nt, t, 0, b[2]);
}

// Stage-1 reverse of one triangle: cotangents of Z^n (CSR order), from
// mu1 = -(dt/V) dL/dW* and the cotangents of the kept parts (in.kn, in.kt;
// null after a forward Euler step).
template <int SCHEME, class P, class MU>
__host__ __device__ inline void adj_tri1_compute(int64_t, const Dev& d, const AdjDev& a, const AdjTriIn<P, MU>& in) {
  double nxd[3], nyd[3];
  tri_normals_p(d, in.p, nxd, nyd, nullptr);
  double Zb[3][4];
  if (tri_adjoint<SCHEME, 1, P, MU>(in.z, nxd, nyd, d.gamma, d.igamma, in.mu, in.kn[0], in.kn[1], in.kt, nullptr,
                                    nullptr, Zb))
    a.flag[1] = 1;
  for (int i = 0; i < 3; ++i) plane_store<double, false>(a.cZ, d.ns, in.slot[i], 0, Zb[i]);
}

// Wall-term transpose at one wall vertex b: sum over its wall edges of
// (dF_v/dW_v)^T (|e|/2)(alpha mu_v + (1 - alpha) mu_other), mu = cotangent of
// the wall term (mu_of(lamA) * sa, plus mu_of(lamB) * sb when useB).
template <class LA, class LB>
__host__ __device__ inline void wall_bar(const Dev& d, int64_t v, const D4* src, const LA& lamA, double sa,
                                         const LB& lamB, double sb, bool useB, double Wb[4]) {
  const int32_t b = d.bc ? wall_index(d.bc[v]) : -1;
  if (b < 0) return;
  const double alpha = 0.75;
  const D4 wv = src[v];
  double ms[4], mo[4], t1[4], t2[4];
  mu_of(d, lamA, v, t1);
  if (useB) mu_of(d, lamB, v, t2);
  for (int k = 0; k < 4; ++k) ms[k] = sa * t1[k] + (useB ? sb * t2[k] : 0.0);
  for (int32_t e = d.wptr[b]; e < d.wptr[b + 1]; ++e) {
    const WallEnt we = d.went[e];
    mu_of(d, lamA, we.other, t1);
    if (useB) mu_of(d, lamB, we.other, t2);
    for (int k = 0; k < 4; ++k) mo[k] = sa * t1[k] + (useB ? sb * t2[k] : 0.0);
    double Fb[4];
    for (int k = 0; k < 4; ++k) Fb[k] = we.hl * (alpha * ms[k] + (1.0 - alpha) * mo[k]);
    wall_flux_bar(wv.v, d.gamma, we.nx, we.ny, Fb, Wb);
  }
}

// Reverse of the stage-2 vertex sums: dL/dW* and the W^n part of W* - W^n.
__host__ __device__ inline void adj_gather2_body(int64_t v, const Dev& d, const AdjDev& a) {
  double zb[4] = {0, 0, 0, 0}, wb[4] = {0, 0, 0, 0};
  const int32_t deg = d.row[v + 1] - d.row[v];
  const int64_t s0 = vslot(d, v);
  auto ld = [&](int32_t j) {
    const int64_t s = s0 + 64 * (int64_t)j;
    ZW c;
    c.z = plane_load<double>(a.cZW, d.ns, s, 0);
    c.w = plane_load<double>(a.cZW, d.ns, s, 1);
    return c;
  };
  for_loaded(deg, ld, [&](int32_t, const ZW& c) {
    for (int k = 0; k < 4; ++k) {
      zb[k] += c.z.v[k];
      wb[k] += c.w.v[k];
    }
  });
  const D4 ws = d.Ws[v], l = a.lam.at(v);
  double ls[4];
  for (int k = 0; k < 4; ++k) ls[k] = l.v[k] + wb[k];
  z_of_w_bar(ws.v, d.gamma, zb, ls);
  wall_bar(d, v, d.Ws, a.lam, 0.5, a.lam, 0.0, false, ls);
  st4<double>(a.lamS, v, ls);
  double ln[4];
  for (int k = 0; k < 4; ++k) ln[k] = -wb[k];
  st4<double>(a.lamN, v, ln);
  // the stage-1 reverse's record of this vertex: Z at W^n and mu1
  AdjRec1 r;
  r.zn = a.Zn[v];
  double mu[4];
  mu_of(d, LamAoS{a.lamS}, v, mu);
  for (int k = 0; k < 4; ++k) r.mu.v[k] = mu[k];
  a.r1[v] = r;
}

// The adjoint's recomputation of the first stage at one vertex: the sums of
// the stage-1 parts and the update (the arithmetic of the stage-1 gather,
// so W* is bitwise the forward step's), writing W* and the vertex's
// stage-2 reverse record: Z at W* (at W^n on ghosts), W* - W^n, mu2.
__host__ __device__ inline void adj_star_body(int64_t v, const Dev& d, const AdjDev& a) {
  const int32_t code = d.bc ? d.bc[v] : -1;
  AdjRec2 r;
  double mu[4];
  mu_of(d, a.lam, v, mu);
  for (int k = 0; k < 4; ++k) r.mu.v[k] = mu[k];
  if (is_ghost(code)) {
    d.Ws[v] = d.W[v];
    r.zc = a.Zn[v];
    for (int k = 0; k < 4; ++k) r.dw.v[k] = 0.0;
    a.r2[v] = r;
    return;
  }
  const int32_t b = wall_index(code);
  double acc[4];
  const int32_t deg = d.row[v + 1] - d.row[v];
  const int64_t s0 = vslot(d, v);
  sum_parts<double>(deg, [&](int32_t j) { return part_load<double>(d, s0 + 64 * (int64_t)j); }, acc);
  if (b >= 0) {
    const D4 wn = d.WCn[b];
    for (int k = 0; k < 4; ++k) acc[k] = acc[k] + wn.v[k];
  }
  const double f = d.dt[0] / d.V[v];
  const D4 win = d.W[v];
  double wo[4];
  vertex_update(win.v, f, acc, wo);
  st4<double>(d.Ws, v, wo);
  const VertexDerived o = derive(d.gamma, wo);
  for (int k = 0; k < 4; ++k) {
    r.zc.v[k] = o.z[k];
    r.dw.v[k] = wo[k] - win.v[k];
  }
  a.r2[v] = r;
  if (!o.ok) d.flag[0] = 1;
}

// Forward Euler: dL/dW* is dL/dW^{n+1} itself; the stage-1 reverse's record
// and the running sums are set from it.
__host__ __device__ inline void adj_euler_prep_body(int64_t v, const Dev& d, const AdjDev& a) {
  const D4 l = a.lam.at(v);
  a.lamS[v] = l;
  const D4 z = {{0.0, 0.0, 0.0, 0.0}};
  a.lamN[v] = z;
  AdjRec1 r;
  r.zn = a.Zn[v];
  double mu[4];
  mu_of(d, a.lam, v, mu);
  for (int k = 0; k < 4; ++k) r.mu.v[k] = mu[k];
  a.r1[v] = r;
}

// Reverse of the stage-1 vertex sums and of W -> Z at W^n: dL/dW^n, written
// structure-of-arrays to out.
__host__ __device__ inline void adj_gather1_body(int64_t v, const Dev& d, const AdjDev& a, bool rk2, double* out) {
  double zb[4] = {0, 0, 0, 0};
  const int32_t deg = d.row[v + 1] - d.row[v];
  const int64_t s0 = vslot(d, v);
  for_loaded(deg, [&](int32_t j) { return plane_load<double>(a.cZ, d.ns, s0 + 64 * (int64_t)j, 0); },
             [&](int32_t, const D4& cz) {
    for (int k = 0; k < 4; ++k) zb[k] += cz.v[k];
  });
  const D4 w = d.W[v], ls = a.lamS[v], ln = a.lamN[v];
  double r[4];
  for (int k = 0; k < 4; ++k) r[k] = ln.v[k] + ls.v[k];
  z_of_w_bar(w.v, d.gamma, zb, r);
  // wall term at W^n: cotangent mu1 (stage 1) + mu2 / 2 (stage 2)
  wall_bar(d, v, d.W, LamAoS{a.lamS}, 1.0, a.lam, 0.5, rk2, r);
  for (int k = 0; k < 4; ++k) out[k * d.nv + v] = r[k];
}

}  // namespace rd
