// Per-element bodies of the residual-distribution step for gfx950.
//
// One triangle body computes, for one triangle, everything Sections 3.2-3.4
// ask of it: the Roe average of its three parameter vectors, the positive and
// negative parts of the three K_i, the triangle residual, the N and LDA
// distributions (one 4x4 pivoted solve with two right-hand sides), the B
// blend, and for the second Runge-Kutta stage the total residuals. One vertex
// body sums a vertex's parts over the vertex->(triangle, corner) CSR in
// ascending triangle order (no atomics), adds the wall term and updates the
// state, then refreshes the parameter vector and signal speed of the vertex.
//
// Parts are stored sliced: vertices are taken 64 at a time (one wavefront of
// the gather), a slice is as wide as its largest vertex degree, and the j-th
// part (ascending triangle order) of the slice's l-th vertex sits at
// slice_base + 64 j + l. The triangle passes write each corner's part
// straight to its slot; the gather's j-th load is then one contiguous,
// fully coalesced read across the wavefront. A corner's slot is formed from
// its vertex v (slice v / 64, lane v % 64) and the rank j of the triangle
// among v's triangles; the three ranks of a triangle are packed 10 bits
// each into one word, so a triangle pass reads 4 bytes of slot data per
// triangle instead of three 32-bit slot positions.
//
// Algebra used on the GPU (equal in exact arithmetic to Appendix A's explicit
// entries): with unit normal n, Roe state (u, v, h, c), w = u n_x + v n_y,
//   E = (1, u, v, h), N = (0, n_x, n_y, w),
//   g(y) = alpha/c y0 - (gamma-1)(u/c y1 + v/c y2 - y3/c),
//   d(y) = -w y0 + n_x y1 + n_y y2,
// the matrix with eigenvalues (l1, l2, l3, l3) on the acoustic and the two
// linear waves acts as
//   K(l) y = l3 y + (l1-l3)/(2c) (g+d) (E + c N) + (l2-l3)/(2c) (g-d) (E - c N),
// i.e. K(l) = l3 I + (l1-l3) r1 l1^T + (l2-l3) r2 l2^T with r_{1,2} = E +- c N
// the acoustic right eigenvectors and l_{1,2}^T the matching rows of R^{-1}.
// This needs no 4x4 matrix per corner; only A = sum_i K_i^+ is built.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace rd {

template <typename R>
struct alignas(4 * sizeof(R)) Q4 {
  R v[4];
};
using D4 = Q4<double>;
using F4 = Q4<float>;

// One wall-edge incidence of a wall vertex (Section 3.5).
struct alignas(16) WallEnt {
  int32_t other;  // the edge's other vertex
  int32_t role;   // 0: this vertex is the edge's start a, 1: its end b
  double hl;      // half the edge length
  double nx, ny;  // outward unit normal
};

enum { SCH_N = 0, SCH_LDA = 1, SCH_B = 2, SCH_BMAX = 3, SCH_BMIN = 4, SCH_BX = 5 };
enum { G_EULER = 0, G_STAGE1 = 1, G_STAGE2 = 2, G_RESIDUAL = 3 };

// Device view of one mesh (or of a batch laid end to end).
struct Dev {
  int64_t nv = 0, nt = 0;
  int32_t nwv = 0;
  double gamma = 1.4, px = 0.0, py = 0.0;
  double hpx = 0.0, hpy = 0.0;  // half periods, +inf on an axis that is not periodic
  double igamma = 1.0 / 1.4;  // 1 / gamma (set with gamma on the host)
  // geometry and connectivity
  const double2* xy = nullptr;   // [nv]
  const double* V = nullptr;     // [nv] vertex volume
  const int32_t* row = nullptr;  // [nv+1] CSR row pointers (row[v+1] - row[v] = degree of v)
  const int32_t* sbase = nullptr; // [ceil(nv/64)] first part slot of each 64-vertex slice
  int64_t ns = 0;                // part slots, including the padding of the 64-vertex slices
  const int32_t* vtri = nullptr; // [ns] triangle of each part slot (padding slots unused)
  const int32_t* bc = nullptr;   // [nv] or null: boundary code, see is_ghost / wall_index
  const int32_t* tv = nullptr;   // [3][nt] corner vertex ids
  const uint32_t* rk = nullptr;  // [nt] rank of t among the triangles of corner i's vertex, bits 10 i .. 10 i + 9
  const int32_t* wv = nullptr;   // [nwv] wall vertex ids
  const int32_t* wptr = nullptr; // [nwv+1]
  const WallEnt* went = nullptr; // wall incidences, ascending edge id per vertex
  const int32_t* tmesh = nullptr; // [nt] mesh id (batch) or null
  const int32_t* vmesh = nullptr; // [nv] mesh id (batch) or null
  // state
  D4* W = nullptr;    // [nv] state
  D4* Ws = nullptr;   // [nv] first-stage state
  D4* Z = nullptr;    // [nv] parameter vector (FP64 arithmetic)
  F4* Zf = nullptr;   // [nv] parameter vector (FP32 arithmetic)
  void* dW = nullptr; // [nv] W* - W^n (D4 or F4)
  double* sig = nullptr;   // [nv] |v| + c
  // triangle buffers
  void* C = nullptr;      // [ns] distributed parts, sliced layout (D4 or F4 records in 16-byte planes)
  void* keepN = nullptr;  // stage-1 N parts of corners 0 and 1 (2 nt records, D4 or F4; 16-byte planes)
  void* keepT = nullptr;  // stage-1 triangle residual (nt records, D4 or F4; 16-byte planes)
  D4* WCn = nullptr;      // [nwv] wall term at W^n
  D4* WCs = nullptr;      // [nwv] wall term at W*
  void* lam = nullptr;    // [nt] l_max^T lambda_max^T per triangle: float from the FP32 triangle
                          // passes, double from the FP64 ones and from the CFL-only pass
  double* dt = nullptr;   // [n meshes] time step
  double* vr = nullptr;   // [3 per mesh] Bx sensor: smallest and largest |v| at the stage's state, domain size L
  int slump = 0;          // selective lumping in stage 2 (else global lumping)
  int* flag = nullptr;    // non-physical state latch, one per mesh (batch) or one
  // tiled form
  D4* R1 = nullptr;       // [nv] stage-1 (or Euler) vertex residual, wall term included
  double* cflv = nullptr; // [nv] 2 V_i / sum_T l_max^T lambda_max^T
};

// Boundary code of a vertex: -1 interior, -2 ghost, b >= 0 wall vertex b,
// -3 - b ghost that is also wall vertex b (its wall term is never applied,
// but its state enters its neighbours' wall terms).
__host__ __device__ inline bool is_ghost(int32_t bc) { return bc == -2 || bc <= -3; }
__host__ __device__ inline int32_t wall_index(int32_t bc) { return bc >= 0 ? bc : (bc <= -3 ? -3 - bc : -1); }

// First part slot of vertex v: its j-th part is at vslot(d, v) + 64 j.
__host__ __device__ inline int64_t vslot(const Dev& d, int64_t v) { return (int64_t)d.sbase[v >> 6] + (v & 63); }

// Part slot of corner i (vertex v) of a triangle with rank word rk.
__host__ __device__ inline int32_t corner_slot(const Dev& d, int32_t v, uint32_t rk, int i) {
  return d.sbase[v >> 6] + (v & 63) + 64 * (int32_t)((rk >> (10 * i)) & 1023u);
}

// Periodic difference: d shifted by one period into [-period/2, period/2]
// on a periodic axis. The half period is given: 0.5 period (exact) on a
// periodic axis, +inf on another (no difference exceeds it), so the
// comparisons read it where it is, with nothing to keep per thread.
__host__ __device__ inline double unwrap(double d, double period, double half) {
  if (d > half) d -= period;
  else if (d < -half) d += period;
  return d;
}

// The same value, selected rather than branched to (the forward triangle
// bodies: no basic-block boundaries between their loads and arithmetic).
__host__ __device__ inline double unwrap_select(double d, double period, double half) {
  const double hi = d - period, lo = d + period;
  return d > half ? hi : (d < -half ? lo : d);
}

// max / min of non-NaN values (one v_max / v_min instruction; the sign of a
// zero result is unspecified, which no result depends on).
template <typename R> __host__ __device__ inline R rmax(R a, R b) { return fmax(a, b); }
template <typename R> __host__ __device__ inline R rmin(R a, R b) { return fmin(a, b); }

// Reciprocal. FP64 with FD (fast division): the hardware approximation
// refined by two Newton-Raphson steps r <- r + r (1 - x r), each of which
// about squares the relative error, so the result is within about an ulp of
// 1/x; where a step is not finite (x zero or infinite, or so small that 1/x
// overflows) the hardware value is kept. FP64 without FD: IEEE division.
// FP32: the hardware reciprocal (about 1 ulp), whose error budget is set by
// FP32 rounding anyway.
template <bool FD = true>
__host__ __device__ inline double rcp(double x) {
#ifdef __HIP_DEVICE_COMPILE__
  if (FD) {
    const double r0 = __builtin_amdgcn_rcp(x);
    double r = fma(r0, fma(-x, r0, 1.0), r0);
    r = fma(r, fma(-x, r, 1.0), r);
    return r == r ? r : r0;
  }
#endif
  return 1.0 / x;
}
template <bool FD = true>
__host__ __device__ inline float rcp(float x) {
#ifdef __HIP_DEVICE_COMPILE__
  return __builtin_amdgcn_rcpf(x);
#else
  return 1.0f / x;
#endif
}

// Length L = sqrt(e2) > 0 and its reciprocal (e2 is a squared edge length or
// the squared sound speed of a Roe state, positive and finite). FP64: iL from
// the hardware reciprocal square root refined by two Newton-Raphson steps
// y <- y + (y / 2)(1 - e2 y^2), and L = e2 iL (each within about an ulp or
// two). FP32: one hardware reciprocal square root (about 1 ulp).
__host__ __device__ inline void len_rcp(double e2, double& L, double& iL) {
#ifdef __HIP_DEVICE_COMPILE__
  double y = __builtin_amdgcn_rsq(e2);
  y = fma(0.5 * y, fma(-(e2 * y), y, 1.0), y);
  y = fma(0.5 * y, fma(-(e2 * y), y, 1.0), y);
  iL = y;
  L = e2 * y;
#else
  L = sqrt(e2);
  iL = 1.0 / L;
#endif
}
__host__ __device__ inline void len_rcp(float e2, float& L, float& iL) {
#ifdef __HIP_DEVICE_COMPILE__
  iL = __builtin_amdgcn_rsqf(e2);
  L = e2 * iL;
#else
  L = sqrtf(e2);
  iL = 1.0f / L;
#endif
}

template <typename R>
__host__ __device__ inline R sel4(int r, R a0, R a1, R a2, R a3) {
  R t = r == 1 ? a1 : a0;
  t = r == 2 ? a2 : t;
  return r == 3 ? a3 : t;
}

// Per-corner coefficients of K_i^{+-} (scaled by s = |n_i|/2).
template <typename R>
struct Corner {
  R nx, ny, w, s;
  R l3p, h1p, h2p;  // s l3^+, s (l1^+ - l3^+)/(2c), s (l2^+ - l3^+)/(2c)
  R l3m, h1m, h2m;  // same for the negative parts
};

template <typename R>
struct Roe {
  R u, v, h, c, ic, ac, uc, vc, g1;
};

// y -> K^{+} y or K^{-} y of one corner.
template <typename R>
__host__ __device__ inline void apply_split(const Roe<R>& q, const Corner<R>& k, R sl3, R h1, R h2,
                                            const R y[4], R out[4]) {
  R g = q.ac * y[0] - q.g1 * (q.uc * y[1] + q.vc * y[2] - q.ic * y[3]);
  R d = -k.w * y[0] + k.nx * y[1] + k.ny * y[2];
  R a1 = h1 * (g + d), a2 = h2 * (g - d);
  R sp = a1 + a2, sm = (a1 - a2) * q.c;
  out[0] = sl3 * y[0] + sp;
  out[1] = sl3 * y[1] + sp * q.u + sm * k.nx;
  out[2] = sl3 * y[2] + sp * q.v + sm * k.ny;
  out[3] = sl3 * y[3] + sp * q.h + sm * k.w;
}

// y -> K y (l = lambda): s (w y + d E + c g N).
template <typename R>
__host__ __device__ inline void apply_full(const Roe<R>& q, const Corner<R>& k, const R y[4], R out[4]) {
  R g = q.ac * y[0] - q.g1 * (q.uc * y[1] + q.vc * y[2] - q.ic * y[3]);
  R d = -k.w * y[0] + k.nx * y[1] + k.ny * y[2];
  R cg = q.c * g;
  out[0] = k.s * (k.w * y[0] + d);
  out[1] = k.s * (k.w * y[1] + d * q.u + cg * k.nx);
  out[2] = k.s * (k.w * y[2] + d * q.v + cg * k.ny);
  out[3] = k.s * (k.w * y[3] + d * q.h + cg * k.w);
}

// A = sum_i K_i^+ as a dense 4x4 matrix:
// A = L3 I + E ev^T + c (sum Q_i N_i) G^T + c sum_i P_i N_i D_i^T with
// P = h1 + h2, Q = h1 - h2, G = (alpha/c, -g1 u/c, -g1 v/c, g1/c), D_i = (-w, nx, ny, 0).
template <typename R>
__host__ __device__ inline void build_A(const Roe<R>& q, const Corner<R> k[3], R A[4][4]) {
  R G[4] = {q.ac, -q.g1 * q.uc, -q.g1 * q.vc, q.g1 * q.ic};
  R E[4] = {R(1), q.u, q.v, q.h};
  R L3 = k[0].l3p + k[1].l3p + k[2].l3p;
  R P[3], Qv[3];
  for (int i = 0; i < 3; ++i) {
    P[i] = k[i].h1p + k[i].h2p;
    Qv[i] = k[i].h1p - k[i].h2p;
  }
  R sP = P[0] + P[1] + P[2];
  R ev[4];
  ev[0] = sP * G[0] - (Qv[0] * k[0].w + Qv[1] * k[1].w + Qv[2] * k[2].w);
  ev[1] = sP * G[1] + (Qv[0] * k[0].nx + Qv[1] * k[1].nx + Qv[2] * k[2].nx);
  ev[2] = sP * G[2] + (Qv[0] * k[0].ny + Qv[1] * k[1].ny + Qv[2] * k[2].ny);
  ev[3] = sP * G[3];
  R nvv[4];
  nvv[0] = R(0);
  nvv[1] = q.c * (Qv[0] * k[0].nx + Qv[1] * k[1].nx + Qv[2] * k[2].nx);
  nvv[2] = q.c * (Qv[0] * k[0].ny + Qv[1] * k[1].ny + Qv[2] * k[2].ny);
  nvv[3] = q.c * (Qv[0] * k[0].w + Qv[1] * k[1].w + Qv[2] * k[2].w);
  // S[r][j] for r = 1..3 (N rows nx, ny, w) and j = 0..2 (D cols -w, nx, ny)
  R S[4][4];
  for (int r = 0; r < 4; ++r)
    for (int j = 0; j < 4; ++j) S[r][j] = R(0);
  for (int i = 0; i < 3; ++i) {
    R cp = q.c * P[i];
    R Nr[4] = {R(0), k[i].nx, k[i].ny, k[i].w};
    R Dc[4] = {-k[i].w, k[i].nx, k[i].ny, R(0)};
    for (int r = 1; r < 4; ++r) {
      R t = cp * Nr[r];
      for (int j = 0; j < 3; ++j) S[r][j] = S[r][j] + t * Dc[j];
    }
  }
  for (int r = 0; r < 4; ++r)
    for (int j = 0; j < 4; ++j) {
      R a = E[r] * ev[j] + nvv[r] * G[j] + S[r][j];
      A[r][j] = r == j ? a + L3 : a;
    }
}

// Gaussian elimination with partial pivoting for two right-hand sides
// (A, b0 and b1 are overwritten).
// Pivot: largest |entry| among rows not yet used, lowest row on ties; a
// column whose best pivot is at most 2^-45 max|A| is skipped and its unknown
// set to 0 (A is singular at stagnation; the K^+ x products stay unique).
// `skipped` reports whether any column was skipped.
template <typename R, bool FD = true>
__host__ __device__ inline void solve2(R A[4][4], R b0[4], R b1[4], R x0[4], R x1[4], bool& skipped) {
  R amax = R(0);
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) amax = rmax(amax, (R)fabs(A[r][c]));
  const R tol = amax * R(2.8421709430404007e-14);  // 2^-45
  bool used[4] = {false, false, false, false};
  R P[4][4], PB0[4], PB1[4], PI[4];
  bool OK[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    R best = R(-1);
    int r = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      R a = (R)fabs(A[i][k]);
      bool take = !used[i] && a > best;
      best = take ? a : best;
      r = take ? i : r;
    }
    const bool ok = best > tol;
    OK[k] = ok;
#pragma unroll
    for (int j = k; j < 4; ++j) P[k][j] = sel4(r, A[0][j], A[1][j], A[2][j], A[3][j]);
    PB0[k] = sel4(r, b0[0], b0[1], b0[2], b0[3]);
    PB1[k] = sel4(r, b1[0], b1[1], b1[2], b1[3]);
    PI[k] = ok ? rcp<FD>(P[k][k]) : R(0);
#pragma unroll
    for (int i = 0; i < 4; ++i) used[i] = used[i] || (ok && r == i);
    // rows not eliminated get factor 0, which leaves them exactly unchanged
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const R f = (ok && !used[i]) ? A[i][k] * PI[k] : R(0);
#pragma unroll
      for (int j = k + 1; j < 4; ++j) A[i][j] = A[i][j] - f * P[k][j];
      b0[i] = b0[i] - f * PB0[k];
      b1[i] = b1[i] - f * PB1[k];
    }
  }
#pragma unroll
  for (int k = 3; k >= 0; --k) {
    R s0 = PB0[k], s1 = PB1[k];
#pragma unroll
    for (int j = k + 1; j < 4; ++j) {
      s0 = s0 - P[k][j] * x0[j];
      s1 = s1 - P[k][j] * x1[j];
    }
    x0[k] = OK[k] ? s0 * PI[k] : R(0);
    x1[k] = OK[k] ? s1 * PI[k] : R(0);
  }
  skipped = !(OK[0] && OK[1] && OK[2] && OK[3]);
}

template <typename R, bool FD = true>
__host__ __device__ inline void solve2(R A[4][4], R b0[4], R b1[4], R x0[4], R x1[4]) {
  bool skipped;
  solve2<R, FD>(A, b0, b1, x0, x1, skipped);
}

// Blend of Section 3.3.3: Theta_k = |res_k| / sum_i |N_{i,k}| (0 if the sum is
// 0, at most 1); BMAX / BMIN use the largest / smallest Theta_k for all k.
// den_k = sum_i |N_{i,k}| is accumulated by the caller in corner order.
// The quotient is a |res_k| times the reciprocal of den_k; where that product
// is not below 1 (the clamp, or a reciprocal that overflowed because den_k
// is below ~1/DBL_MAX, as happens at the edge of a uniform state at rest
// where the parts have decayed to subnormal values) the exact quotient
// decides.
template <typename R, int SCHEME, bool FD = true>
__host__ __device__ inline void blend_theta(const R res[4], const R den[4], R th[4]) {
  for (int k = 0; k < 4; ++k) {
    const R a = (R)fabs(res[k]);
    R q = R(0);
    if (den[k] > R(0) && a > R(0)) {
      q = a * rcp<FD>(den[k]);
      if (!(q < R(1))) q = a < den[k] ? a / den[k] : R(1);
    }
    th[k] = q;
  }
  if (SCHEME == SCH_BMAX || SCHEME == SCH_BMIN) {
    R t = th[0];
    for (int k = 1; k < 4; ++k) {
      bool better = SCHEME == SCH_BMAX ? th[k] > t : th[k] < t;
      t = better ? th[k] : t;
    }
    for (int k = 0; k < 4; ++k) th[k] = t;
  }
}

template <typename R>
__host__ __device__ inline Q4<R> ld4(const void* base, int64_t i) {
  return reinterpret_cast<const Q4<R>*>(base)[i];
}
template <typename R>
__host__ __device__ inline void st4(void* base, int64_t i, const R a[4]) {
  Q4<R> q;
  q.v[0] = a[0];
  q.v[1] = a[1];
  q.v[2] = a[2];
  q.v[3] = a[3];
  reinterpret_cast<Q4<R>*>(base)[i] = q;
}

// Records of four reals in planes of 16-byte chunks: chunk c of record j of
// item i sits at chunk index (KC j + c) n + i, where n is the number of items
// and KC the number of chunks per record (2 for FP64, 1 for FP32). One store
// or load instruction of a wavefront over consecutive items then covers one
// contiguous kilobyte instead of a strided span of partly written lines.
// Used for the distributed parts (item = part slot, one record) and for the
// kept stage-1 records of a triangle (N parts of corners 0 and 1 in keepN,
// phi^T in keepT), which are read back only by the stage-2 pass, after the
// gather: those are stored non-temporally (NT), so that they do not evict
// from the caches the parts and parameter vectors the next kernel reads.
template <typename R> struct Chunk16;
template <> struct Chunk16<double> { typedef double V __attribute__((ext_vector_type(2))); };
template <> struct Chunk16<float> { typedef float V __attribute__((ext_vector_type(4))); };

template <typename R, bool NT>
__host__ __device__ inline void plane_store(void* base, int64_t n, int64_t i, int j, const R a[4]) {
  typedef typename Chunk16<R>::V V;
  constexpr int per = 16 / sizeof(R), kc = 4 / per;
  V* p = reinterpret_cast<V*>(base);
  for (int c = 0; c < kc; ++c) {
    V q;
    for (int e = 0; e < per; ++e) q[e] = a[c * per + e];
#ifdef __HIP_DEVICE_COMPILE__
    if (NT) __builtin_nontemporal_store(q, p + (kc * j + c) * n + i);
    else p[(kc * j + c) * n + i] = q;
#else
    p[(kc * j + c) * n + i] = q;
#endif
  }
}

template <typename R>
__host__ __device__ inline Q4<R> plane_load(const void* base, int64_t n, int64_t i, int j) {
  typedef typename Chunk16<R>::V V;
  constexpr int per = 16 / sizeof(R), kc = 4 / per;
  const V* p = reinterpret_cast<const V*>(base);
  Q4<R> q;
  for (int c = 0; c < kc; ++c) {
    const V x = p[(kc * j + c) * n + i];
    for (int e = 0; e < per; ++e) q.v[c * per + e] = x[e];
  }
  return q;
}

template <typename R>
__host__ __device__ inline void keep_store(void* base, int64_t nt, int64_t t, int j, const R a[4]) {
  plane_store<R, true>(base, nt, t, j, a);
}
template <typename R>
__host__ __device__ inline Q4<R> keep_load(const void* base, int64_t nt, int64_t t, int j) {
  return plane_load<R>(base, nt, t, j);
}
// Part of slot s in C.
template <typename R>
__host__ __device__ inline void part_store(const Dev& d, int64_t s, const R a[4]) {
  plane_store<R, false>(d.C, d.ns, s, 0, a);
}
template <typename R>
__host__ __device__ inline Q4<R> part_load(const Dev& d, int64_t s) {
  return plane_load<R>(d.C, d.ns, s, 0);
}

template <typename R> __host__ __device__ inline const Q4<R>* zbuf(const Dev& d);
template <> __host__ __device__ inline const Q4<double>* zbuf<double>(const Dev& d) { return d.Z; }
template <> __host__ __device__ inline const Q4<float>* zbuf<float>(const Dev& d) { return d.Zf; }

// One triangle, stage 1 (STAGE = 1) or stage 2 (STAGE = 2) of Section 3.4.
// Stage 1 writes the scheme's parts phi_i to C and, when SAVE, keeps phi^N_i
// and phi^T for stage 2. Stage 2 forms the total residuals
//   Phi^N_i = |T|/3 (W*_i - W^n_i)/dt + (phi^N_i(n) + phi^N_i(*))/2,
//   Phi^T   = |T|/3 sum_j (W*_j - W^n_j)/dt + (phi^T(n) + phi^T(*))/2,
//   Phi^LDA_i = K_i^+(*) A(*)^{-1} Phi^T,
// blends them and writes them to C.
// The loads of one triangle, split in two so a kernel can issue them for the
// next triangle while it computes the current one: corner ids and CSR
// positions first, then the vertex records they point to.
template <typename R>
struct TriIn {
  int32_t iv[3], ip[3];
  uint32_t rk;
  double2 p[3];
  Q4<R> Z[3];
  double sig[3];
};

template <typename R>
__host__ __device__ inline void tri_load_ids(int64_t t, const Dev& d, TriIn<R>& in) {
  const int64_t nt = d.nt;
  for (int i = 0; i < 3; ++i) in.iv[i] = d.tv[i * nt + t];
  in.rk = d.rk[t];
}

template <typename R, bool CFL>
__host__ __device__ inline void tri_load_verts(const Dev& d, TriIn<R>& in) {
  const Q4<R>* Zp = zbuf<R>(d);
  for (int i = 0; i < 3; ++i) {
    in.p[i] = d.xy[in.iv[i]];
    in.Z[i] = Zp[in.iv[i]];
    if (CFL) in.sig[i] = d.sig[in.iv[i]];
    in.ip[i] = corner_slot(d, in.iv[i], in.rk, i);
  }
}

// Where a triangle body reads the stage-1 differences W* - W^n of its corners
// and sends its parts: GlobalIO is the two-pass form (vertex arrays and the
// sliced part buffer in HBM); the tiled form has its own (LDS-staged) IO.
// `t` indexes the triangle's saved stage-1 values (keepN, keepT).
// FD: fast FP64 reciprocals in the triangle body (see rcp), else IEEE
// division.
template <typename R, bool FD = true>
struct GlobalIO {
  static constexpr bool kFastDiv = FD;
  const Dev& d;
  const int32_t* iv;
  const int32_t* ip;
  __host__ __device__ R idt(int64_t t) const { return (R)(1.0 / d.dt[d.tmesh ? d.tmesh[t] : 0]); }
  __host__ __device__ const double* vr(int64_t t) const { return d.vr + 3 * (d.tmesh ? d.tmesh[t] : 0); }
  __host__ __device__ Q4<R> dw(int i) const { return reinterpret_cast<const Q4<R>*>(d.dW)[iv[i]]; }
  __host__ __device__ void part(int i, const R out[4]) const {
    part_store<R>(d, ip[i], out);
  }
  __host__ __device__ void cfl(int64_t t, double x) const { reinterpret_cast<R*>(d.lam)[t] = (R)x; }
  // Where the corner coefficients wait while the 4x4 solve runs (kept in
  // registers here; see CornerLds).
};

// LUMP (stage 2 only): selective lumping of Section 3.4 instead of global lumping.
template <typename R, int SCHEME, int STAGE, bool SAVE, bool CFL, bool LUMP = false, class IO>
__host__ __device__ inline void tri_compute(int64_t t, const TriIn<R>& in, const Dev& d, const IO& io) {
  constexpr bool FD = IO::kFastDiv;
  const double2 p0 = in.p[0], p1 = in.p[1], p2 = in.p[2];
  const double d1x = unwrap_select(p1.x - p0.x, d.px, d.hpx), d1y = unwrap_select(p1.y - p0.y, d.py, d.hpy);
  const double d2x = unwrap_select(p2.x - p0.x, d.px, d.hpx), d2y = unwrap_select(p2.y - p0.y, d.py, d.hpy);
  // inward normals scaled by edge length: rotate the opposite edge by +90 degrees
  const double nxd[3] = {-(d2y - d1y), d2y, -d1y};
  const double nyd[3] = {d2x - d1x, -d2x, d1x};

  const Q4<R>* Zc = in.Z;

  // Bx blend coefficient (Section 3.3.3): theta = min(1, s^2 h / L) with the
  // shock sensor s = (-L div v / (|v|max - |v|min))^+, div v that of the
  // linear interpolant of the corner velocities (u = Z_1 / Z_0, v = Z_2 / Z_0),
  // h = sqrt(2 |T|); |v|min, |v|max (at this stage's state) and the domain
  // size L of the triangle's mesh come from io.vr.
  R bx = R(0);
  if (SCHEME == SCH_BX) {
    const double* r = io.vr(t);
    R div = R(0);
    for (int i = 0; i < 3; ++i) div = div + (Zc[i].v[1] * (R)nxd[i] + Zc[i].v[2] * (R)nyd[i]) / Zc[i].v[0];
    const double a2 = d1x * d2y - d1y * d2x;  // 2 |T|
    const R range = (R)(r[1] - r[0]), L = (R)r[2];
    const R sn = range > R(0) ? rmax(-(L * div) / ((R)a2 * range), R(0)) : R(0);
    bx = rmin(sn * sn * (R)sqrt(a2) / L, R(1));
  }

  const R gam = (R)d.gamma;
  Roe<R> q;
  q.g1 = gam - R(1);
  const R third = R(1) / R(3);
  R zb[4];
  for (int k = 0; k < 4; ++k) zb[k] = (Zc[0].v[k] + Zc[1].v[k] + Zc[2].v[k]) * third;
  const R iz = rcp<FD>(zb[0]);
  q.u = zb[1] * iz;
  q.v = zb[2] * iz;
  q.h = zb[3] * iz;
  const R q2 = q.u * q.u + q.v * q.v;
  len_rcp(q.g1 * (q.h - R(0.5) * q2), q.c, q.ic);
  q.ac = R(0.5) * q.g1 * q2 * q.ic;
  q.uc = q.u * q.ic;
  q.vc = q.v * q.ic;

  // dW_i = M(Zbar)(Z_i - Z_0), M = dW/dZ
  R dWh[3][4];
  const R igam = (R)d.igamma;
  for (int k = 0; k < 4; ++k) dWh[0][k] = R(0);
  for (int i = 1; i < 3; ++i) {
    R dz[4];
    for (int k = 0; k < 4; ++k) dz[k] = Zc[i].v[k] - Zc[0].v[k];
    dWh[i][0] = R(2) * zb[0] * dz[0];
    dWh[i][1] = zb[1] * dz[0] + zb[0] * dz[1];
    dWh[i][2] = zb[2] * dz[0] + zb[0] * dz[2];
    dWh[i][3] = (zb[3] * dz[0] + q.g1 * (zb[1] * dz[1] + zb[2] * dz[2]) + zb[0] * dz[3]) * igam;
  }

  Corner<R> kc[3];
  const R hic = R(0.5) * q.ic;
  R lmax = R(0);
  for (int i = 0; i < 3; ++i) {
    // edge geometry in the algebra's precision, from FP64 coordinate differences
    const R ex = (R)nxd[i], ey = (R)nyd[i];
    R L, iL;
    len_rcp(ex * ex + ey * ey, L, iL);
    lmax = rmax(lmax, L);
    Corner<R>& k = kc[i];
    k.nx = ex * iL;
    k.ny = ey * iL;
    k.s = R(0.5) * L;
    k.w = q.u * k.nx + q.v * k.ny;
    const R l1 = k.w + q.c, l2 = k.w - q.c, l3 = k.w;
    const R p1 = rmax(l1, R(0)), p2 = rmax(l2, R(0)), p3 = rmax(l3, R(0));
    const R m1 = rmin(l1, R(0)), m2 = rmin(l2, R(0)), m3 = rmin(l3, R(0));
    const R sh = k.s * hic;
    k.l3p = k.s * p3;
    k.h1p = sh * (p1 - p3);
    k.h2p = sh * (p2 - p3);
    k.l3m = k.s * m3;
    k.h1m = sh * (m1 - m3);
    k.h2m = sh * (m2 - m3);
  }

  if (CFL) {
    // CFL limit of Section 3.2: l_max^T max_j(|v_j| + c_j) of the triangle
    double lam = 0.0;
    for (int i = 0; i < 3; ++i) lam = rmax(lam, in.sig[i]);
    io.cfl(t, (double)lmax * lam);
  }

  // triangle residual and the N right-hand side
  R phiT[4], bN[4], t1[4], t2[4];
  apply_full(q, kc[1], dWh[1], t1);
  apply_full(q, kc[2], dWh[2], t2);
  for (int k = 0; k < 4; ++k) phiT[k] = t1[k] + t2[k];
  R A[4][4];
  build_A(q, kc, A);

  constexpr bool needN = SCHEME != SCH_LDA;
  constexpr bool needL = SCHEME != SCH_N;
  R pN[3][4];
  R rhs1[4];
  R mass = R(0), idt = R(0);
  if (needN) {
    apply_split(q, kc[1], kc[1].l3m, kc[1].h1m, kc[1].h2m, dWh[1], t1);
    apply_split(q, kc[2], kc[2].l3m, kc[2].h1m, kc[2].h2m, dWh[2], t2);
    for (int k = 0; k < 4; ++k) bN[k] = t1[k] + t2[k];
  } else {
    for (int k = 0; k < 4; ++k) bN[k] = R(0);
  }
  if (STAGE == 1) {
    for (int k = 0; k < 4; ++k) rhs1[k] = phiT[k];
  } else {
    idt = io.idt(t);
    mass = (R)((0.5 * (d1x * d2y - d1y * d2x)) * (1.0 / 3.0));
    if (needL) {
      R srate[4] = {R(0), R(0), R(0), R(0)};
      for (int i = 0; i < 3; ++i) {
        const Q4<R> dwv = io.dw(i);
        for (int k = 0; k < 4; ++k) srate[k] = srate[k] + dwv.v[k] * idt;
      }
      const Q4<R> kt = keep_load<R>(d.keepT, d.nt, t, 0);
      for (int k = 0; k < 4; ++k) rhs1[k] = mass * srate[k] + R(0.5) * (kt.v[k] + phiT[k]);
    } else {
      for (int k = 0; k < 4; ++k) rhs1[k] = R(0);
    }
  }
  R xN[4], xL[4], b0[4], b1[4];
  for (int k = 0; k < 4; ++k) {
    b0[k] = bN[k];
    b1[k] = rhs1[k];
  }
  solve2<R, FD>(A, b0, b1, xN, xL);
  // Corner parts. The parts of a distribution sum to the residual they
  // split (sum_i K_i^+ = A): sum_i K_i^+ (dW_i + xN) = phi^T and
  // sum_i K_i^+ xL = rhs1, so corner 2's parts are the residual minus those
  // of corners 0 and 1 (exact in exact arithmetic; saves two K^+ products).
  R pl[3][4];
  if (needL) {
    apply_split(q, kc[0], kc[0].l3p, kc[0].h1p, kc[0].h2p, xL, pl[0]);
    apply_split(q, kc[1], kc[1].l3p, kc[1].h1p, kc[1].h2p, xL, pl[1]);
    for (int k = 0; k < 4; ++k) pl[2][k] = rhs1[k] - pl[0][k] - pl[1][k];
  }
  // Selective lumping (Section 3.4, stage 2): the N and LDA total parts both
  // get sum_j (|T| delta_ij / 3 - m^G_ij) (W*_j - W^n_j) / dt with the
  // Galerkin mass m^G_ij = |T| (1 + delta_ij) / 12, that is
  // (|T| / 12) (3 r_i - r_0 - r_1 - r_2) with r = (W* - W^n) / dt.
  R sl[3][4];
  if (STAGE == 2 && LUMP) {
    R rs[4] = {R(0), R(0), R(0), R(0)};
    for (int i = 0; i < 3; ++i) {
      const Q4<R> dwv = io.dw(i);
      for (int k = 0; k < 4; ++k) {
        sl[i][k] = dwv.v[k] * idt;
        rs[k] = rs[k] + sl[i][k];
      }
    }
    const R m12 = mass * R(0.25);
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 4; ++k) sl[i][k] = m12 * (R(3) * sl[i][k] - rs[k]);
    if (needL)
      for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 4; ++k) pl[i][k] = pl[i][k] + sl[i][k];
  }
  R den[4] = {R(0), R(0), R(0), R(0)};
  if (needN) {
    for (int i = 0; i < 2; ++i) {
      R y[4];
      for (int k = 0; k < 4; ++k) y[k] = dWh[i][k] + xN[k];
      apply_split(q, kc[i], kc[i].l3p, kc[i].h1p, kc[i].h2p, y, pN[i]);
    }
    for (int k = 0; k < 4; ++k) pN[2][k] = phiT[k] - pN[0][k] - pN[1][k];
    // Only corners 0 and 1 of the N parts are kept: corner 2's is phi^T minus
    // those two, and stage 2 forms it again from the kept phi^T with the same
    // two subtractions, which gives back the identical value.
    if (STAGE == 1 && SAVE) {
      keep_store<R>(d.keepN, d.nt, t, 0, pN[0]);
      keep_store<R>(d.keepN, d.nt, t, 1, pN[1]);
    }
    if (STAGE == 2) {
      // Phi^N_i = |T|/3 (W*_i - W^n_i)/dt + (phi^N_i(n) + phi^N_i(*))/2; the
      // kept parts and per-vertex differences are loaded here (cached) to
      // keep them out of registers across the solve
      const Q4<R> k0 = keep_load<R>(d.keepN, d.nt, t, 0), k1 = keep_load<R>(d.keepN, d.nt, t, 1),
                  kt = keep_load<R>(d.keepT, d.nt, t, 0);
      R kn[3][4];
      for (int k = 0; k < 4; ++k) {
        kn[0][k] = k0.v[k];
        kn[1][k] = k1.v[k];
        kn[2][k] = kt.v[k] - k0.v[k] - k1.v[k];
      }
      for (int i = 0; i < 3; ++i) {
        const Q4<R> dwv = io.dw(i);
        for (int k = 0; k < 4; ++k) pN[i][k] = mass * (dwv.v[k] * idt) + R(0.5) * (kn[i][k] + pN[i][k]);
      }
      if (LUMP)
        for (int i = 0; i < 3; ++i)
          for (int k = 0; k < 4; ++k) pN[i][k] = pN[i][k] + sl[i][k];
    }
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 4; ++k) den[k] = den[k] + (R)fabs(pN[i][k]);
  }
  if (STAGE == 1 && SAVE) keep_store<R>(d.keepT, d.nt, t, 0, phiT);
  // rhs1 is the residual being split (phi^T or Phi^T)
  R th[4] = {R(0), R(0), R(0), R(0)};
  if (SCHEME >= SCH_B && SCHEME <= SCH_BMIN) blend_theta<R, SCHEME, FD>(rhs1, den, th);
  if (SCHEME == SCH_BX)
    for (int k = 0; k < 4; ++k) th[k] = bx;
  for (int i = 0; i < 3; ++i) {
    R out[4];
    for (int k = 0; k < 4; ++k) {
      if (SCHEME == SCH_N) out[k] = pN[i][k];
      else if (SCHEME == SCH_LDA) out[k] = pl[i][k];
      else out[k] = pl[i][k] + th[k] * (pN[i][k] - pl[i][k]);
    }
    io.part(i, out);
  }
}

template <typename R, int SCHEME, int STAGE, bool SAVE, bool CFL, bool LUMP = false, bool FD = true>
__host__ __device__ inline void tri_body(int64_t t, const Dev& d) {
  TriIn<R> in;
  tri_load_ids<R>(t, d, in);
  tri_load_verts<R, CFL>(d, in);
  const GlobalIO<R, FD> io{d, in.iv, in.ip};
  tri_compute<R, SCHEME, STAGE, SAVE, CFL, LUMP>(t, in, d, io);
}

// Flow speed |v| of a conserved state.
__host__ __device__ inline double flow_speed(const D4& w) {
  const double u = w.v[1] / w.v[0], v = w.v[2] / w.v[0];
  return sqrt(u * u + v * v);
}

// Parameter vector, signal speed and physicality of one state.
struct VertexDerived {
  double z[4];
  double sig;
  bool ok;
};

// Square root of x >= 0 (NaN for x < 0): on the device from the hardware
// reciprocal square root refined by two Newton-Raphson steps (within about
// an ulp or two; exactly 0 at 0), on the host IEEE.
__host__ __device__ inline double sqrt_nr(double x) {
#ifdef __HIP_DEVICE_COMPILE__
  double y = __builtin_amdgcn_rsq(x);
  y = fma(0.5 * y, fma(-(x * y), y, 1.0), y);
  y = fma(0.5 * y, fma(-(x * y), y, 1.0), y);
  return x == 0.0 ? 0.0 : x * y;
#else
  return sqrt(x);
#endif
}

// Parameter vector Z = sqrt(rho) (1, u, v, h) and |v| + c of a conserved
// state, with one reciprocal of rho (rcp) and Newton-Raphson square roots.
__host__ __device__ inline VertexDerived derive(double gamma, const double w[4]) {
  VertexDerived o;
  const double g1 = gamma - 1.0;
  const double rho = w[0], ir = rcp(rho), u = w[1] * ir, vv = w[2] * ir;
  const double p = g1 * (w[3] - 0.5 * rho * (u * u + vv * vv));
  const double h = (w[3] + p) * ir;
  const double s = sqrt_nr(rho);
  o.z[0] = s;
  o.z[1] = s * u;
  o.z[2] = s * vv;
  o.z[3] = s * h;
  o.sig = sqrt_nr(u * u + vv * vv) + sqrt_nr(gamma * p * ir);
  const bool finite = fabs(o.sig) < INFINITY && fabs(w[1]) < INFINITY && fabs(w[2]) < INFINITY &&
                      fabs(w[3]) < INFINITY;
  o.ok = rho > 0.0 && p > 0.0 && finite;
  return o;
}

template <typename R>
__host__ __device__ inline Q4<R> zq(const VertexDerived& o) {
  Q4<R> q;
  for (int k = 0; k < 4; ++k) q.v[k] = (R)o.z[k];
  return q;
}

// with_sig: also store |v| + c (the CFL limit reads it at the start of a
// step; the first-stage state W* does not need it)
__host__ __device__ inline void vertex_epilogue(const Dev& d, int64_t v, const double w[4], bool fp32,
                                                bool with_sig = true) {
  const VertexDerived o = derive(d.gamma, w);
  if (fp32) d.Zf[v] = zq<float>(o);
  else d.Z[v] = zq<double>(o);
  if (with_sig) d.sig[v] = o.sig;
  if (!o.ok) d.flag[d.vmesh ? d.vmesh[v] : 0] = 1;
}

// f(j, get(j)) for j = 0, ..., n-1 in that order. The loads of four
// consecutive j are issued before any is consumed, so a wavefront keeps
// several independent loads in flight instead of one.
template <class Get, class F>
__host__ __device__ inline void for_loaded(int32_t n, const Get& get, const F& f) {
  using T = decltype(get(0));
  for (int32_t j = 0; j < n; j += 4) {
    T x[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (j + u < n) x[u] = get(j + u);
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (j + u < n) f(j + u, x[u]);
  }
}

// Sum of a vertex's n parts get(0), ..., get(n-1) in that order, in FP64
// (Neumaier-compensated when the parts are FP32).
template <typename R, class Get>
__host__ __device__ inline void sum_parts(int32_t n, const Get& get, double acc[4]) {
  double cmp[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k = 0; k < 4; ++k) acc[k] = 0.0;
  for_loaded(n, get, [&](int32_t, const Q4<R>& c) {
    for (int k = 0; k < 4; ++k) {
      if (sizeof(R) == sizeof(double)) {
        acc[k] += (double)c.v[k];
      } else {
        const double x = (double)c.v[k];
        const double tsum = acc[k] + x;
        cmp[k] += fabs(acc[k]) >= fabs(x) ? (acc[k] - tsum) + x : (x - tsum) + acc[k];
        acc[k] = tsum;
      }
    }
  });
  if (sizeof(R) != sizeof(double))
    for (int k = 0; k < 4; ++k) acc[k] = acc[k] + cmp[k];
}

// The update of Sections 3.3-3.4: out = in - (dt / V) acc.
__host__ __device__ inline void vertex_update(const double in[4], double f, const double acc[4], double out[4]) {
  for (int k = 0; k < 4; ++k) out[k] = in[k] - f * acc[k];
}

// One vertex of the gather (MODE: G_EULER, G_STAGE1, G_STAGE2, G_RESIDUAL).
// R is the arithmetic type of the parts; sums are FP64 (Neumaier-compensated
// when the parts are FP32).
template <typename R, int MODE>
__host__ __device__ inline void gather_body(int64_t v, const Dev& d, double* out_soa) {
  const int32_t code = d.bc ? d.bc[v] : -1;
  const int32_t b = is_ghost(code) ? -1 : wall_index(code);
  if (is_ghost(code) && MODE != G_RESIDUAL) {
    if (MODE == G_STAGE1) {
      d.Ws[v] = d.W[v];
      const R z[4] = {R(0), R(0), R(0), R(0)};
      st4<R>(d.dW, v, z);
    }
    return;
  }
  double acc[4];
  const int32_t deg = d.row[v + 1] - d.row[v];
  const int64_t s0 = vslot(d, v);
  sum_parts<R>(deg, [&](int32_t j) { return part_load<R>(d, s0 + 64 * (int64_t)j); }, acc);
  if (b >= 0) {
    const D4 wn = d.WCn[b];
    if (MODE == G_STAGE2) {
      const D4 ws = d.WCs[b];
      for (int k = 0; k < 4; ++k) acc[k] = acc[k] + 0.5 * (wn.v[k] + ws.v[k]);
    } else {
      for (int k = 0; k < 4; ++k) acc[k] = acc[k] + wn.v[k];
    }
  }
  if (MODE == G_RESIDUAL) {
    for (int k = 0; k < 4; ++k) out_soa[k * d.nv + v] = acc[k];
    return;
  }
  const int m = d.vmesh ? d.vmesh[v] : 0;
  const double f = d.dt[m] / d.V[v];
  const D4 win = MODE == G_STAGE2 ? d.Ws[v] : d.W[v];
  double wo[4];
  vertex_update(win.v, f, acc, wo);
  if (MODE == G_STAGE1) {
    st4<double>(d.Ws, v, wo);
    R dw[4];
    for (int k = 0; k < 4; ++k) dw[k] = (R)(wo[k] - win.v[k]);
    st4<R>(d.dW, v, dw);
  } else {
    st4<double>(d.W, v, wo);
  }
  vertex_epilogue(d, v, wo, sizeof(R) != sizeof(double), MODE != G_STAGE1);
}

// The first-stage state W* = W^n - (dt / V) R1 of vertex v in the tiled form
// (ghosts keep W^n), by the same arithmetic as the two-pass gather.
__host__ __device__ inline D4 star_state(const Dev& d, int64_t v, int32_t code, int m) {
  const D4 win = d.W[v];
  if (is_ghost(code)) return win;
  const double f = d.dt[m] / d.V[v];
  const D4 r = d.R1[v];
  D4 o;
  vertex_update(win.v, f, r.v, o.v);
  return o;
}

// Wall correction of one wall vertex (Section 3.5), at W (STAGE2 = false) or
// W* (held in Ws, or formed from R1 when TILED).
template <bool STAGE2, bool TILED = false>
__host__ __device__ inline void wall_body(int64_t b, const Dev& d) {
  const double alpha = 0.75, g1 = d.gamma - 1.0;
  const D4* src = STAGE2 ? d.Ws : d.W;
  const int32_t v = d.wv[b];
  auto state = [&](int32_t i) -> D4 {
    if (STAGE2 && TILED) return star_state(d, i, d.bc[i], d.vmesh ? d.vmesh[i] : 0);
    return src[i];
  };
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int32_t e = d.wptr[b]; e < d.wptr[b + 1]; ++e) {
    const WallEnt we = d.went[e];
    double F[2][4];
    const int32_t ids[2] = {v, we.other};
    for (int s = 0; s < 2; ++s) {
      const D4 w = state(ids[s]);
      const double u = w.v[1] / w.v[0], vv = w.v[2] / w.v[0];
      const double p = g1 * (w.v[3] - 0.5 * w.v[0] * (u * u + vv * vv));
      const double vn = u * we.nx + vv * we.ny;
      F[s][0] = -vn * w.v[0];
      F[s][1] = -vn * w.v[1];
      F[s][2] = -vn * w.v[2];
      F[s][3] = -vn * (w.v[3] + p);
    }
    for (int k = 0; k < 4; ++k) {
      const double part = we.role == 0 ? alpha * F[0][k] + (1.0 - alpha) * F[1][k]
                                       : (1.0 - alpha) * F[1][k] + alpha * F[0][k];
      acc[k] += we.hl * part;
    }
  }
  st4<double>(STAGE2 ? d.WCs : d.WCn, b, acc);
}

// l_max^T lambda_max^T of one triangle (the same arithmetic as the fused form
// in tri_body).
__host__ __device__ inline void cfl_tri_body(int64_t t, const Dev& d) {
  const int64_t nt = d.nt;
  const int32_t iv[3] = {d.tv[t], d.tv[nt + t], d.tv[2 * nt + t]};
  const double2 p0 = d.xy[iv[0]], p1 = d.xy[iv[1]], p2 = d.xy[iv[2]];
  const double d1x = unwrap_select(p1.x - p0.x, d.px, d.hpx), d1y = unwrap_select(p1.y - p0.y, d.py, d.hpy);
  const double d2x = unwrap_select(p2.x - p0.x, d.px, d.hpx), d2y = unwrap_select(p2.y - p0.y, d.py, d.hpy);
  const double nxd[3] = {-(d2y - d1y), d2y, -d1y};
  const double nyd[3] = {d2x - d1x, -d2x, d1x};
  double lmax = 0.0, lam = 0.0;
  for (int i = 0; i < 3; ++i) {
    lmax = rmax(lmax, (double)sqrt(nxd[i] * nxd[i] + nyd[i] * nyd[i]));
    lam = rmax(lam, d.sig[iv[i]]);
  }
  reinterpret_cast<double*>(d.lam)[t] = lmax * lam;
}

// 2 V_i / sum_{T ni i} l_max lambda_max of U vertices v[u] (terms of type R),
// each vertex's triangles taken in ascending order; out[u] is meaningful
// where in[u]. The triangles of the first J ranks of all U vertices are
// loaded before any term, and all those terms before any sum, so that the U
// chains of dependent loads (row bounds and slice base, triangle, term)
// overlap. Every load is in bounds whatever the degree, so none needs a
// branch: a vertex out of range reads vertex vsafe, a rank past the degree
// rereads the last rank (or slot 0 at degree 0) and its term is replaced by
// an exact zero. Ranks from J on follow one at a time.
template <typename R, int U, int J = 8>
__host__ __device__ inline void cfl_vertex_bounds(const int64_t v[U], const bool in[U], int64_t vsafe,
                                                  const Dev& d, double out[U]) {
  const R* lam = reinterpret_cast<const R*>(d.lam);
  int32_t deg[U];
  int64_t s0[U];
  double vol[U];
  for (int u = 0; u < U; ++u) {
    const int64_t w = in[u] ? v[u] : vsafe;
    deg[u] = d.row[w + 1] - d.row[w];
    s0[u] = vslot(d, w);
    vol[u] = d.V[w];
  }
  int32_t t[U][J];
  for (int u = 0; u < U; ++u)
    for (int j = 0; j < J; ++j) {
      const int64_t k = deg[u] > 0 ? s0[u] + 64 * (int64_t)(j < deg[u] ? j : deg[u] - 1) : 0;
      t[u][j] = d.vtri[k];
    }
  R term[U][J];
  for (int u = 0; u < U; ++u)
    for (int j = 0; j < J; ++j) {
      const R x = lam[t[u][j] > 0 ? t[u][j] : 0];
      term[u][j] = j < deg[u] ? x : R(0);
    }
  for (int u = 0; u < U; ++u) {
    double acc = 0.0;
    for (int j = 0; j < J; ++j) acc += (double)term[u][j];
    for (int32_t j = J; j < deg[u]; ++j) acc += (double)lam[d.vtri[s0[u] + 64 * (int64_t)j]];
    out[u] = 2.0 * vol[u] / acc;
  }
}

}  // namespace rd
