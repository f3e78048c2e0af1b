// Bodies of the tiled (fused) step.
//
// One workgroup takes one tile of triangles (built on the host, see
// rd_tiling.h) in three phases separated by workgroup barriers:
//   load  - each local vertex's coordinates, parameter vector (and signal
//           speed, or for stage 2 the first-stage state and its difference
//           from W^n) go from HBM to LDS once;
//   tri   - each triangle runs the triangle body on its LDS corners; the
//           parts of tile-interior vertices stay in LDS, those of shared
//           vertices go to the shared part buffer;
//   sum   - each interior vertex sums its parts in LDS, ascending triangle
//           id, and is finished: stage 1 (or Euler) stores the vertex
//           residual R1 (and the CFL bound), stage 2 the new state.
// Shared vertices are finished by a vertex pass over the shared list. Stage 1
// never forms W* in HBM: stage 2 (and the wall term at W*) rebuild it as
// W^n - (dt/V) R1, by the arithmetic of the two-pass gather.
#pragma once

#include "rd_device.h"

namespace rd {

struct Tiles {
  int32_t ntiles = 0, tt = 0;
  int32_t max_lv = 0, max_lvi = 0, max_slots = 0;
  int64_t nsv = 0, nss = 0;
  const int32_t* tbeg = nullptr;  // [ntiles+1] tile-major triangle slots
  const int32_t* vbeg = nullptr;  // [ntiles+1] local vertex ranges in tvl
  const int32_t* nvi = nullptr;   // [ntiles] interior vertices (first in each range)
  const int32_t* lpb = nullptr;   // [ntiles] offset of the tile's LDS part ranges in lp
  const int32_t* lp = nullptr;    // nvi + 1 bounds per tile
  const int32_t* tvl = nullptr;   // local -> global vertex
  const uint16_t* lv = nullptr;   // [3][nt] local vertex of each corner, by slot
  const int32_t* dst = nullptr;   // [3][nt] >= 0 shared part slot, < 0 LDS slot -1 - dst
  const int32_t* tmesh = nullptr; // [ntiles] mesh id (batches) or null
  const int32_t* sv = nullptr;    // [nsv] shared vertices
  const int32_t* ssbeg = nullptr; // [nsv] first shared part slot (stride 64)
  void* Cs = nullptr;             // [nss] shared parts (D4 or F4)
  double* lams = nullptr;         // [nss] shared CFL terms
};

// LDS carve-up of one tile workgroup.
template <typename R>
struct TileLds {
  double2* xy = nullptr;  // [max_lv]
  Q4<R>* Z = nullptr;     // [max_lv] parameter vector (at W^n, or W* in stage 2)
  Q4<R>* dW = nullptr;    // [max_lv] stage 2: W* - W^n
  D4* Ws = nullptr;       // [max_lvi] stage 2: W* of interior vertices
  double* sig = nullptr;  // [max_lv] CFL: signal speed
  double* lam = nullptr;  // [max_slots] CFL: l_max lambda_max per interior corner
  Q4<R>* P = nullptr;     // [max_slots] parts of interior corners
};

__host__ __device__ inline size_t lds_align(size_t x) { return (x + 31) & ~size_t(31); }

// Bytes of LDS a tile workgroup needs; with base != null also sets out.
template <typename R>
__host__ __device__ inline size_t tile_lds(const Tiles& tl, int stage, bool cfl, char* base, TileLds<R>* out) {
  size_t o = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + o : nullptr;
    o = lds_align(o + bytes);
    return p;
  };
  TileLds<R> L;
  L.xy = reinterpret_cast<double2*>(take(sizeof(double2) * tl.max_lv));
  L.Z = reinterpret_cast<Q4<R>*>(take(sizeof(Q4<R>) * tl.max_lv));
  if (stage == 2) {
    L.dW = reinterpret_cast<Q4<R>*>(take(sizeof(Q4<R>) * tl.max_lv));
    L.Ws = reinterpret_cast<D4*>(take(sizeof(D4) * tl.max_lvi));
  }
  if (cfl) {
    L.sig = reinterpret_cast<double*>(take(sizeof(double) * tl.max_lv));
    L.lam = reinterpret_cast<double*>(take(sizeof(double) * tl.max_slots));
  }
  L.P = reinterpret_cast<Q4<R>*>(take(sizeof(Q4<R>) * tl.max_slots));
  if (out) *out = L;
  return o;
}

__host__ __device__ inline int tile_mesh(const Tiles& tl, int64_t tile) { return tl.tmesh ? tl.tmesh[tile] : 0; }

// Triangle IO of the tiled form.
template <typename R>
struct TileIO {
  // fast FP64 reciprocals in the triangle body (see rcp)
  static constexpr bool kFastDiv = true;
  const TileLds<R>& L;
  int lvi[3];
  int32_t dst[3];
  void* Cs;
  double* lams;
  R idt_;
  const double* vr_;
  __host__ __device__ R idt(int64_t) const { return idt_; }
  __host__ __device__ const double* vr(int64_t) const { return vr_; }
  __host__ __device__ Q4<R> dw(int i) const { return L.dW[lvi[i]]; }
  __host__ __device__ void part(int i, const R out[4]) const {
    Q4<R> q;
    for (int k = 0; k < 4; ++k) q.v[k] = out[k];
    if (dst[i] < 0) L.P[-1 - dst[i]] = q;
    else reinterpret_cast<Q4<R>*>(Cs)[dst[i]] = q;
  }
  // the triangle's CFL term goes to each of its corners (interior corners in
  // LDS, shared ones to the shared-slot buffer)
  __host__ __device__ void cfl(int64_t, double x) const {
    for (int i = 0; i < 3; ++i) {
      if (dst[i] < 0) L.lam[-1 - dst[i]] = x;
      else lams[dst[i]] = x;
    }
  }
};

// ---- phase bodies (tile = workgroup id, l / j = local vertex / triangle) --

template <typename R, bool CFL>
__host__ __device__ inline void tile_load1(int64_t tile, int32_t l, const Dev& d, const Tiles& tl,
                                           const TileLds<R>& L) {
  const int32_t v = tl.tvl[tl.vbeg[tile] + l];
  L.xy[l] = d.xy[v];
  L.Z[l] = zbuf<R>(d)[v];
  if (CFL) L.sig[l] = d.sig[v];
}

template <typename R>
__host__ __device__ inline void tile_load2(int64_t tile, int32_t l, const Dev& d, const Tiles& tl,
                                           const TileLds<R>& L) {
  const int32_t v = tl.tvl[tl.vbeg[tile] + l];
  L.xy[l] = d.xy[v];
  const int32_t code = d.bc ? d.bc[v] : -1;
  Q4<R> dw;
  if (is_ghost(code)) {
    L.Z[l] = zbuf<R>(d)[v];
    for (int k = 0; k < 4; ++k) dw.v[k] = R(0);
    L.dW[l] = dw;
    return;
  }
  const D4 win = d.W[v];
  const D4 ws = star_state(d, v, code, tile_mesh(tl, tile));
  for (int k = 0; k < 4; ++k) dw.v[k] = (R)(ws.v[k] - win.v[k]);
  L.dW[l] = dw;
  const VertexDerived o = derive(d.gamma, ws.v);
  L.Z[l] = zq<R>(o);
  if (!o.ok) d.flag[tile_mesh(tl, tile)] = 1;
  if (l < tl.nvi[tile]) L.Ws[l] = ws;
}

template <typename R, int SCHEME, int STAGE, bool SAVE, bool CFL, bool LUMP = false>
__host__ __device__ inline void tile_tri(int64_t tile, int32_t j, const Dev& d, const Tiles& tl,
                                         const TileLds<R>& L) {
  const int64_t s = (int64_t)tl.tbeg[tile] + j;
  const int64_t nt = d.nt;
  TileIO<R> io{L, {0, 0, 0}, {0, 0, 0}, tl.Cs, tl.lams, R(0), d.vr + 3 * tile_mesh(tl, tile)};
  TriIn<R> in;
  for (int i = 0; i < 3; ++i) {
    const int q = tl.lv[i * nt + s];
    io.lvi[i] = q;
    io.dst[i] = tl.dst[i * nt + s];
    in.p[i] = L.xy[q];
    in.Z[i] = L.Z[q];
    if (CFL) in.sig[i] = L.sig[q];
  }
  if (STAGE == 2) io.idt_ = (R)(1.0 / d.dt[tile_mesh(tl, tile)]);
  tri_compute<R, SCHEME, STAGE, SAVE, CFL, LUMP>(s, in, d, io);
}

// Stage-1 (or Euler) sum of interior vertex l: R1 = sum of parts + wall term,
// and with CFL the vertex bound 2 V / sum l_max lambda_max.
template <typename R, bool CFL>
__host__ __device__ inline void tile_sum1(int64_t tile, int32_t l, const Dev& d, const Tiles& tl,
                                          const TileLds<R>& L) {
  const int32_t v = tl.tvl[tl.vbeg[tile] + l];
  const int32_t* lp = tl.lp + tl.lpb[tile];
  const int32_t a = lp[l], n = lp[l + 1] - a;
  if (CFL) {
    double acc = 0.0;
    for (int32_t j = 0; j < n; ++j) acc += L.lam[a + j];
    d.cflv[v] = 2.0 * d.V[v] / acc;
  }
  const int32_t code = d.bc ? d.bc[v] : -1;
  if (is_ghost(code)) return;
  D4 acc;
  sum_parts<R>(n, [&](int32_t j) { return L.P[a + j]; }, acc.v);
  const int32_t b = wall_index(code);
  if (b >= 0) {
    const D4 wn = d.WCn[b];
    for (int k = 0; k < 4; ++k) acc.v[k] = acc.v[k] + wn.v[k];
  }
  d.R1[v] = acc;
}

// Stage-2 sum and update of interior vertex l.
template <typename R>
__host__ __device__ inline void tile_sum2(int64_t tile, int32_t l, const Dev& d, const Tiles& tl,
                                          const TileLds<R>& L) {
  const int32_t v = tl.tvl[tl.vbeg[tile] + l];
  const int32_t code = d.bc ? d.bc[v] : -1;
  if (is_ghost(code)) return;
  const int32_t* lp = tl.lp + tl.lpb[tile];
  const int32_t a = lp[l], n = lp[l + 1] - a;
  double acc[4];
  sum_parts<R>(n, [&](int32_t j) { return L.P[a + j]; }, acc);
  const int32_t b = wall_index(code);
  if (b >= 0) {
    const D4 wn = d.WCn[b], ws = d.WCs[b];
    for (int k = 0; k < 4; ++k) acc[k] = acc[k] + 0.5 * (wn.v[k] + ws.v[k]);
  }
  const double f = d.dt[tile_mesh(tl, tile)] / d.V[v];
  const D4 win = L.Ws[l];
  double wo[4];
  vertex_update(win.v, f, acc, wo);
  st4<double>(d.W, v, wo);
  vertex_epilogue(d, v, wo, sizeof(R) != sizeof(double));
}

// Shared vertex k, stage 1 (or Euler): as tile_sum1 over the shared buffer.
template <typename R, bool CFL>
__host__ __device__ inline void shared_sum1(int64_t k, const Dev& d, const Tiles& tl) {
  const int32_t v = tl.sv[k];
  const int32_t n = d.row[v + 1] - d.row[v];
  const int64_t s0 = tl.ssbeg[k];
  if (CFL) {
    double acc = 0.0;
    for_loaded(n, [&](int32_t j) { return tl.lams[s0 + 64 * (int64_t)j]; }, [&](int32_t, double x) { acc += x; });
    d.cflv[v] = 2.0 * d.V[v] / acc;
  }
  const int32_t code = d.bc ? d.bc[v] : -1;
  if (is_ghost(code)) return;
  D4 acc;
  sum_parts<R>(n, [&](int32_t j) { return ld4<R>(tl.Cs, s0 + 64 * (int64_t)j); }, acc.v);
  const int32_t b = wall_index(code);
  if (b >= 0) {
    const D4 wn = d.WCn[b];
    for (int k = 0; k < 4; ++k) acc.v[k] = acc.v[k] + wn.v[k];
  }
  d.R1[v] = acc;
}

// Shared vertex k, stage 2: rebuild W*, sum, update.
template <typename R>
__host__ __device__ inline void shared_sum2(int64_t k, const Dev& d, const Tiles& tl) {
  const int32_t v = tl.sv[k];
  const int32_t code = d.bc ? d.bc[v] : -1;
  if (is_ghost(code)) return;
  const int m = d.vmesh ? d.vmesh[v] : 0;
  const D4 ws = star_state(d, v, code, m);
  const int32_t n = d.row[v + 1] - d.row[v];
  const int64_t s0 = tl.ssbeg[k];
  double acc[4];
  sum_parts<R>(n, [&](int32_t j) { return ld4<R>(tl.Cs, s0 + 64 * (int64_t)j); }, acc);
  const int32_t b = wall_index(code);
  if (b >= 0) {
    const D4 wn = d.WCn[b], wcs = d.WCs[b];
    for (int q = 0; q < 4; ++q) acc[q] = acc[q] + 0.5 * (wn.v[q] + wcs.v[q]);
  }
  const double f = d.dt[m] / d.V[v];
  double wo[4];
  vertex_update(ws.v, f, acc, wo);
  st4<double>(d.W, v, wo);
  vertex_epilogue(d, v, wo, sizeof(R) != sizeof(double));
}

// Forward-Euler update of vertex v from R1.
__host__ __device__ inline void euler_apply(int64_t v, const Dev& d, bool fp32) {
  const int32_t code = d.bc ? d.bc[v] : -1;
  if (is_ghost(code)) return;
  const D4 wo = star_state(d, v, code, d.vmesh ? d.vmesh[v] : 0);
  d.W[v] = wo;
  vertex_epilogue(d, v, wo.v, fp32);
}

}  // namespace rd
