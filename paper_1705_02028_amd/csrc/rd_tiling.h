// Host-side construction of the triangle tiles of the fused step.
//
// Triangles are ordered along a Morton curve of their centroids (within each
// mesh of a batch, on that mesh's own bounding box) and cut into tiles of
// `tt` consecutive triangles; tiles never straddle two meshes. A vertex whose
// triangles all lie in one tile is interior to that tile: the tile sums its
// parts in LDS and finishes it. Every other vertex is shared: its parts go
// to a sliced buffer (64-vertex slices, j-th part of the slice's l-th vertex
// at slice_base + 64 j + l) and a vertex pass sums them. Both sums run over a
// vertex's triangles in ascending triangle id, the order of the two-pass
// form, so both forms give bitwise equal results for every tile size.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <utility>
#include <vector>

namespace rd {

struct TilePlan {
  int32_t tt = 0, ntiles = 0;
  int32_t max_lv = 0, max_lvi = 0, max_slots = 0;
  std::vector<int32_t> order;      // [nt] tile-major slot -> triangle id
  std::vector<int32_t> tbeg;       // [ntiles + 1] slot range of each tile
  std::vector<int32_t> vbeg;       // [ntiles + 1] range of each tile in tvl
  std::vector<int32_t> nvi;        // [ntiles] interior vertices (listed first in tvl)
  std::vector<int32_t> lpb;        // [ntiles] offset of the tile's part ranges in lp
  std::vector<int32_t> lp;         // per tile nvi + 1 LDS slot bounds, one range per interior vertex
  std::vector<int32_t> tvl;        // local vertex -> global vertex
  std::vector<uint16_t> lv;        // [3][nt] local vertex of corner i of slot s, at i nt + s
  std::vector<int32_t> dst;        // [3][nt] >= 0: shared part slot; < 0: LDS part slot -1 - dst
  std::vector<int32_t> tmesh;      // [ntiles] mesh of each tile
  std::vector<int32_t> sv;         // shared vertices, ascending
  std::vector<int32_t> ssbeg;      // [nsv] first slot of each shared vertex (stride 64)
  int64_t nss = 0;                 // shared part slots (with slice padding)
};

inline double tiling_unwrap(double d, double period) {
  if (period > 0.0) {
    if (d > 0.5 * period) d -= period;
    else if (d < -0.5 * period) d += period;
  }
  return d;
}

inline uint32_t morton_spread(uint32_t v) {
  v &= 0xffffu;
  v = (v | (v << 8)) & 0x00ff00ffu;
  v = (v | (v << 4)) & 0x0f0f0f0fu;
  v = (v | (v << 2)) & 0x33333333u;
  v = (v | (v << 1)) & 0x55555555u;
  return v;
}

// Builds the tiles of a mesh made of `voff.size() - 1` consecutive meshes
// (vertex ranges voff[k]..voff[k+1], triangle ranges toff[k]..toff[k+1]).
// row/slot: vertex -> corner CSR (corner 3 t + i), ascending t in each row.
// Returns an empty string on success, else the reason.
inline std::string build_tile_plan(int64_t nv, int64_t nt, const int32_t* tri, const double* x, const double* y,
                                   double px, double py, const int32_t* row, const int32_t* slot,
                                   const std::vector<int64_t>& voff, const std::vector<int64_t>& toff, int32_t tt,
                                   TilePlan& P) {
  if (tt < 1 || tt > 1024) return "tile size out of range";
  P = TilePlan();
  P.tt = tt;
  const size_t nmesh = voff.size() - 1;
  // Morton order of centroids within each mesh
  P.order.resize(nt);
  std::vector<std::pair<uint32_t, int32_t>> key;
  std::vector<int32_t> tile_of(nt);
  P.tbeg.push_back(0);
  for (size_t k = 0; k < nmesh; ++k) {
    double x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
    for (int64_t v = voff[k]; v < voff[k + 1]; ++v) {
      x0 = std::min(x0, x[v]);
      x1 = std::max(x1, x[v]);
      y0 = std::min(y0, y[v]);
      y1 = std::max(y1, y[v]);
    }
    double ext = std::max(x1 - x0, y1 - y0);
    if (!(ext > 0.0)) ext = 1.0;
    key.clear();
    for (int64_t t = toff[k]; t < toff[k + 1]; ++t) {
      const int32_t a = tri[3 * t], b = tri[3 * t + 1], c = tri[3 * t + 2];
      double cx = x[a] + (tiling_unwrap(x[b] - x[a], px) + tiling_unwrap(x[c] - x[a], px)) / 3.0;
      double cy = y[a] + (tiling_unwrap(y[b] - y[a], py) + tiling_unwrap(y[c] - y[a], py)) / 3.0;
      if (px > 0.0) cx = x0 + (cx - x0) - px * std::floor((cx - x0) / px);
      if (py > 0.0) cy = y0 + (cy - y0) - py * std::floor((cy - y0) / py);
      const double fx = std::min(std::max((cx - x0) / ext, 0.0), 1.0);
      const double fy = std::min(std::max((cy - y0) / ext, 0.0), 1.0);
      const uint32_t qx = (uint32_t)std::min(65535.0, std::floor(fx * 65536.0));
      const uint32_t qy = (uint32_t)std::min(65535.0, std::floor(fy * 65536.0));
      key.emplace_back(morton_spread(qx) | (morton_spread(qy) << 1), (int32_t)t);
    }
    std::sort(key.begin(), key.end());
    const int64_t base = toff[k];
    for (size_t j = 0; j < key.size(); ++j) P.order[base + j] = key[j].second;
    for (int64_t s = toff[k]; s < toff[k + 1]; s += tt) {
      const int64_t e = std::min<int64_t>(s + tt, toff[k + 1]);
      const int32_t id = (int32_t)P.tbeg.size() - 1;
      for (int64_t q = s; q < e; ++q) tile_of[P.order[q]] = id;
      P.tbeg.push_back((int32_t)e);
      P.tmesh.push_back((int32_t)k);
    }
  }
  P.ntiles = (int32_t)P.tmesh.size();

  // interior / shared classification and the shared sliced layout
  std::vector<uint8_t> shared(nv, 0);
  for (int64_t v = 0; v < nv; ++v) {
    const int32_t t0 = tile_of[slot[row[v]] / 3];
    for (int32_t j = row[v] + 1; j < row[v + 1]; ++j)
      if (tile_of[slot[j] / 3] != t0) {
        shared[v] = 1;
        break;
      }
    if (shared[v]) P.sv.push_back((int32_t)v);
  }
  std::vector<int32_t> cdst(3 * nt, 0);
  const int64_t nsv = (int64_t)P.sv.size();
  P.ssbeg.resize(nsv);
  int64_t base = 0;
  for (int64_t g0 = 0; g0 < nsv; g0 += 64) {
    const int64_t g1 = std::min<int64_t>(g0 + 64, nsv);
    int32_t width = 0;
    for (int64_t k = g0; k < g1; ++k) width = std::max(width, row[P.sv[k] + 1] - row[P.sv[k]]);
    for (int64_t k = g0; k < g1; ++k) {
      P.ssbeg[k] = (int32_t)(base + (k - g0));
      const int32_t v = P.sv[k];
      for (int32_t j = 0; j < row[v + 1] - row[v]; ++j) cdst[slot[row[v] + j]] = P.ssbeg[k] + 64 * j;
    }
    base += 64 * (int64_t)width;
    if (base >= (int64_t(1) << 31)) return "mesh too large for 32-bit part slots";
  }
  P.nss = base;

  // per tile: local vertex list (interior first), LDS part slots, corner tables
  std::vector<int32_t> loc(nv, -1);
  P.lv.resize(3 * nt);
  P.dst.resize(3 * nt);
  P.vbeg.push_back(0);
  std::vector<int32_t> inner, outer;
  for (int32_t k = 0; k < P.ntiles; ++k) {
    inner.clear();
    outer.clear();
    for (int32_t s = P.tbeg[k]; s < P.tbeg[k + 1]; ++s) {
      const int32_t t = P.order[s];
      for (int i = 0; i < 3; ++i) {
        const int32_t v = tri[3 * t + i];
        if (loc[v] == k) continue;  // already listed for this tile (marked with the tile id)
        loc[v] = k;
        (shared[v] ? outer : inner).push_back(v);
      }
    }
    std::sort(inner.begin(), inner.end());
    std::sort(outer.begin(), outer.end());
    const int32_t lvi = (int32_t)inner.size(), lvn = lvi + (int32_t)outer.size();
    if (lvn > 65535) return "tile has too many vertices";
    P.nvi.push_back(lvi);
    P.lpb.push_back((int32_t)P.lp.size());
    int32_t q = 0;
    for (int32_t l = 0; l < lvi; ++l) {
      const int32_t v = inner[l];
      P.lp.push_back(q);
      for (int32_t j = row[v]; j < row[v + 1]; ++j) cdst[slot[j]] = -1 - q++;
    }
    P.lp.push_back(q);
    for (int32_t v : inner) P.tvl.push_back(v);
    for (int32_t v : outer) P.tvl.push_back(v);
    P.vbeg.push_back((int32_t)P.tvl.size());
    // local index of each listed vertex (reuses loc, now as index + ntiles offset-free map)
    for (int32_t l = 0; l < lvn; ++l) loc[P.tvl[P.vbeg[k] + l]] = -2 - l;
    for (int32_t s = P.tbeg[k]; s < P.tbeg[k + 1]; ++s) {
      const int32_t t = P.order[s];
      for (int i = 0; i < 3; ++i) {
        P.lv[(int64_t)i * nt + s] = (uint16_t)(-2 - loc[tri[3 * t + i]]);
        P.dst[(int64_t)i * nt + s] = cdst[3 * t + i];
      }
    }
    for (int32_t l = 0; l < lvn; ++l) loc[P.tvl[P.vbeg[k] + l]] = -1;
    P.max_lv = std::max(P.max_lv, lvn);
    P.max_lvi = std::max(P.max_lvi, lvi);
    P.max_slots = std::max(P.max_slots, q);
  }
  if ((int64_t)P.tvl.size() >= (int64_t(1) << 31)) return "too many tile vertices";
  return std::string();
}

}  // namespace rd
