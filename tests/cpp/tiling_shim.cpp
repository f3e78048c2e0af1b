// Test shim: exposes the host tile builder (paper_1705_02028_amd/csrc/rd_tiling.h)
// to the CPU tests through a plain C interface.
#include <cstring>
#include <vector>

#include "rd_tiling.h"

extern "C" {

// Builds the plan and copies it into caller-sized arrays (sizes first via
// tiling_sizes). Returns 0 on success, 1 if the builder refused.
static rd::TilePlan g_plan;

int tiling_build(int64_t nv, int64_t nt, const int32_t* tri, const double* x, const double* y, double px, double py,
                 int nmesh, const int64_t* voff, const int64_t* toff, int tt) {
  std::vector<int32_t> row(nv + 1, 0), slot(3 * nt);
  for (int64_t s = 0; s < 3 * nt; ++s) row[tri[s] + 1]++;
  for (int64_t i = 0; i < nv; ++i) row[i + 1] += row[i];
  std::vector<int32_t> fill(row.begin(), row.end() - 1);
  for (int64_t s = 0; s < 3 * nt; ++s) slot[fill[tri[s]]++] = (int32_t)s;
  std::vector<int64_t> vo(voff, voff + nmesh + 1), to(toff, toff + nmesh + 1);
  return rd::build_tile_plan(nv, nt, tri, x, y, px, py, row.data(), slot.data(), vo, to, tt, g_plan).empty() ? 0 : 1;
}

// sizes: ntiles, max_lv, max_lvi, max_slots, len(tvl), len(lp), nsv, nss
void tiling_sizes(int64_t* out) {
  const rd::TilePlan& P = g_plan;
  out[0] = P.ntiles;
  out[1] = P.max_lv;
  out[2] = P.max_lvi;
  out[3] = P.max_slots;
  out[4] = (int64_t)P.tvl.size();
  out[5] = (int64_t)P.lp.size();
  out[6] = (int64_t)P.sv.size();
  out[7] = P.nss;
}

void tiling_arrays(int32_t* order, int32_t* tbeg, int32_t* vbeg, int32_t* nvi, int32_t* lpb, int32_t* lp, int32_t* tvl,
                   uint16_t* lv, int32_t* dst, int32_t* tmesh, int32_t* sv, int32_t* ssbeg) {
  const rd::TilePlan& P = g_plan;
  auto cp = [](auto* out, const auto& v) {
    if (!v.empty()) std::memcpy(out, v.data(), v.size() * sizeof(v[0]));
  };
  cp(order, P.order);
  cp(tbeg, P.tbeg);
  cp(vbeg, P.vbeg);
  cp(nvi, P.nvi);
  cp(lpb, P.lpb);
  cp(lp, P.lp);
  cp(tvl, P.tvl);
  cp(lv, P.lv);
  cp(dst, P.dst);
  cp(tmesh, P.tmesh);
  cp(sv, P.sv);
  cp(ssbeg, P.ssbeg);
}
}
