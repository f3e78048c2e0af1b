// Host run of the device code that forms the per-vertex CFL bounds
// (rd::cfl_vertex_bounds, rd_device.h) on random sliced slot layouts with
// irregular degrees (0 to 13, so some vertices have none and some pass the
// eight ranks loaded up front), in both term precisions and with a partial
// last group of vertices. Each bound must equal, bitwise, 2 V / (the
// vertex's terms summed in ascending rank order), and every array is sized
// exactly as the library sizes it, so that a build with AddressSanitizer
// reports any access outside them. Prints "ok" and exits 0 on success.
#include "rd_device.h"

#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

int main() {
  std::mt19937 gen(1);
  for (int trial = 0; trial < 200; ++trial) {
    const int nv = 1 + (int)(gen() % 300);
    std::vector<int32_t> deg(nv), row(nv + 1, 0);
    for (int v = 0; v < nv; ++v) deg[v] = gen() % 10 == 0 ? 0 : (int)(gen() % 14);
    for (int v = 0; v < nv; ++v) row[v + 1] = row[v] + deg[v];
    // 64-vertex slices, each as deep as its largest degree
    const int nsl = (nv + 63) / 64;
    std::vector<int32_t> sbase(nsl);
    int64_t ns = 0;
    for (int s = 0; s < nsl; ++s) {
      int md = 0;
      for (int v = 64 * s; v < std::min(nv, 64 * s + 64); ++v) md = std::max(md, deg[v]);
      sbase[s] = (int32_t)ns;
      ns += 64 * (int64_t)md;
    }
    const int nt = 1 + (int)(gen() % 500);
    std::vector<int32_t> vtri(std::max<int64_t>(ns, 1), -1);  // padding slots hold -1
    for (int v = 0; v < nv; ++v)
      for (int j = 0; j < deg[v]; ++j) vtri[sbase[v >> 6] + (v & 63) + 64 * j] = (int32_t)(gen() % nt);
    std::vector<float> lamf(nt);
    std::vector<double> lamd(nt), V(nv);
    for (int t = 0; t < nt; ++t) {
      lamf[t] = (float)(gen() % 1000 + 1) / 7.0f;
      lamd[t] = (double)(gen() % 100000 + 1) / 3.0;
    }
    for (int v = 0; v < nv; ++v) V[v] = (double)(gen() % 100 + 1) / 3.0;
    rd::Dev d;
    d.nv = nv;
    d.nt = nt;
    d.ns = ns;
    d.row = row.data();
    d.sbase = sbase.data();
    d.vtri = vtri.data();
    d.V = V.data();
    for (int prec = 0; prec < 2; ++prec) {
      d.lam = prec ? static_cast<void*>(lamd.data()) : static_cast<void*>(lamf.data());
      for (int v0 = 0; v0 < nv; v0 += 4) {
        int64_t vv[4];
        bool in[4];
        for (int u = 0; u < 4; ++u) {
          vv[u] = v0 + u;
          in[u] = vv[u] < nv;
        }
        double out[4];
        if (prec) rd::cfl_vertex_bounds<double, 4>(vv, in, v0, d, out);
        else rd::cfl_vertex_bounds<float, 4>(vv, in, v0, d, out);
        for (int u = 0; u < 4; ++u) {
          if (!in[u]) continue;
          double acc = 0.0;
          for (int j = 0; j < deg[vv[u]]; ++j) {
            const int32_t t = vtri[sbase[vv[u] >> 6] + (vv[u] & 63) + 64 * j];
            acc += prec ? lamd[t] : (double)lamf[t];
          }
          const double want = 2.0 * V[vv[u]] / acc;
          if (!(want == out[u] || (std::isinf(want) && std::isinf(out[u])))) {
            std::printf("mismatch: trial %d vertex %lld degree %d: %.17g vs %.17g\n", trial, (long long)vv[u],
                        deg[vv[u]], want, out[u]);
            return 1;
          }
        }
      }
    }
  }
  std::printf("ok\n");
  return 0;
}
