// Host side of the librd C ABI: mesh validation and precompute, device
// buffers, and the order of kernel launches for one step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <type_traits>
#include <vector>

#include "rd.h"
#include "rd3_launch.h"
#include "rd_delaunay.h"
#include "rd_launch.h"
#include "rd_noalloc.h"
#include "rd_tiling.h"

#define RD_API extern "C" __attribute__((visibility("default")))

namespace {

thread_local std::string g_last_error;

rd_status fail(rd_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

#define HIPCHK(call)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return fail(RD_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));          \
  } while (0)

double unwrap_h(double d, double period) {
  if (period > 0.0) {
    if (d > 0.5 * period) d -= period;
    else if (d < -0.5 * period) d += period;
  }
  return d;
}

// Largest vertex degree (triangles per vertex) a mesh may have: the rank of
// a triangle among the triangles of each of its corner vertices is packed in
// 10 bits.
constexpr int32_t kMaxDegree = 1023;

// Geometry the device does not recompute: vertex volumes (median dual).
// Also the checks of rd_mesh_validate.
struct HostGeom {
  std::vector<double> V;
};

rd_status check_desc(const rd_mesh_desc* d, HostGeom* out) {
  if (!d) return fail(RD_EINVAL, "null mesh description");
  if (d->n_vertices <= 0 || d->n_triangles <= 0) return fail(RD_EINVAL, "empty mesh");
  if (d->n_vertices >= (int64_t(1) << 31) || 3 * d->n_triangles >= (int64_t(1) << 31))
    return fail(RD_EINVAL, "mesh too large for 32-bit indices");
  if (!d->x || !d->y || !d->tri) return fail(RD_EINVAL, "null coordinate or triangle array");
  if (!(d->gamma > 1.0)) return fail(RD_EINVAL, "gamma must exceed 1");
  if (d->period_x < 0.0 || d->period_y < 0.0) return fail(RD_EINVAL, "negative period");
  if (d->n_wall_edges < 0 || (d->n_wall_edges > 0 && !d->wall_edges))
    return fail(RD_EINVAL, "bad wall edge list");
  const int64_t nv = d->n_vertices, nt = d->n_triangles;
  std::vector<double> V(nv, 0.0), area(nt, 0.0);
  for (int64_t t = 0; t < nt; ++t) {
    int32_t v[3] = {d->tri[3 * t], d->tri[3 * t + 1], d->tri[3 * t + 2]};
    for (int k = 0; k < 3; ++k)
      if (v[k] < 0 || v[k] >= nv)
        return fail(RD_EINVAL, "triangle " + std::to_string(t) + " has a vertex index out of range");
    double px[3] = {0.0, 0.0, 0.0}, py[3] = {0.0, 0.0, 0.0};
    for (int k = 1; k < 3; ++k) {
      px[k] = unwrap_h(d->x[v[k]] - d->x[v[0]], d->period_x);
      py[k] = unwrap_h(d->y[v[k]] - d->y[v[0]], d->period_y);
    }
    const double a = 0.5 * (px[1] * py[2] - py[1] * px[2]);
    if (!(a > 0.0))
      return fail(RD_EINVAL, "triangle " + std::to_string(t) + " is not counter-clockwise with positive area");
    area[t] = a;
  }
  std::vector<int32_t> deg(nv, 0);
  for (int64_t t = 0; t < nt; ++t)
    for (int k = 0; k < 3; ++k) {
      V[d->tri[3 * t + k]] += area[t] / 3.0;
      ++deg[d->tri[3 * t + k]];
    }
  for (int64_t i = 0; i < nv; ++i) {
    if (!(V[i] > 0.0)) return fail(RD_EINVAL, "vertex " + std::to_string(i) + " belongs to no triangle");
    // a triangle's rank among the triangles of each corner vertex is packed in 10 bits
    if (deg[i] > kMaxDegree)
      return fail(RD_EINVAL, "vertex " + std::to_string(i) + " belongs to " + std::to_string(deg[i]) +
                                 " triangles; at most " + std::to_string(kMaxDegree) + " are supported");
  }
  for (int64_t e = 0; e < d->n_wall_edges; ++e) {
    const int32_t a = d->wall_edges[2 * e], b = d->wall_edges[2 * e + 1];
    if (a < 0 || a >= nv || b < 0 || b >= nv || a == b)
      return fail(RD_EINVAL, "wall edge " + std::to_string(e) + " is invalid");
  }
  if (out) out->V.swap(V);
  return RD_OK;
}

}  // namespace

struct rd_mesh {
  rd::Dev d;
  hipStream_t stream = nullptr;
  int device = 0;
  int ncu = 0;      // compute units of the device
  int lds_max = 0;  // bytes of LDS one workgroup may use on the device
  // host copies, kept for batches
  std::vector<double> x, y, V;
  std::vector<int32_t> tri, wall, row, slot, bc, wv, wptr;
  std::vector<uint8_t> ghost;
  std::vector<rd::WallEnt> went;
  double px = 0.0, py = 0.0, gamma = 1.4;
  double Ldom = 0.0;  // domain size of the Bx sensor
  // device buffers
  std::vector<void*> allocs;
  rd::CflPlan cfl;
  void* C[2] = {nullptr, nullptr};
  void* keepN[2] = {nullptr, nullptr};
  void* keepT[2] = {nullptr, nullptr};
  void* dW[2] = {nullptr, nullptr};
  double* scratch = nullptr;  // [4 * max(nv, nt)]
  int zprec = -1;             // precision the parameter vectors are valid for
  // adjoint buffers, allocated on first use
  rd::AdjDev adj;
  rd::D4* adjW = nullptr;     // W^n of the step being reversed
  double* adjSig = nullptr;   // [nv] signal speeds of the recomputation (the mesh's stay with its state)
  double* adjIn = nullptr;    // [4 nv] host staging: W^n in, then dL/dW^n out
  double* adjOut = nullptr;   // [4 nv] host staging: dL/dW^{n+1} in
  hipEvent_t events[RD_NKERNELS + 1] = {};
  // tiled form
  int tile = 0;                     // triangles per tile, 0: two-pass form
  rd::Tiles tiles;
  int64_t tile_info[4] = {0, 0, 0, 0};
  std::vector<void*> tile_allocs;
  std::vector<int64_t> voff, toff;  // vertex / triangle ranges of the meshes laid end to end
};

namespace {

template <class T>
rd_status dalloc_in(std::vector<void*>& list, T** p, size_t n) {
  void* q = nullptr;
  if (n == 0) n = 1;
  hipError_t e = hipMalloc(&q, n * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(RD_ENOMEM, "hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed");
  }
  list.push_back(q);
  *p = static_cast<T*>(q);
  return RD_OK;
}

template <class T>
rd_status dalloc(rd_mesh* m, T** p, size_t n) {
  return dalloc_in(m->allocs, p, n);
}

template <class T>
rd_status upload_in(std::vector<void*>& list, T** p, const std::vector<T>& h) {
  rd_status st = dalloc_in(list, p, h.size());
  if (st != RD_OK) return st;
  if (!h.empty()) HIPCHK(hipMemcpy(*p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return RD_OK;
}

template <class T>
rd_status upload(rd_mesh* m, T** p, const std::vector<T>& h) {
  return upload_in(m->allocs, p, h);
}

void free_list(std::vector<void*>& list) {
  for (void* p : list) (void)hipFree(p);
  list.clear();
}

void free_all(rd_mesh* m) {
  free_list(m->tile_allocs);
  free_list(m->allocs);
}

// Buffers of one arithmetic precision, allocated on first use.
rd_status ensure_prec(rd_mesh* m, int fp32) {
  if (m->C[fp32]) return RD_OK;
  const size_t q = fp32 ? sizeof(rd::F4) : sizeof(rd::D4);
  const int64_t nt = m->d.nt, nv = m->d.nv;
  char* p = nullptr;
  rd_status st;
  if ((st = dalloc(m, &p, q * m->d.ns)) != RD_OK) return st;
  m->C[fp32] = p;
  if ((st = dalloc(m, &p, q * 2 * nt)) != RD_OK) return st;
  m->keepN[fp32] = p;
  if ((st = dalloc(m, &p, q * nt)) != RD_OK) return st;
  m->keepT[fp32] = p;
  if ((st = dalloc(m, &p, q * nv)) != RD_OK) return st;
  m->dW[fp32] = p;
  if (fp32 && !m->d.Zf) {
    rd::F4* z = nullptr;
    if ((st = dalloc(m, &z, nv)) != RD_OK) return st;
    m->d.Zf = z;
  }
  return RD_OK;
}

rd::Dev dev_for(const rd_mesh* m, int fp32) {
  rd::Dev d = m->d;
  d.C = m->C[fp32];
  d.keepN = m->keepN[fp32];
  d.keepT = m->keepT[fp32];
  d.dW = m->dW[fp32];
  return d;
}

// The parameter vectors must be valid for the arithmetic about to run.
rd_status ensure_z(rd_mesh* m, int fp32) {
  if (m->zprec == fp32) return RD_OK;
  HIPCHK(rd::launch_refresh(dev_for(m, fp32), fp32, m->stream));
  m->zprec = fp32;
  return RD_OK;
}

// One step of Sections 3.2-3.4. With cfl > 0 the time step is computed on
// the device from the state at the start of the step (the stage-1 triangle
// pass writes l_max lambda_max per corner, two small passes reduce it);
// otherwise it is already in d.dt. With `ev` (RD_NKERNELS + 1 events) an
// event is recorded before every kernel slot and after the last.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

rd_status run_step_tiled(rd_mesh* m, int scheme, int time, int fp32, double cfl, hipEvent_t* ev);

rd_status run_step(rd_mesh* m, int scheme, int time, int fp32, double cfl, hipEvent_t* ev = nullptr) {
  if (m->tile > 0) return run_step_tiled(m, scheme, time, fp32, cfl, ev);
  const rd::Dev d = dev_for(m, fp32);
  hipStream_t s = m->stream;
  auto mark = [&](int k) -> hipError_t { return ev ? hipEventRecord(ev[k], s) : hipSuccess; };
  const bool with_cfl = cfl > 0.0, bx = scheme == RD_BX;
  HIPCHK(mark(RD_K_WALL1));
  HIPCHK(rd::launch_wall(d, false, s));
  HIPCHK(mark(RD_K_TRI1));
  if (bx) HIPCHK(rd::launch_vrange(d, m->cfl, 0, s));
  HIPCHK(rd::launch_tri(d, fp32, scheme, 1, time == RD_RK2, with_cfl, s));
  HIPCHK(mark(RD_K_SHARED1));
  HIPCHK(mark(RD_K_CFL));
  if (with_cfl) {
    HIPCHK(rd::launch_cfl_part(d, m->cfl, cfl, 1, s, fp32));
    HIPCHK(rd::launch_cfl_part(d, m->cfl, cfl, 2, s));
  }
  HIPCHK(mark(RD_K_GATHER1));
  HIPCHK(rd::launch_gather(d, fp32, time == RD_RK2 ? rd::G_STAGE1 : rd::G_EULER, nullptr, s));
  HIPCHK(mark(RD_K_WALL2));
  if (time == RD_RK2) {
    HIPCHK(rd::launch_wall(d, true, s));
    HIPCHK(mark(RD_K_TRI2));
    if (bx) HIPCHK(rd::launch_vrange(d, m->cfl, 1, s));
    HIPCHK(rd::launch_tri(d, fp32, scheme, 2, false, false, s));
    HIPCHK(mark(RD_K_GATHER2));
    HIPCHK(rd::launch_gather(d, fp32, rd::G_STAGE2, nullptr, s));
  } else {
    HIPCHK(mark(RD_K_TRI2));
    HIPCHK(mark(RD_K_GATHER2));
  }
  HIPCHK(mark(RD_NKERNELS));
  m->zprec = fp32;
  return RD_OK;
}

// The tiled form of the same step: the tile pass finishes interior vertices
// (stage 1: their residual R1 and CFL bound; stage 2: their new state), the
// shared pass the rest. Stage 1 stores R1 only; W* is rebuilt from it where
// needed, after dt is known.
rd_status run_step_tiled(rd_mesh* m, int scheme, int time, int fp32, double cfl, hipEvent_t* ev) {
  const rd::Dev d = dev_for(m, fp32);
  const rd::Tiles& tl = m->tiles;
  hipStream_t s = m->stream;
  auto mark = [&](int k) -> hipError_t { return ev ? hipEventRecord(ev[k], s) : hipSuccess; };
  const bool with_cfl = cfl > 0.0, rk2 = time == RD_RK2, bx = scheme == RD_BX;
  HIPCHK(mark(RD_K_WALL1));
  HIPCHK(rd::launch_wall(d, false, s));
  HIPCHK(mark(RD_K_TRI1));
  if (bx) HIPCHK(rd::launch_vrange(d, m->cfl, 0, s));
  HIPCHK(rd::launch_tile(d, tl, fp32, scheme, 1, rk2, with_cfl, s));
  HIPCHK(mark(RD_K_SHARED1));
  HIPCHK(rd::launch_shared(d, tl, fp32, 1, with_cfl, s));
  HIPCHK(mark(RD_K_CFL));
  if (with_cfl) {
    HIPCHK(rd::launch_cfl_part(d, m->cfl, cfl, 3, s));
    HIPCHK(rd::launch_cfl_part(d, m->cfl, cfl, 2, s));
  }
  HIPCHK(mark(RD_K_GATHER1));
  if (!rk2) HIPCHK(rd::launch_euler_apply(d, fp32, s));
  HIPCHK(mark(RD_K_WALL2));
  if (rk2) HIPCHK(rd::launch_wall(d, true, s, true));
  HIPCHK(mark(RD_K_TRI2));
  if (rk2 && bx) HIPCHK(rd::launch_vrange(d, m->cfl, 2, s));
  if (rk2) HIPCHK(rd::launch_tile(d, tl, fp32, scheme, 2, false, false, s));
  HIPCHK(mark(RD_K_GATHER2));
  if (rk2) HIPCHK(rd::launch_shared(d, tl, fp32, 2, false, s));
  HIPCHK(mark(RD_NKERNELS));
  m->zprec = fp32;
  return RD_OK;
}

// Builds (or drops, tt = 0) the tiles of a mesh.
rd_status set_tile(rd_mesh* m, int tt) {
  if (tt == m->tile) return RD_OK;
  if (tt != 0 && (tt < 32 || tt > 1024)) return fail(RD_EINVAL, "tile size must be 0 or in [32, 1024]");
  DeviceGuard g(m->device);
  HIPCHK(hipStreamSynchronize(m->stream));
  if (tt == 0) {
    free_list(m->tile_allocs);
    m->tiles = rd::Tiles();
    m->tile = 0;
    for (int64_t& x : m->tile_info) x = 0;
    return RD_OK;
  }
  const rd::Dev& d = m->d;
  rd::TilePlan P;
  const std::string why = rd::build_tile_plan(d.nv, d.nt, m->tri.data(), m->x.data(), m->y.data(), m->px, m->py,
                                              m->row.data(), m->slot.data(), m->voff, m->toff, tt, P);
  if (!why.empty()) return fail(RD_EINVAL, why);
  rd::Tiles tl;
  tl.ntiles = P.ntiles;
  tl.tt = P.tt;
  tl.max_lv = P.max_lv;
  tl.max_lvi = P.max_lvi;
  tl.max_slots = P.max_slots;
  tl.nsv = (int64_t)P.sv.size();
  tl.nss = P.nss;
  const size_t need = std::max(rd::tile_lds_bytes(tl, 0, 1, true), rd::tile_lds_bytes(tl, 0, 2, false));
  if (need > (size_t)m->lds_max)
    return fail(RD_EUNSUPPORTED, "tiles of " + std::to_string(tt) + " triangles need " + std::to_string(need) +
                                     " bytes of LDS");
  std::vector<void*> list;
  int32_t *tbeg, *vbeg, *nvi, *lpb, *lp, *tvl, *dst, *tm, *sv, *ssbeg;
  uint16_t* lv;
  rd::D4* cs;
  double* lams;
  rd_status st;
  if ((st = upload_in(list, &tbeg, P.tbeg)) || (st = upload_in(list, &vbeg, P.vbeg)) ||
      (st = upload_in(list, &nvi, P.nvi)) || (st = upload_in(list, &lpb, P.lpb)) ||
      (st = upload_in(list, &lp, P.lp)) || (st = upload_in(list, &tvl, P.tvl)) ||
      (st = upload_in(list, &lv, P.lv)) || (st = upload_in(list, &dst, P.dst)) ||
      (st = upload_in(list, &tm, P.tmesh)) || (st = upload_in(list, &sv, P.sv)) ||
      (st = upload_in(list, &ssbeg, P.ssbeg)) || (st = dalloc_in(list, &cs, (size_t)P.nss)) ||
      (st = dalloc_in(list, &lams, (size_t)P.nss))) {
    free_list(list);
    return st;
  }
  if (!m->d.R1) {
    rd::D4* r1;
    double* cv;
    if ((st = dalloc(m, &r1, d.nv)) || (st = dalloc(m, &cv, d.nv))) {
      free_list(list);
      return st;
    }
    m->d.R1 = r1;
    m->d.cflv = cv;
  }
  tl.tbeg = tbeg;
  tl.vbeg = vbeg;
  tl.nvi = nvi;
  tl.lpb = lpb;
  tl.lp = lp;
  tl.tvl = tvl;
  tl.lv = lv;
  tl.dst = dst;
  tl.tmesh = m->voff.size() > 2 ? tm : nullptr;
  tl.sv = sv;
  tl.ssbeg = ssbeg;
  tl.Cs = cs;
  tl.lams = lams;
  free_list(m->tile_allocs);
  m->tile_allocs.swap(list);
  m->tiles = tl;
  m->tile = tt;
  int64_t nsc = 0;
  for (int32_t v : P.sv) nsc += m->row[v + 1] - m->row[v];
  m->tile_info[0] = P.ntiles;
  m->tile_info[1] = (int64_t)P.tvl.size();
  m->tile_info[2] = (int64_t)P.sv.size();
  m->tile_info[3] = nsc;
  return RD_OK;
}

rd_status check_step_args(int scheme, int time, int precision) {
  if (scheme < RD_N || scheme > RD_BX) return fail(RD_EINVAL, "unknown scheme");
  if (time != RD_EULER1 && time != RD_RK2) return fail(RD_EINVAL, "unknown time integration");
  if (precision != RD_FP64 && precision != RD_FP32_ACC64) return fail(RD_EINVAL, "unknown precision");
  return RD_OK;
}

bool physical(const double* W, int64_t nv, int64_t i, double gamma) {
  const double rho = W[i], mx = W[nv + i], my = W[2 * nv + i], e = W[3 * nv + i];
  if (!std::isfinite(rho) || !std::isfinite(mx) || !std::isfinite(my) || !std::isfinite(e)) return false;
  if (!(rho > 0.0)) return false;
  const double p = (gamma - 1.0) * (e - 0.5 * (mx * mx + my * my) / rho);
  return p > 0.0;
}

}  // namespace

RD_API rd_status rd_mesh_validate(const rd_mesh_desc* desc) { return check_desc(desc, nullptr); }

RD_API rd_status rd_mesh_create(const rd_mesh_desc* desc, void* stream, rd_mesh** out) {
  if (!out) return fail(RD_EINVAL, "null output pointer");
  *out = nullptr;
  HostGeom geo;
  rd_status st = check_desc(desc, &geo);
  if (st != RD_OK) return st;
  rd_mesh* m = new rd_mesh();
  m->stream = static_cast<hipStream_t>(stream);
  if (hipGetDevice(&m->device) != hipSuccess ||
      hipDeviceGetAttribute(&m->ncu, hipDeviceAttributeMultiprocessorCount, m->device) != hipSuccess ||
      hipDeviceGetAttribute(&m->lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, m->device) != hipSuccess ||
      m->ncu <= 0 || m->lds_max <= 0) {
    delete m;
    return fail(RD_EDEVICE, "no HIP device");
  }
  const int64_t nv = desc->n_vertices, nt = desc->n_triangles;
  m->x.assign(desc->x, desc->x + nv);
  m->y.assign(desc->y, desc->y + nv);
  m->tri.assign(desc->tri, desc->tri + 3 * nt);
  m->ghost.assign(nv, 0);
  if (desc->ghost)
    for (int64_t i = 0; i < nv; ++i) m->ghost[i] = desc->ghost[i] ? 1 : 0;
  if (desc->n_wall_edges > 0) m->wall.assign(desc->wall_edges, desc->wall_edges + 2 * desc->n_wall_edges);
  m->px = desc->period_x;
  m->py = desc->period_y;
  m->gamma = desc->gamma;
  m->V.swap(geo.V);
  m->voff = {0, nv};
  m->toff = {0, nt};

  // vertex -> (triangle, corner) CSR, ascending triangle order in every row
  m->row.assign(nv + 1, 0);
  for (int64_t s = 0; s < 3 * nt; ++s) m->row[m->tri[s] + 1]++;
  for (int64_t i = 0; i < nv; ++i) m->row[i + 1] += m->row[i];
  m->slot.assign(3 * nt, 0);
  {
    std::vector<int32_t> fill(m->row.begin(), m->row.end() - 1);
    for (int64_t s = 0; s < 3 * nt; ++s) m->slot[fill[m->tri[s]]++] = (int32_t)s;
  }
  // boundary kinds and wall incidences (ascending edge id per vertex)
  bool has_bc = false;
  for (int64_t i = 0; i < nv; ++i) has_bc |= m->ghost[i] != 0;
  has_bc |= !m->wall.empty();
  if (has_bc) {
    m->bc.assign(nv, -1);
    std::vector<std::vector<rd::WallEnt>> per(nv);
    const int64_t nw = (int64_t)m->wall.size() / 2;
    for (int64_t e = 0; e < nw; ++e) {
      const int32_t a = m->wall[2 * e], b = m->wall[2 * e + 1];
      const double dx = unwrap_h(m->x[b] - m->x[a], m->px), dy = unwrap_h(m->y[b] - m->y[a], m->py);
      const double len = std::sqrt(dx * dx + dy * dy);
      rd::WallEnt ea{b, 0, len / 2.0, dy / len, -dx / len};
      rd::WallEnt eb{a, 1, len / 2.0, dy / len, -dx / len};
      per[a].push_back(ea);
      per[b].push_back(eb);
    }
    m->wptr.push_back(0);
    for (int64_t i = 0; i < nv; ++i) {
      int32_t b = -1;
      if (!per[i].empty()) {
        b = (int32_t)m->wv.size();
        m->wv.push_back((int32_t)i);
        for (const auto& e : per[i]) m->went.push_back(e);
        m->wptr.push_back((int32_t)m->went.size());
      }
      if (m->ghost[i]) m->bc[i] = b >= 0 ? -3 - b : -2;
      else m->bc[i] = b;
    }
  }

  rd::Dev& d = m->d;
  d.nv = nv;
  d.nt = nt;
  d.nwv = (int32_t)m->wv.size();
  d.gamma = m->gamma;
  d.igamma = 1.0 / m->gamma;
  d.px = m->px;
  d.py = m->py;
  d.hpx = m->px > 0.0 ? 0.5 * m->px : HUGE_VAL;
  d.hpy = m->py > 0.0 ? 0.5 * m->py : HUGE_VAL;
  {
    DeviceGuard g(m->device);
    std::vector<double2> xy(nv);
    for (int64_t i = 0; i < nv; ++i) xy[i] = make_double2(m->x[i], m->y[i]);
    std::vector<int32_t> tv(3 * nt);
    std::vector<uint32_t> rk(nt, 0u);
    for (int64_t t = 0; t < nt; ++t)
      for (int k = 0; k < 3; ++k) tv[k * nt + t] = m->tri[3 * t + k];
    // sliced part layout: 64-vertex slices, each as wide as its largest
    // degree; the j-th part of vertex v sits at sbase[v / 64] + v % 64 + 64 j
    const int64_t nsl = (nv + 63) / 64;
    std::vector<int32_t> sbase(nsl);
    int64_t base = 0;
    int32_t maxdeg = 0;
    for (int64_t g0 = 0; g0 < nv; g0 += 64) {
      const int64_t g1 = std::min<int64_t>(g0 + 64, nv);
      int32_t width = 0;
      for (int64_t v = g0; v < g1; ++v) width = std::max(width, m->row[v + 1] - m->row[v]);
      sbase[g0 / 64] = (int32_t)std::min<int64_t>(base, INT32_MAX);
      base += 64 * (int64_t)width;
      maxdeg = std::max(maxdeg, width);
    }
    if (base >= (int64_t(1) << 31)) {
      free_all(m);
      delete m;
      return fail(RD_EINVAL, "mesh too large for 32-bit part slots");
    }
    if (maxdeg > kMaxDegree) {  // rd_mesh_validate's check has run; kept as a guard
      free_all(m);
      delete m;
      return fail(RD_EINVAL, "a vertex belongs to " + std::to_string(maxdeg) + " triangles; at most " +
                                 std::to_string(kMaxDegree) + " are supported");
    }
    d.ns = base;
    // rank of each triangle among the triangles of each of its corner vertices
    // (10 bits per corner), and the triangle of every part slot
    std::vector<int32_t> vtri(std::max<int64_t>(base, 1), -1);
    for (int64_t v = 0; v < nv; ++v)
      for (int32_t j = 0; j < m->row[v + 1] - m->row[v]; ++j) {
        const int32_t cs = m->slot[m->row[v] + j];  // corner 3 t + k is the j-th part of v
        rk[cs / 3] |= (uint32_t)j << (10 * (cs % 3));
        vtri[sbase[v / 64] + v % 64 + 64 * (int64_t)j] = cs / 3;
      }
    double2* pxy;
    double* pV;
    int32_t *prow, *ptv, *psbase, *pvtri;
    uint32_t* prk;
    if ((st = upload(m, &pxy, xy)) || (st = upload(m, &pV, m->V)) || (st = upload(m, &prow, m->row)) ||
        (st = upload(m, &ptv, tv)) || (st = upload(m, &prk, rk)) || (st = upload(m, &psbase, sbase)) ||
        (st = upload(m, &pvtri, vtri))) {
      free_all(m);
      delete m;
      return st;
    }
    d.xy = pxy;
    d.V = pV;
    d.row = prow;
    d.tv = ptv;
    d.rk = prk;
    d.sbase = psbase;
    d.vtri = pvtri;
    if (has_bc) {
      int32_t *pbc, *pwv, *pwptr;
      rd::WallEnt* pwent;
      if ((st = upload(m, &pbc, m->bc)) || (st = upload(m, &pwv, m->wv)) || (st = upload(m, &pwptr, m->wptr)) ||
          (st = upload(m, &pwent, m->went))) {
        free_all(m);
        delete m;
        return st;
      }
      d.bc = pbc;
      d.wv = pwv;
      d.wptr = pwptr;
      d.went = pwent;
      rd::D4 *wcn, *wcs;
      if ((st = dalloc(m, &wcn, d.nwv)) || (st = dalloc(m, &wcs, d.nwv))) {
        free_all(m);
        delete m;
        return st;
      }
      d.WCn = wcn;
      d.WCs = wcs;
    }
    rd::D4 *W, *Ws, *Z;
    double *sig, *lam, *dt, *scratch;
    int* flag;
    if ((st = dalloc(m, &W, nv)) || (st = dalloc(m, &Ws, nv)) || (st = dalloc(m, &Z, nv)) ||
        (st = dalloc(m, &sig, nv)) || (st = dalloc(m, &lam, nt)) || (st = dalloc(m, &dt, 1)) ||
        (st = dalloc(m, &flag, 1)) || (st = dalloc(m, &scratch, 4 * std::max(nv, nt)))) {
      free_all(m);
      delete m;
      return st;
    }
    d.W = W;
    d.Ws = Ws;
    d.Z = Z;
    d.sig = sig;
    d.lam = lam;
    d.dt = dt;
    d.flag = flag;
    m->scratch = scratch;
    // CFL reduction plan: vertex blocks of kBlock, one segment
    const int32_t nb = (int32_t)((nv + rd::kCflSpan - 1) / rd::kCflSpan);
    std::vector<int32_t> v0(nb), v1(nb), b0 = {0, nb};
    for (int32_t b = 0; b < nb; ++b) {
      v0[b] = b * rd::kCflSpan;
      v1[b] = (int32_t)std::min<int64_t>(nv, (int64_t)(b + 1) * rd::kCflSpan);
    }
    int32_t *pv0, *pv1, *pb0;
    double *part, *vpart, *vr;
    // domain size L of the Bx sensor: the period on a periodic axis, else the coordinate extent
    {
      const auto xr = std::minmax_element(m->x.begin(), m->x.end());
      const auto yr = std::minmax_element(m->y.begin(), m->y.end());
      const double lx = m->px > 0.0 ? m->px : *xr.second - *xr.first;
      const double ly = m->py > 0.0 ? m->py : *yr.second - *yr.first;
      m->Ldom = std::max(lx, ly);
    }
    const std::vector<double> vr0 = {0.0, 0.0, m->Ldom};
    if ((st = upload(m, &pv0, v0)) || (st = upload(m, &pv1, v1)) || (st = upload(m, &pb0, b0)) ||
        (st = dalloc(m, &part, nb)) || (st = dalloc(m, &vpart, 2 * nb)) || (st = upload(m, &vr, vr0))) {
      free_all(m);
      delete m;
      return st;
    }
    d.vr = vr;
    m->cfl.vpart = vpart;
    m->cfl.nblocks = nb;
    m->cfl.nmesh = 1;
    m->cfl.blk_v0 = pv0;
    m->cfl.blk_v1 = pv1;
    m->cfl.mesh_b0 = pb0;
    m->cfl.part = part;
    if ((st = ensure_prec(m, 0)) != RD_OK) {
      free_all(m);
      delete m;
      return st;
    }
    hipError_t e = hipMemset(W, 0, sizeof(rd::D4) * nv);
    if (e == hipSuccess) e = hipMemset(flag, 0, sizeof(int));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
      free_all(m);
      delete m;
      return fail(RD_EDEVICE, std::string("initialising buffers: ") + hipGetErrorString(e));
    }
  }
  *out = m;
  return RD_OK;
}

RD_API rd_status rd_mesh_destroy(rd_mesh* m) {
  if (!m) return RD_OK;
  DeviceGuard g(m->device);
  (void)hipStreamSynchronize(m->stream);
  for (hipEvent_t e : m->events)
    if (e) (void)hipEventDestroy(e);
  free_all(m);
  delete m;
  return RD_OK;
}

RD_API rd_status rd_mesh_info(const rd_mesh* m, int64_t* nv, int64_t* nt) {
  if (!m) return fail(RD_EINVAL, "null mesh");
  if (nv) *nv = m->d.nv;
  if (nt) *nt = m->d.nt;
  return RD_OK;
}

RD_API rd_status rd_set_stream(rd_mesh* m, void* stream) {
  if (!m) return fail(RD_EINVAL, "null mesh");
  m->stream = static_cast<hipStream_t>(stream);
  return RD_OK;
}

RD_API rd_status rd_set_state(rd_mesh* m, const double* W, int on_device) {
  if (!m || !W) return fail(RD_EINVAL, "null argument");
  DeviceGuard g(m->device);
  const int64_t nv = m->d.nv;
  const double* src = W;
  if (!on_device) {
    for (int64_t i = 0; i < nv; ++i)
      if (!physical(W, nv, i, m->gamma))
        return fail(RD_ENONPHYS, "vertex " + std::to_string(i) + " has rho <= 0, p <= 0 or a non-finite value");
    HIPCHK(hipMemcpyAsync(m->scratch, W, sizeof(double) * 4 * nv, hipMemcpyHostToDevice, m->stream));
    src = m->scratch;
  }
  rd::Dev d = dev_for(m, 0);
  HIPCHK(rd::launch_set_int(d.flag, 0, m->stream));
  HIPCHK(rd::launch_set_state(d, src, 0, m->stream));
  m->zprec = 0;
  if (!on_device) HIPCHK(hipStreamSynchronize(m->stream));
  return RD_OK;
}

RD_API rd_status rd_get_state(rd_mesh* m, double* W, int on_device) {
  if (!m || !W) return fail(RD_EINVAL, "null argument");
  DeviceGuard g(m->device);
  const int64_t nv = m->d.nv;
  if (on_device) {
    HIPCHK(rd::launch_get_state(m->d, m->d.W, W, m->stream));
    return RD_OK;
  }
  HIPCHK(rd::launch_get_state(m->d, m->d.W, m->scratch, m->stream));
  HIPCHK(hipMemcpyAsync(W, m->scratch, sizeof(double) * 4 * nv, hipMemcpyDeviceToHost, m->stream));
  int flag = 0;
  HIPCHK(hipMemcpyAsync(&flag, m->d.flag, sizeof(int), hipMemcpyDeviceToHost, m->stream));
  HIPCHK(hipStreamSynchronize(m->stream));
  if (flag) return fail(RD_ENONPHYS, "a non-physical state was produced");
  return RD_OK;
}

RD_API rd_status rd_max_dt(rd_mesh* m, double cfl, double* dt_out) {
  if (!m || !dt_out) return fail(RD_EINVAL, "null argument");
  if (!(cfl > 0.0)) return fail(RD_EINVAL, "cfl must be positive");
  DeviceGuard g(m->device);
  // the signal speeds are valid for the state whenever the parameter vectors
  // are; after a tune, a batch run or an adjoint step they are refreshed first
  if (m->zprec < 0) {
    rd_status st = ensure_z(m, 0);
    if (st != RD_OK) return st;
  }
  HIPCHK(rd::launch_cfl(m->d, m->cfl, cfl, m->stream));
  HIPCHK(hipMemcpyAsync(dt_out, m->d.dt, sizeof(double), hipMemcpyDeviceToHost, m->stream));
  HIPCHK(hipStreamSynchronize(m->stream));
  return RD_OK;
}

RD_API rd_status rd_step(rd_mesh* m, double dt, int scheme, int time, int precision) {
  if (!m) return fail(RD_EINVAL, "null mesh");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(RD_EINVAL, "dt must be positive and finite");
  rd_status st = check_step_args(scheme, time, precision);
  if (st != RD_OK) return st;
  DeviceGuard g(m->device);
  const int fp32 = precision == RD_FP32_ACC64;
  if ((st = ensure_prec(m, fp32)) != RD_OK) return st;
  if ((st = ensure_z(m, fp32)) != RD_OK) return st;
  HIPCHK(rd::launch_set_scalar(m->d.dt, dt, m->stream));
  return run_step(m, scheme, time, fp32, 0.0);
}

RD_API rd_status rd_step_cfl(rd_mesh* m, int n_steps, double cfl, int scheme, int time, int precision) {
  if (!m) return fail(RD_EINVAL, "null mesh");
  if (n_steps < 0) return fail(RD_EINVAL, "negative step count");
  if (!(cfl > 0.0)) return fail(RD_EINVAL, "cfl must be positive");
  rd_status st = check_step_args(scheme, time, precision);
  if (st != RD_OK) return st;
  DeviceGuard g(m->device);
  const int fp32 = precision == RD_FP32_ACC64;
  if ((st = ensure_prec(m, fp32)) != RD_OK) return st;
  if ((st = ensure_z(m, fp32)) != RD_OK) return st;
  for (int n = 0; n < n_steps; ++n)
    if ((st = run_step(m, scheme, time, fp32, cfl)) != RD_OK) return st;
  return RD_OK;
}

RD_API rd_status rd_step_timed(rd_mesh* m, double cfl, int scheme, int time, int precision, double* ms) {
  if (!m || !ms) return fail(RD_EINVAL, "null argument");
  if (!(cfl > 0.0)) return fail(RD_EINVAL, "cfl must be positive");
  rd_status st = check_step_args(scheme, time, precision);
  if (st != RD_OK) return st;
  DeviceGuard g(m->device);
  const int fp32 = precision == RD_FP32_ACC64;
  if ((st = ensure_prec(m, fp32)) != RD_OK) return st;
  if ((st = ensure_z(m, fp32)) != RD_OK) return st;
  if (!m->events[0])
    for (int k = 0; k <= RD_NKERNELS; ++k) HIPCHK(hipEventCreate(&m->events[k]));
  hipEvent_t* ev = m->events;
  if ((st = run_step(m, scheme, time, fp32, cfl, ev)) != RD_OK) return st;
  HIPCHK(hipEventSynchronize(ev[RD_NKERNELS]));
  for (int k = 0; k < RD_NKERNELS; ++k) {
    float t = 0.0f;
    HIPCHK(hipEventElapsedTime(&t, ev[k], ev[k + 1]));
    ms[k] = t;
  }
  return RD_OK;
}

RD_API rd_status rd_mesh_set_tile(rd_mesh* m, int tile_triangles) {
  if (!m) return fail(RD_EINVAL, "null mesh");
  return set_tile(m, tile_triangles);
}

RD_API rd_status rd_mesh_get_tile(const rd_mesh* m, int* tile_triangles) {
  if (!m || !tile_triangles) return fail(RD_EINVAL, "null argument");
  *tile_triangles = m->tile;
  return RD_OK;
}

RD_API rd_status rd_mesh_set_lumping(rd_mesh* m, int lumping) {
  if (!m) return fail(RD_EINVAL, "null mesh");
  if (lumping != RD_LUMP_GLOBAL && lumping != RD_LUMP_SELECTIVE) return fail(RD_EINVAL, "unknown lumping");
  m->d.slump = lumping == RD_LUMP_SELECTIVE;
  return RD_OK;
}

RD_API rd_status rd_mesh_get_lumping(const rd_mesh* m, int* lumping) {
  if (!m || !lumping) return fail(RD_EINVAL, "null argument");
  *lumping = m->d.slump ? RD_LUMP_SELECTIVE : RD_LUMP_GLOBAL;
  return RD_OK;
}

RD_API rd_status rd_mesh_tile_info(const rd_mesh* m, int64_t* info) {
  if (!m || !info) return fail(RD_EINVAL, "null argument");
  for (int k = 0; k < 4; ++k) info[k] = m->tile_info[k];
  return RD_OK;
}

namespace {

const int kTuneDefault[] = {0, 64, 128, 256, 512};
// A later candidate replaces the one kept so far only when it is faster by
// more than this fraction (the run-to-run spread of one timing is about 1-2%),
// so the tuner does not switch forms on noise.
constexpr float kTuneMargin = 0.02f;

rd_status tune_args(double cfl, int scheme, int time, int precision, int n_steps, const int*& cand, int& nc,
                    int* best) {
  if (!best) return fail(RD_EINVAL, "null argument");
  if (!(cfl > 0.0)) return fail(RD_EINVAL, "cfl must be positive");
  if (n_steps < 1) return fail(RD_EINVAL, "n_steps must be at least 1");
  if (!cand) {
    cand = kTuneDefault;
    nc = (int)(sizeof(kTuneDefault) / sizeof(kTuneDefault[0]));
  }
  if (nc < 1) return fail(RD_EINVAL, "no candidates");
  return check_step_args(scheme, time, precision);
}

// Times `body` (enqueued on s) with two events; returns milliseconds.
template <class F>
rd_status time_on(hipStream_t s, F body, float* ms) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(RD_EDEVICE, "hipEventCreate failed");
  }
  rd_status st = RD_OK;
  hipError_t e = hipEventRecord(e0, s);
  if (e == hipSuccess) st = body();
  if (e == hipSuccess && st == RD_OK) e = hipEventRecord(e1, s);
  if (e == hipSuccess && st == RD_OK) e = hipEventSynchronize(e1);
  if (e == hipSuccess && st == RD_OK) e = hipEventElapsedTime(ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != RD_OK) return st;
  if (e != hipSuccess) return fail(RD_EDEVICE, std::string("timing: ") + hipGetErrorString(e));
  return RD_OK;
}

}  // namespace

RD_API rd_status rd_tune(rd_mesh* m, double cfl, int scheme, int time, int precision, int n_steps,
                         const int* candidates, int n_candidates, double* ms_per_step, int* best) {
  if (!m) return fail(RD_EINVAL, "null mesh");
  rd_status st = tune_args(cfl, scheme, time, precision, n_steps, candidates, n_candidates, best);
  if (st != RD_OK) return st;
  DeviceGuard g(m->device);
  const int fp32 = precision == RD_FP32_ACC64;
  if ((st = ensure_prec(m, fp32)) != RD_OK) return st;
  hipStream_t s = m->stream;
  // the state and the flag are saved in the scratch buffer (4 max(nv, nt) doubles)
  rd::D4* saveW = reinterpret_cast<rd::D4*>(m->scratch);
  HIPCHK(rd::launch_copy4(saveW, m->d.W, m->d.nv, s));
  int flag0 = 0;
  HIPCHK(hipMemcpyAsync(&flag0, m->d.flag, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  auto restore = [&]() -> rd_status {
    HIPCHK(rd::launch_copy4(m->d.W, saveW, m->d.nv, s));
    HIPCHK(rd::launch_set_int(m->d.flag, flag0, s));
    m->zprec = -1;
    return RD_OK;
  };
  const int prev = m->tile;
  int pick = -1;
  float pick_ms = 0.0f;
  for (int i = 0; i < n_candidates; ++i) {
    if (ms_per_step) ms_per_step[i] = -1.0;
    st = set_tile(m, candidates[i]);
    if (st == RD_EUNSUPPORTED || st == RD_EINVAL) continue;
    if (st != RD_OK) break;
    if ((st = ensure_z(m, fp32)) != RD_OK || (st = run_step(m, scheme, time, fp32, cfl)) != RD_OK) break;
    float t = 0.0f;
    st = time_on(s, [&]() -> rd_status {
      for (int k = 0; k < n_steps; ++k) {
        rd_status r = run_step(m, scheme, time, fp32, cfl);
        if (r != RD_OK) return r;
      }
      return RD_OK;
    }, &t);
    if (st != RD_OK) break;
    if ((st = restore()) != RD_OK) break;
    if (ms_per_step) ms_per_step[i] = t / n_steps;
    if (pick < 0 || t < pick_ms * (1.0f - kTuneMargin)) {
      pick = candidates[i];
      pick_ms = t;
    }
  }
  if (st == RD_EUNSUPPORTED || st == RD_EINVAL) st = RD_OK;
  rd_status st2 = set_tile(m, pick >= 0 ? pick : prev);
  rd_status st3 = restore();
  HIPCHK(hipStreamSynchronize(s));
  if (st != RD_OK) return st;
  if (st2 != RD_OK) return st2;
  if (st3 != RD_OK) return st3;
  if (pick < 0) return fail(RD_EUNSUPPORTED, "no candidate tile size is usable");
  *best = pick;
  return RD_OK;
}

RD_API rd_status rd_residual(rd_mesh* m, int scheme, double* R, double* phiT, int on_device) {
  if (!m || !R) return fail(RD_EINVAL, "null argument");
  if (scheme < RD_N || scheme > RD_BX) return fail(RD_EINVAL, "unknown scheme");
  DeviceGuard g(m->device);
  rd_status st;
  if ((st = ensure_z(m, 0)) != RD_OK) return st;
  const rd::Dev d = dev_for(m, 0);
  hipStream_t s = m->stream;
  const int64_t nv = d.nv, nt = d.nt;
  HIPCHK(rd::launch_wall(d, false, s));
  if (scheme == RD_BX) HIPCHK(rd::launch_vrange(d, m->cfl, 0, s));
  HIPCHK(rd::launch_tri(d, 0, scheme, 1, true, false, s));
  if (on_device) {
    HIPCHK(rd::launch_gather(d, 0, rd::G_RESIDUAL, R, s));
    if (phiT) HIPCHK(rd::launch_keep_to_soa(d.keepT, phiT, nt, s));
    return RD_OK;
  }
  HIPCHK(rd::launch_gather(d, 0, rd::G_RESIDUAL, m->scratch, s));
  HIPCHK(hipMemcpyAsync(R, m->scratch, sizeof(double) * 4 * nv, hipMemcpyDeviceToHost, s));
  if (phiT) {
    HIPCHK(rd::launch_keep_to_soa(d.keepT, m->scratch, nt, s));
    HIPCHK(hipMemcpyAsync(phiT, m->scratch, sizeof(double) * 4 * nt, hipMemcpyDeviceToHost, s));
  }
  HIPCHK(hipStreamSynchronize(s));
  return RD_OK;
}

namespace {

// Waits for the mesh's stream and reports (then clears) the adjoint's latches:
// a non-physical recomputed step, or a triangle whose solve skipped a column.
rd_status adjoint_status(rd_mesh* m) {
  int flag[2] = {0, 0};
  if (m->adj.flag) HIPCHK(hipMemcpyAsync(flag, m->adj.flag, sizeof(flag), hipMemcpyDeviceToHost, m->stream));
  HIPCHK(hipStreamSynchronize(m->stream));
  if (!flag[0] && !flag[1]) return RD_OK;
  HIPCHK(rd::launch_set_int(m->adj.flag, 0, m->stream));
  HIPCHK(rd::launch_set_int(m->adj.flag + 1, 0, m->stream));
  HIPCHK(hipStreamSynchronize(m->stream));
  if (flag[0]) return fail(RD_ENONPHYS, "the adjoint's input state W_n or its recomputed first stage is non-physical");
  return fail(RD_EUNSUPPORTED,
              "the adjoint met a triangle whose pivoted solve skipped a column (exact stagnation, Section 3.3.1); "
              "the gradient of that branch is not computed");
}

}  // namespace

namespace {

rd_status adjoint_args(rd_mesh* m, double dt, int scheme, int time) {
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(RD_EINVAL, "dt must be positive and finite");
  rd_status st = check_step_args(scheme, time, RD_FP64);
  if (st != RD_OK) return st;
  if (scheme == RD_BX) return fail(RD_EUNSUPPORTED, "the adjoint does not cover the Bx scheme");
  if (m->d.slump && time == RD_RK2)
    return fail(RD_EUNSUPPORTED, "the adjoint does not cover selective lumping");
  return RD_OK;
}

// Enqueues the reverse of one step on the mesh's stream, all pointers on the
// device: the step from W_n is recomputed on the buffers of `a` (W^n copy Wa,
// signal speeds sig, latches a.flag) and the mesh's stage buffers; the mesh's
// own state, signal speeds and latch are not touched.
rd_status adjoint_enqueue(rd_mesh* m, const rd::AdjDev& a, rd::D4* Wa, double* sig, const double* W_n,
                          double dt, int scheme, int time, const double* lam_np1, double* lam_n) {
  hipStream_t s = m->stream;
  rd::Dev d = dev_for(m, 0);
  d.W = Wa;
  d.sig = sig;
  d.flag = a.flag;
  // parameter vectors at W^n go straight to Zn (read by the stage-1 passes and
  // the adjoint); the first-stage vertex pass writes W* and the stage-2
  // reverse records
  rd::Dev dn = d;
  dn.Z = a.Zn;
  rd::AdjDev ad = a;
  ad.lam = rd::LamSoA{lam_np1, m->d.nv};  // read in the caller's layout
  ad.idt = 1.0 / dt;
  ad.waves = rd::kAdjWavesPerCu * m->ncu;
  HIPCHK(rd::launch_set_state(dn, W_n, 0, s));
  HIPCHK(rd::launch_set_scalar(d.dt, dt, s));
  const bool rk2 = time == RD_RK2;
  if (rk2) {
    HIPCHK(rd::launch_wall(dn, false, s));
    HIPCHK(rd::launch_tri(dn, 0, scheme, 1, true, false, s));
    HIPCHK(rd::launch_adj_star(d, ad, s));
  }
  HIPCHK(rd::launch_adjoint(d, ad, scheme, rk2 ? 1 : 0, lam_n, s));
  m->zprec = -1;  // the parameter-vector buffer now holds the recomputation's values
  return RD_OK;
}

}  // namespace

RD_API rd_status rd_adjoint_step(rd_mesh* m, const double* W_n, double dt, int scheme, int time,
                                 const double* lam_np1, double* lam_n, int on_device) {
  if (!m || !W_n || !lam_np1 || !lam_n) return fail(RD_EINVAL, "null argument");
  rd_status st = adjoint_args(m, dt, scheme, time);
  if (st != RD_OK) return st;
  DeviceGuard g(m->device);
  const int64_t nv = m->d.nv, nt = m->d.nt;
  if (!m->adjW) {
    rd::AdjDev& a = m->adj;
    rd::D4 *lamS, *lamN, *Zn, *cZ, *kN, *kT, *Wa;
    rd::ZW* cZW;
    rd::AdjRec2* r2;
    rd::AdjRec1* r1;
    double *in, *out, *sig;
    int* flag;
    if ((st = dalloc(m, &lamS, nv)) || (st = dalloc(m, &lamN, nv)) || (st = dalloc(m, &r2, nv)) ||
        (st = dalloc(m, &r1, nv)) ||
        (st = dalloc(m, &Zn, nv)) || (st = dalloc(m, &cZ, m->d.ns)) || (st = dalloc(m, &cZW, m->d.ns)) ||
        (st = dalloc(m, &kN, 2 * nt)) || (st = dalloc(m, &kT, nt)) || (st = dalloc(m, &Wa, nv)) ||
        (st = dalloc(m, &in, 4 * nv)) || (st = dalloc(m, &out, 4 * nv)) || (st = dalloc(m, &sig, nv)) ||
        (st = dalloc(m, &flag, 2)))
      return st;
    HIPCHK(rd::launch_set_int(flag, 0, m->stream));
    HIPCHK(rd::launch_set_int(flag + 1, 0, m->stream));
    a.flag = flag;
    m->adjSig = sig;
    a.lamS = lamS;
    a.lamN = lamN;
    a.r2 = r2;
    a.r1 = r1;
    a.Zn = Zn;
    a.cZ = cZ;
    a.cZW = cZW;
    a.kN = kN;
    a.kT = kT;
    m->adjW = Wa;
    m->adjIn = in;
    m->adjOut = out;
  }
  hipStream_t s = m->stream;
  const double* src = W_n;
  if (!on_device) {
    HIPCHK(hipMemcpyAsync(m->adjIn, W_n, sizeof(double) * 4 * nv, hipMemcpyHostToDevice, s));
    src = m->adjIn;
  }
  // dL/dW^n is written back to adjIn: its copy of W^n is consumed by the first
  // kernel of the recomputation, which runs before (stream order)
  const double* lsrc = lam_np1;
  if (!on_device) {
    HIPCHK(hipMemcpyAsync(m->adjOut, lam_np1, sizeof(double) * 4 * nv, hipMemcpyHostToDevice, s));
    lsrc = m->adjOut;
  }
  double* out = on_device ? lam_n : m->adjIn;
  if ((st = adjoint_enqueue(m, m->adj, m->adjW, m->adjSig, src, dt, scheme, time, lsrc, out)) != RD_OK) return st;
  if (!on_device) {
    HIPCHK(hipMemcpyAsync(lam_n, m->adjIn, sizeof(double) * 4 * nv, hipMemcpyDeviceToHost, s));
    return adjoint_status(m);
  }
  return RD_OK;
}

RD_API rd_status rd_adjoint_step_noalloc(rd_mesh* m, const double* W_n, double dt, int scheme, int time,
                                         const double* lam_np1, double* lam_n, int* flags) {
  if (!m || !W_n || !lam_np1 || !lam_n || !flags) return fail(RD_EINVAL, "null argument");
  rd_status st = adjoint_args(m, dt, scheme, time);
  if (st != RD_OK) return st;
  const int64_t nv = m->d.nv, nt = m->d.nt, ns = m->d.ns;
  // workspace layout: every buffer starts on a 256-byte boundary
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += (bytes + 255) & ~size_t(255);
    return at;
  };
  const size_t oR2 = take(sizeof(rd::AdjRec2) * nv), oR1 = take(sizeof(rd::AdjRec1) * nv),
               oLamS = take(sizeof(rd::D4) * nv),
               oLamN = take(sizeof(rd::D4) * nv), oZn = take(sizeof(rd::D4) * nv), oWa = take(sizeof(rd::D4) * nv),
               oSig = take(sizeof(double) * nv), oCZ = take(sizeof(rd::D4) * ns), oCZW = take(sizeof(rd::ZW) * ns),
               oKN = take(sizeof(rd::D4) * 2 * nt), oKT = take(sizeof(rd::D4) * nt);
  if (off > rd::kNoallocScratchBytes)
    return fail(RD_EINVAL, "mesh too large for the allocation-free adjoint: it needs " + std::to_string(off) +
                               " bytes of workspace, the fixed workspace holds " +
                               std::to_string(rd::kNoallocScratchBytes));
  DeviceGuard g(m->device);
  void* base = nullptr;
  HIPCHK(rd::noalloc_scratch(&base));
  char* p = static_cast<char*>(base);
  rd::AdjDev a;
  a.r2 = reinterpret_cast<rd::AdjRec2*>(p + oR2);
  a.r1 = reinterpret_cast<rd::AdjRec1*>(p + oR1);
  a.lamS = reinterpret_cast<rd::D4*>(p + oLamS);
  a.lamN = reinterpret_cast<rd::D4*>(p + oLamN);
  a.Zn = reinterpret_cast<rd::D4*>(p + oZn);
  a.cZ = reinterpret_cast<rd::D4*>(p + oCZ);
  a.cZW = reinterpret_cast<rd::ZW*>(p + oCZW);
  a.kN = reinterpret_cast<rd::D4*>(p + oKN);
  a.kT = reinterpret_cast<rd::D4*>(p + oKT);
  a.flag = flags;
  // the latches start cleared on every call (a fill kernel, so the call can be captured)
  HIPCHK(rd::launch_fill_int(flags, 0, 2, m->stream));
  return adjoint_enqueue(m, a, reinterpret_cast<rd::D4*>(p + oWa), reinterpret_cast<double*>(p + oSig), W_n, dt,
                         scheme, time, lam_np1, lam_n);
}

// ------------------------------------------------------------- batches --
//
// A batch lays its meshes end to end as one disjoint mesh (vertex and
// triangle ids offset in order), adds a mesh id per vertex and per triangle so
// every kernel reads its own mesh's time step, and reduces the CFL limit per
// mesh over vertex blocks that never straddle two meshes. n steps are
// captured once into a HIP graph and replayed; the members' states are
// copied in before and out after.

struct rd_batch {
  rd_mesh* flat = nullptr;
  std::vector<rd_mesh*> members;
  std::vector<int64_t> voff, toff;
  hipStream_t stream = nullptr;  // the caller's stream
  hipStream_t own = nullptr;     // the batch's own stream (a null stream cannot be captured)
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  struct Graph {
    int n_steps, scheme, time, fp32, slump;
    double cfl;
    hipGraph_t graph;
    hipGraphExec_t exec;
  };
  std::vector<Graph> graphs;
};

namespace {

void destroy_graphs(rd_batch* b) {
  for (auto& g : b->graphs) {
    (void)hipGraphExecDestroy(g.exec);
    (void)hipGraphDestroy(g.graph);
  }
  b->graphs.clear();
}

}  // namespace

RD_API rd_status rd_batch_create(rd_mesh* const* meshes, int n, void* stream, rd_batch** out) {
  if (!out) return fail(RD_EINVAL, "null output pointer");
  *out = nullptr;
  if (!meshes || n <= 0) return fail(RD_EINVAL, "empty batch");
  const double gamma = meshes[0] ? meshes[0]->gamma : 0.0;
  // The batch unwraps triangles with one period per axis: the members that
  // are periodic on an axis must share their period there. A member that is
  // not periodic on that axis is laid out as it is; unwrapping leaves its
  // triangles and wall edges alone when every coordinate difference along
  // them is at most half the period, and its tiles' centroids (strictly
  // inside its extent) stay put when that extent is at most the period (both
  // checked).
  double bp[2] = {0.0, 0.0};
  for (int k = 0; k < n; ++k) {
    const rd_mesh* m = meshes[k];
    if (!m) return fail(RD_EINVAL, "null mesh in batch");
    const double mp[2] = {m->px, m->py};
    for (int a = 0; a < 2; ++a)
      if (mp[a] > 0.0) {
        if (bp[a] == 0.0) bp[a] = mp[a];
        else if (mp[a] != bp[a])
          return fail(RD_EINVAL, "batched meshes periodic on the same axis must share the period");
      }
  }
  for (int k = 0; k < n; ++k) {
    const rd_mesh* m = meshes[k];
    const double mp[2] = {m->px, m->py};
    const std::vector<double>* c[2] = {&m->x, &m->y};
    for (int a = 0; a < 2; ++a) {
      if (bp[a] == 0.0 || mp[a] > 0.0) continue;
      const std::vector<double>& q = *c[a];
      const auto r = std::minmax_element(q.begin(), q.end());
      bool ok = *r.second - *r.first <= bp[a];
      for (size_t t = 0; ok && t < m->tri.size(); t += 3)
        for (int i = 1; i < 3; ++i) ok = ok && std::fabs(q[m->tri[t + i]] - q[m->tri[t]]) <= 0.5 * bp[a];
      for (size_t e = 0; ok && e < m->wall.size(); e += 2)
        ok = std::fabs(q[m->wall[e + 1]] - q[m->wall[e]]) <= 0.5 * bp[a];
      if (!ok)
        return fail(RD_EINVAL, "batched mesh " + std::to_string(k) + " is not periodic on an axis where others are, "
                               "and its extent or a triangle's extent along that axis is too large for their period");
    }
  }
  std::vector<double> x, y;
  std::vector<int32_t> tri, wall;
  std::vector<uint8_t> ghost;
  std::vector<int64_t> voff{0}, toff{0};
  for (int k = 0; k < n; ++k) {
    const rd_mesh* m = meshes[k];
    if (m->gamma != gamma) return fail(RD_EINVAL, "batched meshes must share gamma");
    if (m->device != meshes[0]->device) return fail(RD_EINVAL, "batched meshes must live on one device");
    const int32_t vo = (int32_t)voff.back();
    x.insert(x.end(), m->x.begin(), m->x.end());
    y.insert(y.end(), m->y.begin(), m->y.end());
    for (int32_t v : m->tri) tri.push_back(v + vo);
    for (int32_t v : m->wall) wall.push_back(v + vo);
    ghost.insert(ghost.end(), m->ghost.begin(), m->ghost.end());
    voff.push_back(voff.back() + m->d.nv);
    toff.push_back(toff.back() + m->d.nt);
  }
  if (voff.back() >= (int64_t(1) << 31) || 3 * toff.back() >= (int64_t(1) << 31))
    return fail(RD_EINVAL, "batch too large for 32-bit indices");
  rd_mesh_desc desc{};
  desc.n_vertices = voff.back();
  desc.n_triangles = toff.back();
  desc.x = x.data();
  desc.y = y.data();
  desc.tri = tri.data();
  desc.period_x = bp[0];
  desc.period_y = bp[1];
  desc.ghost = ghost.data();
  desc.n_wall_edges = (int64_t)wall.size() / 2;
  desc.wall_edges = wall.empty() ? nullptr : wall.data();
  desc.gamma = gamma;
  DeviceGuard g(meshes[0]->device);
  hipStream_t own = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  HIPCHK(hipStreamCreateWithFlags(&own, hipStreamNonBlocking));
  if (hipEventCreateWithFlags(&ev_in, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ev_out, hipEventDisableTiming) != hipSuccess) {
    (void)hipStreamDestroy(own);
    return fail(RD_EDEVICE, "hipEventCreate failed");
  }
  rd_mesh* flat = nullptr;
  rd_status st = rd_mesh_create(&desc, own, &flat);
  if (st != RD_OK) {
    (void)hipEventDestroy(ev_in);
    (void)hipEventDestroy(ev_out);
    (void)hipStreamDestroy(own);
    return st;
  }
  // mesh ids, per-mesh time steps, per-mesh CFL segments
  std::vector<int32_t> vm(voff.back()), tm(toff.back()), v0, v1, b0{0};
  for (int k = 0; k < n; ++k) {
    for (int64_t i = voff[k]; i < voff[k + 1]; ++i) vm[i] = k;
    for (int64_t t = toff[k]; t < toff[k + 1]; ++t) tm[t] = k;
    for (int64_t v = voff[k]; v < voff[k + 1]; v += rd::kCflSpan) {
      v0.push_back((int32_t)v);
      v1.push_back((int32_t)std::min<int64_t>(v + rd::kCflSpan, voff[k + 1]));
    }
    b0.push_back((int32_t)v0.size());
  }
  int32_t *pvm, *ptm, *pv0, *pv1, *pb0;
  double *dt, *part, *vpart, *vr;
  int* mflag;  // one non-physical latch per member
  std::vector<double> vr0(3 * n, 0.0);
  for (int k = 0; k < n; ++k) vr0[3 * k + 2] = meshes[k]->Ldom;  // each member's own domain size
  if ((st = upload(flat, &pvm, vm)) || (st = upload(flat, &ptm, tm)) || (st = upload(flat, &pv0, v0)) ||
      (st = upload(flat, &pv1, v1)) || (st = upload(flat, &pb0, b0)) || (st = dalloc(flat, &dt, n)) ||
      (st = dalloc(flat, &part, v0.size())) || (st = dalloc(flat, &vpart, 2 * v0.size())) ||
      (st = upload(flat, &vr, vr0)) || (st = upload(flat, &mflag, std::vector<int>(n, 0)))) {
    rd_mesh_destroy(flat);
    return st;
  }
  flat->d.flag = mflag;
  flat->d.vr = vr;
  flat->cfl.vpart = vpart;
  flat->voff = voff;
  flat->toff = toff;
  flat->d.vmesh = pvm;
  flat->d.tmesh = ptm;
  flat->d.dt = dt;
  flat->cfl.nblocks = (int32_t)v0.size();
  flat->cfl.nmesh = n;
  flat->cfl.blk_v0 = pv0;
  flat->cfl.blk_v1 = pv1;
  flat->cfl.mesh_b0 = pb0;
  flat->cfl.part = part;
  rd_batch* b = new rd_batch();
  b->flat = flat;
  b->members.assign(meshes, meshes + n);
  b->voff = voff;
  b->toff = toff;
  b->stream = static_cast<hipStream_t>(stream);
  b->own = own;
  b->ev_in = ev_in;
  b->ev_out = ev_out;
  *out = b;
  return RD_OK;
}

namespace {

// Orders the batch's stream after the caller's and the members' pending work
// and copies the members' states in.
rd_status batch_begin(rd_batch* b, int fp32, std::vector<hipStream_t>& outer) {
  rd_mesh* f = b->flat;
  // the members' lumping, which must agree
  for (rd_mesh* m : b->members)
    if (m->d.slump != b->members[0]->d.slump)
      return fail(RD_EINVAL, "the meshes of a batch use different lumpings");
  f->d.slump = b->members[0]->d.slump;
  hipStream_t s = f->stream;  // the batch's own stream
  outer.assign(1, b->stream);
  for (rd_mesh* m : b->members)
    if (std::find(outer.begin(), outer.end(), m->stream) == outer.end()) outer.push_back(m->stream);
  for (hipStream_t o : outer) {
    HIPCHK(hipEventRecord(b->ev_in, o));
    HIPCHK(hipStreamWaitEvent(s, b->ev_in, 0));
  }
  for (size_t k = 0; k < b->members.size(); ++k) {
    rd_mesh* m = b->members[k];
    HIPCHK(rd::launch_copy4(f->d.W + b->voff[k], m->d.W, m->d.nv, s));
  }
  HIPCHK(rd::launch_fill_int(f->d.flag, 0, (int64_t)b->members.size(), s));
  f->zprec = -1;
  return ensure_z(f, fp32);
}

// The captured graph of n_steps steps (cached per configuration; the cache
// is dropped whenever the tile size changes).
rd_status batch_graph(rd_batch* b, int n_steps, double cfl, int scheme, int time, int fp32,
                      hipGraphExec_t* exec) {
  rd_mesh* f = b->flat;
  hipStream_t s = f->stream;
  for (auto& c : b->graphs)
    if (c.n_steps == n_steps && c.scheme == scheme && c.time == time && c.fp32 == fp32 && c.cfl == cfl &&
        c.slump == f->d.slump) {
      *exec = c.exec;
      return RD_OK;
    }
  rd_batch::Graph c{n_steps, scheme, time, fp32, f->d.slump, cfl, nullptr, nullptr};
  HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  rd_status rs = RD_OK;
  for (int k = 0; k < n_steps && rs == RD_OK; ++k) rs = run_step(f, scheme, time, fp32, cfl);
  hipError_t ce = hipStreamEndCapture(s, &c.graph);
  if (rs != RD_OK) {
    if (ce == hipSuccess) (void)hipGraphDestroy(c.graph);
    return rs;
  }
  if (ce != hipSuccess) return fail(RD_EDEVICE, std::string("graph capture: ") + hipGetErrorString(ce));
  hipError_t ie = hipGraphInstantiate(&c.exec, c.graph, nullptr, nullptr, 0);
  if (ie != hipSuccess) {
    (void)hipGraphDestroy(c.graph);
    return fail(RD_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(ie));
  }
  b->graphs.push_back(c);
  *exec = c.exec;
  return RD_OK;
}

rd_status batch_set_tile(rd_batch* b, int tt) {
  if (tt == b->flat->tile) return RD_OK;
  DeviceGuard g(b->flat->device);
  (void)hipStreamSynchronize(b->own);
  destroy_graphs(b);
  return set_tile(b->flat, tt);
}

}  // namespace

RD_API rd_status rd_batch_run(rd_batch* b, int n_steps, double cfl, int scheme, int time, int precision) {
  if (!b) return fail(RD_EINVAL, "null batch");
  if (n_steps < 0) return fail(RD_EINVAL, "negative step count");
  if (!(cfl > 0.0)) return fail(RD_EINVAL, "cfl must be positive");
  rd_status st = check_step_args(scheme, time, precision);
  if (st != RD_OK) return st;
  rd_mesh* f = b->flat;
  DeviceGuard g(f->device);
  const int fp32 = precision == RD_FP32_ACC64;
  if ((st = ensure_prec(f, fp32)) != RD_OK) return st;
  hipStream_t s = f->stream;
  std::vector<hipStream_t> outer;
  if ((st = batch_begin(b, fp32, outer)) != RD_OK) return st;
  if (n_steps > 0) {
    hipGraphExec_t exec = nullptr;
    if ((st = batch_graph(b, n_steps, cfl, scheme, time, fp32, &exec)) != RD_OK) return st;
    HIPCHK(hipGraphLaunch(exec, s));
  }
  // states out; each member refreshes its parameter vectors before its next step
  for (size_t k = 0; k < b->members.size(); ++k) {
    rd_mesh* m = b->members[k];
    HIPCHK(rd::launch_copy4(m->d.W, f->d.W + b->voff[k], m->d.nv, s));
    HIPCHK(rd::launch_or_int(m->d.flag, f->d.flag + k, s));
    m->zprec = -1;
  }
  HIPCHK(hipEventRecord(b->ev_out, s));
  for (hipStream_t o : outer) HIPCHK(hipStreamWaitEvent(o, b->ev_out, 0));
  return RD_OK;
}

RD_API rd_status rd_batch_set_tile(rd_batch* b, int tile_triangles) {
  if (!b) return fail(RD_EINVAL, "null batch");
  return batch_set_tile(b, tile_triangles);
}

RD_API rd_status rd_batch_tune(rd_batch* b, double cfl, int scheme, int time, int precision, int n_steps,
                               const int* candidates, int n_candidates, double* ms_per_step, int* best) {
  if (!b) return fail(RD_EINVAL, "null batch");
  rd_status st = tune_args(cfl, scheme, time, precision, n_steps, candidates, n_candidates, best);
  if (st != RD_OK) return st;
  rd_mesh* f = b->flat;
  DeviceGuard g(f->device);
  const int fp32 = precision == RD_FP32_ACC64;
  if ((st = ensure_prec(f, fp32)) != RD_OK) return st;
  hipStream_t s = f->stream;
  const int prev = f->tile;
  int pick = -1;
  float pick_ms = 0.0f;
  std::vector<hipStream_t> outer;
  for (int i = 0; i < n_candidates; ++i) {
    if (ms_per_step) ms_per_step[i] = -1.0;
    st = batch_set_tile(b, candidates[i]);
    if (st == RD_EUNSUPPORTED || st == RD_EINVAL) continue;
    if (st != RD_OK) break;
    hipGraphExec_t exec = nullptr;
    if ((st = batch_begin(b, fp32, outer)) != RD_OK) break;
    if ((st = batch_graph(b, n_steps, cfl, scheme, time, fp32, &exec)) != RD_OK) break;
    HIPCHK(hipGraphLaunch(exec, s));  // warm-up replay
    if ((st = batch_begin(b, fp32, outer)) != RD_OK) break;
    float t = 0.0f;
    st = time_on(s, [&]() -> rd_status {
      HIPCHK(hipGraphLaunch(exec, s));
      return RD_OK;
    }, &t);
    if (st != RD_OK) break;
    if (ms_per_step) ms_per_step[i] = t / n_steps;
    if (pick < 0 || t < pick_ms * (1.0f - kTuneMargin)) {
      pick = candidates[i];
      pick_ms = t;
    }
  }
  if (st == RD_EUNSUPPORTED || st == RD_EINVAL) st = RD_OK;
  rd_status st2 = batch_set_tile(b, pick >= 0 ? pick : prev);
  HIPCHK(hipStreamSynchronize(s));
  if (st != RD_OK) return st;
  if (st2 != RD_OK) return st2;
  if (pick < 0) return fail(RD_EUNSUPPORTED, "no candidate tile size is usable");
  *best = pick;
  return RD_OK;
}

RD_API rd_status rd_batch_destroy(rd_batch* b) {
  if (!b) return RD_OK;
  DeviceGuard g(b->flat->device);
  (void)hipStreamSynchronize(b->own);
  destroy_graphs(b);
  rd_mesh_destroy(b->flat);
  (void)hipEventDestroy(b->ev_in);
  (void)hipEventDestroy(b->ev_out);
  (void)hipStreamDestroy(b->own);
  delete b;
  return RD_OK;
}

RD_API rd_status rd_sync(rd_mesh* m) {
  if (!m) return fail(RD_EINVAL, "null mesh");
  DeviceGuard g(m->device);
  int flag = 0;
  HIPCHK(hipMemcpyAsync(&flag, m->d.flag, sizeof(int), hipMemcpyDeviceToHost, m->stream));
  HIPCHK(hipStreamSynchronize(m->stream));
  if (flag) return fail(RD_ENONPHYS, "a non-physical state was produced");
  return adjoint_status(m);
}

RD_API const char* rd_last_error(void) { return g_last_error.c_str(); }

// ---------------------------------------------------- mesh generation --
//
// A triangulation is checked as a mesh is (indices, counter-clockwise
// triangles after unwrapping); the neighbour table is built on the host from
// sorted vertex pairs; the flip rounds and refinement iterations run on the
// current device (rd_delaunay.hip), the host reading a few counters per
// round.

namespace {

// Device buffers of one mesh-generation call, freed together.
struct DlBuffers {
  std::vector<void*> p;
  DlBuffers() = default;
  DlBuffers(const DlBuffers&) = delete;
  DlBuffers& operator=(const DlBuffers&) = delete;
  ~DlBuffers() {
    for (void* q : p) (void)hipFree(q);
  }
  template <class T>
  bool get(T** out, size_t n) {
    void* q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) return false;
    p.push_back(q);
    *out = static_cast<T*>(q);
    return true;
  }
};

// Corner and neighbour tables [3][ts] of nt triangles (tri: [nt][3]).
rd_status dl_tables(int64_t nv, int64_t nt, int64_t ts, const int32_t* tri, std::vector<int32_t>& tsoa,
                    std::vector<int32_t>& nbr) {
  tsoa.assign(3 * ts, -1);
  nbr.assign(3 * ts, -1);
  struct Edge {
    int64_t key;
    int32_t t, i;
  };
  std::vector<Edge> edges(3 * nt);
  for (int64_t t = 0; t < nt; ++t)
    for (int i = 0; i < 3; ++i) {
      const int64_t b = tri[3 * t + (i + 1) % 3], c = tri[3 * t + (i + 2) % 3];
      edges[3 * t + i] = {std::min(b, c) * nv + std::max(b, c), (int32_t)t, i};
      tsoa[i * ts + t] = tri[3 * t + i];
    }
  std::sort(edges.begin(), edges.end(), [](const Edge& p, const Edge& q) { return p.key < q.key; });
  for (size_t k = 0; k < edges.size();) {
    size_t l = k + 1;
    while (l < edges.size() && edges[l].key == edges[k].key) ++l;
    if (l - k > 2) return fail(RD_EINVAL, "an edge belongs to more than two triangles");
    if (l - k == 2) {
      nbr[edges[k].i * ts + edges[k].t] = edges[k + 1].t;
      nbr[edges[k + 1].i * ts + edges[k + 1].t] = edges[k].t;
    }
    k = l;
  }
  return RD_OK;
}

bool hip_ok(hipError_t e) { return e == hipSuccess; }

// Flip rounds until no interior edge of m is illegal. Round and test-pass
// numbers continue across calls (*round, *pass: the pass about to run, whose
// marked triangles' edges are tested); m.work is allocated on first need.
rd_status dl_flip_all(rd::dl::Mesh& m, DlBuffers& b, hipStream_t s, int64_t* flips, int32_t* round, int32_t* pass) {
  const int64_t cap = 3 * m.ts / 2 + 1;  // interior edges at most
  const int64_t chunk = std::min<int64_t>(cap, 4096);  // exact tests per launch
  int32_t cnt[3] = {0, 0, 0};
  auto read_counts = [&]() {
    return hip_ok(hipMemcpyAsync(cnt, m.count, sizeof(cnt), hipMemcpyDeviceToHost, s)) &&
           hip_ok(hipStreamSynchronize(s));
  };
  const int32_t kMaxRounds = 1000000;
  for (int32_t n = 0;; ++n) {
    const int32_t p = (*pass)++;
    if (!hip_ok(rd::dl::launch_reset(m, s)) || !hip_ok(rd::dl::launch_mark(m, p, s)) || !read_counts())
      return fail(RD_EDEVICE, "in-circle pass failed");
    if (cnt[2] > 0) {
      if (!m.work && !b.get(&m.work, chunk * rd::dl::exact_scratch()))
        return fail(RD_ENOMEM, "device allocation failed");
      for (int64_t f = 0; f < cnt[2]; f += chunk)
        if (!hip_ok(rd::dl::launch_exact(m, f, std::min<int64_t>(cnt[2], f + chunk), s)))
          return fail(RD_EDEVICE, "exact in-circle pass failed");
      if (!read_counts()) return fail(RD_EDEVICE, "exact in-circle pass failed");
    }
    if (cnt[1] == 0) return RD_OK;
    if (n >= kMaxRounds) return fail(RD_EDEVICE, "flipping did not finish");
    ++*round;
    if (!hip_ok(rd::dl::launch_flip(m, *round, p, s)) || !hip_ok(rd::dl::launch_fix(m, *round, s)) ||
        !read_counts())
      return fail(RD_EDEVICE, "flip pass failed");
    if (cnt[0] < 1) return fail(RD_EDEVICE, "a round flipped no edge");
    *flips += cnt[0];
  }
}

// Device arrays of the flip passes for a capacity of ts triangles.
bool dl_flip_arrays(rd::dl::Mesh& m, DlBuffers& b, int64_t ts) {
  return b.get(&m.tri, 3 * ts) && b.get(&m.nbr, 3 * ts) && b.get(&m.claim, ts) && b.get(&m.cand, ts) &&
         b.get(&m.flipped, ts) && b.get(&m.partner, ts) && b.get(&m.count, 3) && b.get(&m.mark, ts) &&
         b.get(&m.undecided, 3 * ts / 2 + 1);
}

// Renumber vertices, then triangles, in Morton order (the moved arrays are
// swapped in: m's and o's pointers trade places).
rd_status dl_reorder(rd::dl::Mesh& m, rd::dl::Order& o, int64_t nv, void* tmp, size_t tmp_bytes, hipStream_t s) {
  if (!hip_ok(rd::dl::launch_vkeys(m, o, nv, s)) || !hip_ok(rd::dl::launch_sort(o, nv, tmp, tmp_bytes, s)) ||
      !hip_ok(rd::dl::launch_invert(o, nv, s)) || !hip_ok(rd::dl::launch_vapply(m, o, nv, s)) ||
      !hip_ok(rd::dl::launch_vrename(m, o, s)))
    return fail(RD_EDEVICE, "vertex reordering failed");
  std::swap(m.x, o.xt);
  std::swap(m.y, o.yt);
  if (!hip_ok(rd::dl::launch_tkeys(m, o, s)) || !hip_ok(rd::dl::launch_sort(o, m.nt, tmp, tmp_bytes, s)) ||
      !hip_ok(rd::dl::launch_invert(o, m.nt, s)) || !hip_ok(rd::dl::launch_tapply(m, o, s)))
    return fail(RD_EDEVICE, "triangle reordering failed");
  std::swap(m.tri, o.tt);
  std::swap(m.nbr, o.nb);
  return RD_OK;
}

struct StreamGuard {
  hipStream_t s = nullptr;
  ~StreamGuard() {
    if (s) {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
    }
  }
};

}  // namespace

RD_API rd_status rd_delaunay_flip(int64_t n_vertices, const double* x, const double* y, double period_x,
                                  double period_y, int64_t n_triangles, int32_t* tri, int64_t* n_flips,
                                  int32_t* n_rounds) {
  rd_mesh_desc desc{};
  desc.n_vertices = n_vertices;
  desc.n_triangles = n_triangles;
  desc.x = x;
  desc.y = y;
  desc.tri = tri;
  desc.period_x = period_x;
  desc.period_y = period_y;
  desc.gamma = 1.4;  // not used; the check requires a valid value
  rd_status st = check_desc(&desc, nullptr);
  if (st != RD_OK) return st;
  const int64_t nt = n_triangles, nv = n_vertices;
  std::vector<int32_t> nbr, tsoa;
  if ((st = dl_tables(nv, nt, nt, tri, tsoa, nbr)) != RD_OK) return st;
  DlBuffers b;
  StreamGuard g;  // declared after the buffers: the stream is drained before they are freed
  rd::dl::Mesh m;
  m.nt = nt;
  m.ts = nt;
  m.px = period_x;
  m.py = period_y;
  if (!b.get(&m.x, nv) || !b.get(&m.y, nv) || !dl_flip_arrays(m, b, nt))
    return fail(RD_ENOMEM, "device allocation failed");
  if (hipStreamCreate(&g.s) != hipSuccess) return fail(RD_EDEVICE, "hipStreamCreate failed");
  const hipStream_t s = g.s;
  if (!hip_ok(hipMemcpyAsync(m.x, x, sizeof(double) * nv, hipMemcpyHostToDevice, s)) ||
      !hip_ok(hipMemcpyAsync(m.y, y, sizeof(double) * nv, hipMemcpyHostToDevice, s)) ||
      !hip_ok(hipMemcpyAsync(m.tri, tsoa.data(), sizeof(int32_t) * 3 * nt, hipMemcpyHostToDevice, s)) ||
      !hip_ok(hipMemcpyAsync(m.nbr, nbr.data(), sizeof(int32_t) * 3 * nt, hipMemcpyHostToDevice, s)) ||
      !hip_ok(hipMemsetAsync(m.flipped, 0, sizeof(int32_t) * nt, s)) ||
      !hip_ok(hipMemsetAsync(m.mark, 0, sizeof(int32_t) * nt, s)))
    return fail(RD_EDEVICE, "upload failed");
  int64_t flips = 0;
  int32_t round = 0, pass = 0;  // every mark is 0: the first pass tests every edge
  if ((st = dl_flip_all(m, b, s, &flips, &round, &pass)) != RD_OK) return st;
  if (!hip_ok(hipMemcpyAsync(tsoa.data(), m.tri, sizeof(int32_t) * 3 * nt, hipMemcpyDeviceToHost, s)) ||
      !hip_ok(hipStreamSynchronize(s)))
    return fail(RD_EDEVICE, "download failed");
  for (int64_t t = 0; t < nt; ++t)
    for (int i = 0; i < 3; ++i) tri[3 * t + i] = tsoa[i * nt + t];
  if (n_flips) *n_flips = flips;
  if (n_rounds) *n_rounds = round;
  return RD_OK;
}

RD_API rd_status rd_delaunay_refine(int64_t* n_vertices, double* x, double* y, int64_t max_vertices,
                                    double period_x, double period_y, int64_t* n_triangles, int32_t* tri,
                                    int64_t max_triangles, double max_radius, double max_ratio,
                                    const double* size_grid, int32_t grid_nx, int32_t grid_ny,
                                    int32_t max_iterations, int32_t morton, int32_t* n_iterations,
                                    int64_t* n_flips) {
  if (!n_vertices || !n_triangles) return fail(RD_EINVAL, "null count pointer");
  const int64_t nv0 = *n_vertices, nt0 = *n_triangles;
  if (max_vertices < nv0 || max_triangles < nt0) return fail(RD_EINVAL, "capacity below the current size");
  if (max_vertices >= INT32_MAX || max_triangles >= INT32_MAX / 3)  // edge keys 3 t + i are int32
    return fail(RD_EINVAL, "capacity beyond the 32-bit index range");
  if (!(max_radius >= 0.0) || !std::isfinite(max_radius)) return fail(RD_EINVAL, "max_radius must be >= 0");
  if (!(max_ratio == 0.0 || max_ratio >= 1.0) || !std::isfinite(max_ratio))
    return fail(RD_EINVAL, "max_ratio must be 0 (no bound) or >= 1");
  if (max_iterations < 1) return fail(RD_EINVAL, "max_iterations must be >= 1");
  if (morton != 0 && morton != 1) return fail(RD_EINVAL, "morton must be 0 or 1");
  if (size_grid) {
    if (grid_nx < 1 || grid_ny < 1 || (int64_t)grid_nx * grid_ny > (1 << 26))
      return fail(RD_EINVAL, "size grid dimensions must be >= 1 (at most 2^26 nodes)");
    for (int64_t k = 0; k < (int64_t)grid_nx * grid_ny; ++k)
      if (!(size_grid[k] > 0.0) || !std::isfinite(size_grid[k]))
        return fail(RD_EINVAL, "size grid values must be positive and finite");
  }
  rd_mesh_desc desc{};
  desc.n_vertices = nv0;
  desc.n_triangles = nt0;
  desc.x = x;
  desc.y = y;
  desc.tri = tri;
  desc.period_x = period_x;
  desc.period_y = period_y;
  desc.gamma = 1.4;  // not used; the check requires a valid value
  rd_status st = check_desc(&desc, nullptr);
  if (st != RD_OK) return st;
  for (int64_t v = 0; v < nv0; ++v)
    if ((period_x > 0.0 && !(x[v] >= 0.0 && x[v] < period_x)) || (period_y > 0.0 && !(y[v] >= 0.0 && y[v] < period_y)))
      return fail(RD_EINVAL, "a coordinate on a periodic axis is outside [0, period)");
  const int64_t ts = max_triangles;
  std::vector<int32_t> nbr, tsoa;
  if ((st = dl_tables(nv0, nt0, ts, tri, tsoa, nbr)) != RD_OK) return st;
  for (int64_t t = 0; t < nt0; ++t)
    for (int i = 0; i < 3; ++i) {
      if (nbr[i * ts + t] >= 0) continue;
      const int32_t b = tsoa[((i + 1) % 3) * ts + t], c = tsoa[((i + 2) % 3) * ts + t];
      if (x[b] != x[c] && y[b] != y[c]) return fail(RD_EINVAL, "a boundary edge is not axis-aligned");
    }
  DlBuffers b;
  StreamGuard g;
  rd::dl::Mesh m;
  rd::dl::Refine r;
  m.nt = nt0;
  m.ts = ts;
  m.px = period_x;
  m.py = period_y;
  r.nv = nv0;
  r.r2 = max_radius * max_radius;
  r.b2 = max_ratio * max_ratio;
  if (!b.get(&m.x, max_vertices) || !b.get(&m.y, max_vertices) || !dl_flip_arrays(m, b, ts) ||
      !b.get(&r.prio, ts) || !b.get(&r.px, ts) || !b.get(&r.py, ts) || !b.get(&r.loc, ts) ||
      !b.get(&r.where, ts) || !b.get(&r.lock, ts) || !b.get(&r.win, ts) || !b.get(&r.wpos, ts) ||
      !b.get(&r.tnew, ts) || !b.get(&r.tpos, ts) || !b.get(&r.split, ts) || !b.get(&r.child, 2 * ts) ||
      !b.get(&r.count, 3))
    return fail(RD_ENOMEM, "device allocation failed");
  if (size_grid) {
    // grid frame: the period on a periodic axis (nodes wrap), else the input's extent
    auto frame = [&](const double* c, double period, int32_t n, double& g0, double& gd) {
      double lo = c[0], hi = c[0];
      for (int64_t v = 1; v < nv0; ++v) {
        lo = std::min(lo, c[v]);
        hi = std::max(hi, c[v]);
      }
      g0 = period > 0.0 ? 0.0 : lo;
      gd = period > 0.0 ? period / n : (n > 1 ? (hi - lo) / (n - 1) : 1.0);
    };
    frame(x, period_x, grid_nx, r.gx0, r.gdx);
    frame(y, period_y, grid_ny, r.gy0, r.gdy);
    double* g = nullptr;
    const int64_t ng = (int64_t)grid_nx * grid_ny;
    if (!b.get(&g, ng)) return fail(RD_ENOMEM, "device allocation failed");
    if (hipMemcpy(g, size_grid, sizeof(double) * ng, hipMemcpyHostToDevice) != hipSuccess)
      return fail(RD_EDEVICE, "upload failed");
    r.sgrid = g;
    r.gnx = grid_nx;
    r.gny = grid_ny;
  }
  const size_t scan_bytes = rd::dl::scan_tmp_bytes(ts);
  char* scan_tmp = nullptr;
  if (!b.get(&scan_tmp, scan_bytes)) return fail(RD_ENOMEM, "device allocation failed");
  rd::dl::Order o;
  size_t sort_bytes = 0;
  char* sort_tmp = nullptr;
  if (morton) {
    // Morton frame: the period on a periodic axis, else the input's extent
    auto frame = [&](const double* c, double period, double& c0, double& sc) {
      double lo = c[0], hi = c[0];
      for (int64_t v = 1; v < nv0; ++v) {
        lo = std::min(lo, c[v]);
        hi = std::max(hi, c[v]);
      }
      c0 = period > 0.0 ? 0.0 : lo;
      sc = 4294967296.0 / (period > 0.0 ? period : hi - lo);
    };
    frame(x, period_x, o.x0, o.sx);
    frame(y, period_y, o.y0, o.sy);
    const int64_t n = std::max(max_vertices, ts);
    sort_bytes = rd::dl::sort_tmp_bytes(n);
    if (!b.get(&o.key, n) || !b.get(&o.skey, n) || !b.get(&o.idx, n) || !b.get(&o.perm, n) || !b.get(&o.inv, n) ||
        !b.get(&o.xt, max_vertices) || !b.get(&o.yt, max_vertices) || !b.get(&o.tt, 3 * ts) ||
        !b.get(&o.nb, 3 * ts) || !b.get(&sort_tmp, sort_bytes))
      return fail(RD_ENOMEM, "device allocation failed");
  }
  if (hipStreamCreate(&g.s) != hipSuccess) return fail(RD_EDEVICE, "hipStreamCreate failed");
  const hipStream_t s = g.s;
  if (!hip_ok(hipMemcpyAsync(m.x, x, sizeof(double) * nv0, hipMemcpyHostToDevice, s)) ||
      !hip_ok(hipMemcpyAsync(m.y, y, sizeof(double) * nv0, hipMemcpyHostToDevice, s)) ||
      !hip_ok(hipMemcpyAsync(m.tri, tsoa.data(), sizeof(int32_t) * 3 * ts, hipMemcpyHostToDevice, s)) ||
      !hip_ok(hipMemcpyAsync(m.nbr, nbr.data(), sizeof(int32_t) * 3 * ts, hipMemcpyHostToDevice, s)) ||
      !hip_ok(hipMemsetAsync(m.flipped, 0, sizeof(int32_t) * ts, s)) ||
      !hip_ok(hipMemsetAsync(m.mark, 0, sizeof(int32_t) * ts, s)) ||
      !hip_ok(hipMemsetAsync(r.split, 0, sizeof(int32_t) * ts, s)))
    return fail(RD_EDEVICE, "upload failed");
  int64_t flips = 0;
  int32_t round = 0, it = 0, pass = 0;  // every mark is 0: the first pass tests every edge
  int64_t nv = nv0, nt = nt0, nt_ordered = nt0;
  // the mesh reached so far goes back to the caller, also when a limit stops the loop
  auto download = [&](rd_status result) {
    if (!hip_ok(hipMemcpyAsync(x, m.x, sizeof(double) * nv, hipMemcpyDeviceToHost, s)) ||
        !hip_ok(hipMemcpyAsync(y, m.y, sizeof(double) * nv, hipMemcpyDeviceToHost, s)) ||
        !hip_ok(hipMemcpyAsync(tsoa.data(), m.tri, sizeof(int32_t) * 3 * ts, hipMemcpyDeviceToHost, s)) ||
        !hip_ok(hipStreamSynchronize(s)))
      return fail(RD_EDEVICE, "download failed");
    for (int64_t t = 0; t < nt; ++t)
      for (int i = 0; i < 3; ++i) tri[3 * t + i] = tsoa[i * ts + t];
    *n_vertices = nv;
    *n_triangles = nt;
    if (n_iterations) *n_iterations = it;
    if (n_flips) *n_flips = flips;
    return result;
  };
  if ((st = dl_flip_all(m, b, s, &flips, &round, &pass)) != RD_OK) return st;
  int32_t cnt[3];
  for (;;) {
    r.seed = 0x9e3779b9u * (uint32_t)(it + 1);
    if (!hip_ok(hipMemsetAsync(r.count, 0, sizeof(cnt), s)) || !hip_ok(rd::dl::launch_quality(m, r, s)) ||
        !hip_ok(hipMemcpyAsync(cnt, r.count, sizeof(cnt), hipMemcpyDeviceToHost, s)) ||
        !hip_ok(hipStreamSynchronize(s)))
      return fail(RD_EDEVICE, "quality pass failed");
    if (cnt[0] == 0) {
      if (cnt[1] > 0)
        return download(fail(RD_EUNSUPPORTED, "a circumcentre lies more than a quarter period from its triangle"));
      if (morton && nt != nt_ordered && (st = dl_reorder(m, o, nv, sort_tmp, sort_bytes, s)) != RD_OK) return st;
      return download(RD_OK);
    }
    if (it >= max_iterations) return download(fail(RD_EINVAL, "refinement needs more than max_iterations iterations"));
    ++it;
    if (!hip_ok(rd::dl::launch_locate(m, r, s)) || !hip_ok(rd::dl::launch_lock(m, r, s)) ||
        !hip_ok(rd::dl::launch_check(m, r, s)) ||
        !hip_ok(rd::dl::launch_scan(r.win, r.wpos, nt, scan_tmp, scan_bytes, s)) ||
        !hip_ok(rd::dl::launch_scan(r.tnew, r.tpos, nt, scan_tmp, scan_bytes, s)))
      return fail(RD_EDEVICE, "insertion-set passes failed");
    int32_t last[4];
    if (!hip_ok(hipMemcpyAsync(&last[0], r.win + nt - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s)) ||
        !hip_ok(hipMemcpyAsync(&last[1], r.wpos + nt - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s)) ||
        !hip_ok(hipMemcpyAsync(&last[2], r.tnew + nt - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s)) ||
        !hip_ok(hipMemcpyAsync(&last[3], r.tpos + nt - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s)) ||
        !hip_ok(hipMemcpyAsync(cnt, r.count, sizeof(cnt), hipMemcpyDeviceToHost, s)) ||
        !hip_ok(hipStreamSynchronize(s)))
      return fail(RD_EDEVICE, "insertion-set passes failed");
    const int64_t nwin = (int64_t)last[0] + last[1], nadd = (int64_t)last[2] + last[3];
    if (nwin == 0)
      return download(fail(RD_EUNSUPPORTED, "no candidate could be inserted (" + std::to_string(cnt[1]) +
                                                " not located, " + std::to_string(cnt[2]) + " cavities too large)"));
    if (nv + nwin > max_vertices || nt + nadd > max_triangles)
      return download(fail(RD_ENOMEM, "the refined mesh needs more than max_vertices or max_triangles"));
    r.nv = nv;
    if (!hip_ok(rd::dl::launch_insert(m, r, it, pass, s)) ||
        !hip_ok(rd::dl::launch_fixsplit(m, r, it, nt + nadd, s)))
      return fail(RD_EDEVICE, "insertion failed");
    nv += nwin;
    nt += nadd;
    m.nt = nt;
    if ((st = dl_flip_all(m, b, s, &flips, &round, &pass)) != RD_OK) return st;
    if (morton && 4 * nt >= 5 * nt_ordered) {  // renumber after every 25 % of growth, and at the end
      if ((st = dl_reorder(m, o, nv, sort_tmp, sort_bytes, s)) != RD_OK) return st;
      nt_ordered = nt;
    }
  }
}

// --------------------------------------------------------- three dimensions --
//
// Host side of the tetrahedral path: validation and geometry (face normals,
// volumes, vertex volumes), the sliced-ELL slot order of the vertex sums,
// buffers and the launch order of a step (kernels in rd3_kernels.hip).

struct rd3_mesh {
  rd3::Dev3 d;
  std::vector<void*> bufs;
  hipStream_t stream = nullptr;
  ~rd3_mesh() {
    if (stream) {
      (void)hipStreamSynchronize(stream);
      (void)hipStreamDestroy(stream);
    }
    for (void* q : bufs) (void)hipFree(q);
  }
};

namespace {

double unwrap3(double d, double period) {
  if (period > 0.0) {
    if (d > 0.5 * period) d -= period;
    else if (d < -0.5 * period) d += period;
  }
  return d;
}

template <class T>
bool dev_get(rd3_mesh* m, T** out, size_t n) {
  void* q = nullptr;
  if (hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) return false;
  m->bufs.push_back(q);
  *out = static_cast<T*>(q);
  return true;
}

rd_status rd3_check_step(int scheme, int time) {
  if (scheme < RD_N || scheme > RD_BMIN) return fail(RD_EINVAL, "unknown scheme for three dimensions");
  if (time != RD_EULER1 && time != RD_RK2) return fail(RD_EINVAL, "unknown time integration");
  return RD_OK;
}

// One step after *d.dt is set on the stream.
rd_status rd3_stages(rd3_mesh* m, int scheme, int time, hipEvent_t* ev) {
  const rd3::Dev3& d = m->d;
  const hipStream_t s = m->stream;
  auto mark = [&](int k) { return ev ? hipEventRecord(ev[k], s) : hipSuccess; };
  HIPCHK(rd3::launch3_tet(d, 1, scheme, time == RD_RK2, s));
  HIPCHK(mark(2));
  HIPCHK(rd3::launch3_gather(d, time == RD_RK2 ? 1 : 0, s));
  HIPCHK(mark(3));
  if (time == RD_RK2) {
    HIPCHK(rd3::launch3_tet(d, 2, scheme, false, s));
    HIPCHK(mark(4));
    HIPCHK(rd3::launch3_gather(d, 2, s));
    HIPCHK(mark(5));
  }
  return RD_OK;
}

}  // namespace

RD_API rd_status rd3_mesh_create(const rd3_mesh_desc* desc, rd3_mesh** out) {
  if (!desc || !out) return fail(RD_EINVAL, "null argument");
  *out = nullptr;
  const int64_t nv = desc->n_vertices, nt = desc->n_tets;
  if (nv < 4 || nt < 1) return fail(RD_EINVAL, "empty mesh");
  if (nv >= INT32_MAX || nt >= INT32_MAX / 4) return fail(RD_EINVAL, "mesh too large for 32-bit indices");
  if (!desc->x || !desc->y || !desc->z || !desc->tet) return fail(RD_EINVAL, "null array");
  if (!(desc->gamma > 1.0)) return fail(RD_EINVAL, "gamma must exceed 1");
  const double per[3] = {desc->period_x, desc->period_y, desc->period_z};
  for (double p : per)
    if (!(p >= 0.0) || !std::isfinite(p)) return fail(RD_EINVAL, "invalid period");
  const double* xyz[3] = {desc->x, desc->y, desc->z};
  std::vector<double> nrm(12 * nt), vol(nt), smax(nt), V(nv, 0.0);
  std::vector<int32_t> tsoa(4 * nt), cnt(nv + 1, 0);
  for (int64_t t = 0; t < nt; ++t) {
    int32_t v[4];
    for (int i = 0; i < 4; ++i) {
      v[i] = desc->tet[4 * t + i];
      if (v[i] < 0 || v[i] >= nv) return fail(RD_EINVAL, "tetrahedron " + std::to_string(t) + ": index out of range");
      tsoa[i * nt + t] = v[i];
    }
    double p[4][3];
    for (int i = 0; i < 4; ++i)
      for (int k = 0; k < 3; ++k) p[i][k] = i == 0 ? 0.0 : unwrap3(xyz[k][v[i]] - xyz[k][v[0]], per[k]);
    auto cr = [](const double* a, const double* b, double* c) {
      c[0] = a[1] * b[2] - a[2] * b[1];
      c[1] = a[2] * b[0] - a[0] * b[2];
      c[2] = a[0] * b[1] - a[1] * b[0];
    };
    double c[3];
    cr(p[2], p[3], c);
    const double six = p[1][0] * c[0] + p[1][1] * c[1] + p[1][2] * c[2];
    if (!(six > 0.0)) return fail(RD_EINVAL, "tetrahedron " + std::to_string(t) + " is not positively oriented");
    vol[t] = six / 6.0;
    double sm = 0.0;
    for (int i = 0; i < 4; ++i) {
      const double* a = p[(i + 1) % 4];
      const double* b = p[(i + 2) % 4];
      const double* e = p[(i + 3) % 4];
      const double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
      const double e2[3] = {e[0] - a[0], e[1] - a[1], e[2] - a[2]};
      double n[3];
      cr(e1, e2, n);
      const double to[3] = {p[i][0] - a[0], p[i][1] - a[1], p[i][2] - a[2]};
      const double sgn = (n[0] * to[0] + n[1] * to[1] + n[2] * to[2]) < 0.0 ? -0.5 : 0.5;
      for (int k = 0; k < 3; ++k) nrm[(3 * i + k) * nt + t] = sgn * n[k];
      sm = std::max(sm, 0.5 * std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]));
    }
    smax[t] = sm;
    for (int i = 0; i < 4; ++i) {
      V[v[i]] += vol[t] / 4.0;
      ++cnt[v[i] + 1];
    }
  }
  for (int64_t v = 0; v < nv; ++v)
    if (!(V[v] > 0.0)) return fail(RD_EINVAL, "vertex " + std::to_string(v) + " belongs to no tetrahedron");
  // sliced-ELL slots: slices of 64 vertices, each as wide as its largest degree
  const int64_t nslice = (nv + 63) / 64;
  std::vector<int32_t> deg(nv), sbase(nslice);
  int64_t ns = 0;
  for (int64_t q = 0; q < nslice; ++q) {
    int32_t w = 0;
    for (int64_t v = 64 * q; v < std::min(nv, 64 * q + 64); ++v) {
      deg[v] = cnt[v + 1];
      w = std::max(w, deg[v]);
    }
    sbase[q] = (int32_t)ns;
    ns += 64 * (int64_t)w;
  }
  if (ns >= INT32_MAX) return fail(RD_EINVAL, "mesh too large for 32-bit slot indices");
  std::vector<int32_t> slot(4 * nt), fill(nv, 0);
  for (int64_t t = 0; t < nt; ++t)  // ascending tetrahedron within each vertex
    for (int i = 0; i < 4; ++i) {
      const int32_t v = tsoa[i * nt + t];
      slot[i * nt + t] = sbase[v / 64] + 64 * fill[v]++ + v % 64;
    }
  std::unique_ptr<rd3_mesh> m(new rd3_mesh());
  rd3::Dev3& d = m->d;
  d.nv = nv;
  d.nt = nt;
  d.ns = ns;
  d.gamma = desc->gamma;
  int32_t *dtet, *dslot, *ddeg, *dsbase;
  double *dnrm, *dvol, *dsmax, *dV;
  const int nb = rd3::cfl_blocks(nv);
  if (!dev_get(m.get(), &dtet, 4 * nt) || !dev_get(m.get(), &dslot, 4 * nt) || !dev_get(m.get(), &ddeg, nv) ||
      !dev_get(m.get(), &dsbase, nslice) ||
      !dev_get(m.get(), &dnrm, 12 * nt) || !dev_get(m.get(), &dvol, nt) || !dev_get(m.get(), &dsmax, nt) ||
      !dev_get(m.get(), &dV, nv) || !dev_get(m.get(), &d.W, 5 * nv) || !dev_get(m.get(), &d.Ws, 5 * nv) ||
      !dev_get(m.get(), &d.Z, 5 * nv) || !dev_get(m.get(), &d.rate, 5 * nv) || !dev_get(m.get(), &d.sig, nv) || !dev_get(m.get(), &d.part, 5 * ns) ||
      !dev_get(m.get(), &d.keepN, 15 * nt) || !dev_get(m.get(), &d.keepT, 5 * nt) ||
      !dev_get(m.get(), &d.cpart, ns) || !dev_get(m.get(), &d.dt, 1) || !dev_get(m.get(), &d.bmin, nb) ||
      !dev_get(m.get(), &d.flag, 1))
    return fail(RD_ENOMEM, "device allocation failed");
  HIPCHK(hipStreamCreate(&m->stream));
  const hipStream_t s = m->stream;
  HIPCHK(hipMemcpyAsync(dtet, tsoa.data(), sizeof(int32_t) * 4 * nt, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(dslot, slot.data(), sizeof(int32_t) * 4 * nt, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(ddeg, deg.data(), sizeof(int32_t) * nv, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(dsbase, sbase.data(), sizeof(int32_t) * nslice, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(dnrm, nrm.data(), sizeof(double) * 12 * nt, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(dvol, vol.data(), sizeof(double) * nt, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(dsmax, smax.data(), sizeof(double) * nt, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(dV, V.data(), sizeof(double) * nv, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemsetAsync(d.W, 0, sizeof(double) * 5 * nv, s));
  HIPCHK(hipMemsetAsync(d.flag, 0, sizeof(int), s));
  HIPCHK(hipStreamSynchronize(s));
  d.tet = dtet;
  d.slot = dslot;
  d.deg = ddeg;
  d.sbase = dsbase;
  d.nrm = dnrm;
  d.vol = dvol;
  d.smax = dsmax;
  d.V = dV;
  *out = m.release();
  return RD_OK;
}

RD_API rd_status rd3_mesh_destroy(rd3_mesh* mesh) {
  delete mesh;
  return RD_OK;
}

RD_API rd_status rd3_set_state(rd3_mesh* m, const double* W, int on_device) {
  if (!m || !W) return fail(RD_EINVAL, "null argument");
  const int64_t nv = m->d.nv;
  if (!on_device) {
    for (int64_t i = 0; i < nv; ++i) {
      const double rho = W[i], e = W[4 * nv + i];
      const double q = W[nv + i] * W[nv + i] + W[2 * nv + i] * W[2 * nv + i] + W[3 * nv + i] * W[3 * nv + i];
      if (!(rho > 0.0) || !std::isfinite(e) || !((m->d.gamma - 1.0) * (e - 0.5 * q / rho) > 0.0))
        return fail(RD_ENONPHYS, "vertex " + std::to_string(i) + ": rho <= 0, p <= 0 or not finite");
    }
  }
  HIPCHK(hipMemcpyAsync(m->d.W, W, sizeof(double) * 5 * nv, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                        m->stream));
  HIPCHK(hipMemsetAsync(m->d.flag, 0, sizeof(int), m->stream));
  HIPCHK(rd3::launch3_z(m->d, m->d.W, m->stream));
  if (!on_device) HIPCHK(hipStreamSynchronize(m->stream));
  return RD_OK;
}

RD_API rd_status rd3_get_state(rd3_mesh* m, double* W, int on_device) {
  if (!m || !W) return fail(RD_EINVAL, "null argument");
  HIPCHK(hipMemcpyAsync(W, m->d.W, sizeof(double) * 5 * m->d.nv,
                        on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, m->stream));
  HIPCHK(hipStreamSynchronize(m->stream));
  return RD_OK;
}

RD_API rd_status rd3_max_dt(rd3_mesh* m, double cfl, double* dt) {
  if (!m || !dt) return fail(RD_EINVAL, "null argument");
  if (!(cfl > 0.0)) return fail(RD_EINVAL, "cfl must be positive");
  HIPCHK(rd3::launch3_cfl(m->d, cfl, m->stream));
  HIPCHK(hipMemcpyAsync(dt, m->d.dt, sizeof(double), hipMemcpyDeviceToHost, m->stream));
  HIPCHK(hipStreamSynchronize(m->stream));
  return RD_OK;
}

RD_API rd_status rd3_step(rd3_mesh* m, double dt, int scheme, int time) {
  if (!m) return fail(RD_EINVAL, "null mesh");
  rd_status st = rd3_check_step(scheme, time);
  if (st != RD_OK) return st;
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(RD_EINVAL, "dt must be positive");
  HIPCHK(rd3::launch3_set_dt(m->d, dt, m->stream));
  return rd3_stages(m, scheme, time, nullptr);
}

RD_API rd_status rd3_step_cfl(rd3_mesh* m, int n_steps, double cfl, int scheme, int time) {
  if (!m) return fail(RD_EINVAL, "null mesh");
  rd_status st = rd3_check_step(scheme, time);
  if (st != RD_OK) return st;
  if (!(cfl > 0.0) || n_steps < 0) return fail(RD_EINVAL, "cfl must be positive and n_steps >= 0");
  for (int k = 0; k < n_steps; ++k) {
    HIPCHK(rd3::launch3_cfl(m->d, cfl, m->stream));
    if ((st = rd3_stages(m, scheme, time, nullptr)) != RD_OK) return st;
  }
  return RD_OK;
}

RD_API rd_status rd3_step_timed(rd3_mesh* m, int n_steps, double cfl, int scheme, int time, double* ms) {
  if (!m || !ms) return fail(RD_EINVAL, "null argument");
  rd_status st = rd3_check_step(scheme, time);
  if (st != RD_OK) return st;
  if (!(cfl > 0.0) || n_steps < 1) return fail(RD_EINVAL, "cfl must be positive and n_steps >= 1");
  hipEvent_t ev[6];
  for (auto& e : ev) HIPCHK(hipEventCreate(&e));
  struct Free {
    hipEvent_t* e;
    ~Free() {
      for (int k = 0; k < 6; ++k) (void)hipEventDestroy(e[k]);
    }
  } guard{ev};
  for (int k = 0; k < 5; ++k) ms[k] = 0.0;
  for (int n = 0; n < n_steps; ++n) {
    HIPCHK(hipEventRecord(ev[0], m->stream));
    HIPCHK(rd3::launch3_cfl(m->d, cfl, m->stream));
    HIPCHK(hipEventRecord(ev[1], m->stream));
    if ((st = rd3_stages(m, scheme, time, ev)) != RD_OK) return st;
    HIPCHK(hipStreamSynchronize(m->stream));
    const int last = time == RD_RK2 ? 5 : 3;
    for (int k = 0; k < last; ++k) {
      float t = 0.0f;
      HIPCHK(hipEventElapsedTime(&t, ev[k], ev[k + 1]));
      ms[k] += t / n_steps;
    }
  }
  return RD_OK;
}

RD_API rd_status rd3_sync(rd3_mesh* m) {
  if (!m) return fail(RD_EINVAL, "null mesh");
  int flag = 0;
  HIPCHK(hipMemcpyAsync(&flag, m->d.flag, sizeof(int), hipMemcpyDeviceToHost, m->stream));
  HIPCHK(hipStreamSynchronize(m->stream));
  if (flag) return fail(RD_ENONPHYS, "a non-physical state was produced");
  return RD_OK;
}

