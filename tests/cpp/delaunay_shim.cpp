// Host build of the mesh-generation bodies (rd_delaunay_kern.h) for their
// CPU tests: the same per-element code the GPU kernels run, executed one
// element at a time in the order of the device driver (each pass reads only
// what earlier passes wrote, so this sequential run equals the parallel one).
// Built with g++ and -ffp-contract=off.
#include <algorithm>
#include <cstdint>
#include <vector>

#include "rd_delaunay_kern.h"

namespace {

using rd::dl::Mesh;
using rd::dl::Refine;

struct Host {
  std::vector<double> x, y, work;
  std::vector<int32_t> tri, nbr, claim, cand, flipped, partner, mark, count{0, 0, 0};
  std::vector<int64_t> undecided;
  std::vector<unsigned long long> prio, lock;
  std::vector<double> px, py;
  std::vector<int32_t> loc, where, win, wpos, tnew, tpos, split, child, rcount{0, 0, 0};
};

void tables(int64_t nv, int64_t nt, int64_t ts, const int32_t* tri, Host& h) {
  h.tri.assign(3 * ts, -1);
  h.nbr.assign(3 * ts, -1);
  struct Edge {
    int64_t key;
    int32_t t, i;
  };
  std::vector<Edge> e(3 * nt);
  for (int64_t t = 0; t < nt; ++t)
    for (int i = 0; i < 3; ++i) {
      const int64_t b = tri[3 * t + (i + 1) % 3], c = tri[3 * t + (i + 2) % 3];
      e[3 * t + i] = {std::min(b, c) * nv + std::max(b, c), (int32_t)t, i};
      h.tri[i * ts + t] = tri[3 * t + i];
    }
  std::sort(e.begin(), e.end(), [](const Edge& p, const Edge& q) { return p.key < q.key; });
  for (size_t k = 0; k + 1 < e.size(); ++k)
    if (e[k].key == e[k + 1].key) {
      h.nbr[e[k].i * ts + e[k].t] = e[k + 1].t;
      h.nbr[e[k + 1].i * ts + e[k + 1].t] = e[k].t;
    }
}

Mesh view(Host& h, int64_t nt, int64_t ts, double px, double py) {
  Mesh m;
  m.nt = nt;
  m.ts = ts;
  m.x = h.x.data();
  m.y = h.y.data();
  m.px = px;
  m.py = py;
  m.tri = h.tri.data();
  m.nbr = h.nbr.data();
  m.claim = h.claim.data();
  m.cand = h.cand.data();
  m.flipped = h.flipped.data();
  m.partner = h.partner.data();
  m.mark = h.mark.data();
  m.count = h.count.data();
  m.undecided = h.undecided.data();
  m.work = h.work.data();
  return m;
}

void alloc(Host& h, int64_t ts) {
  h.claim.assign(ts, 0);
  h.cand.assign(ts, 0);
  h.flipped.assign(ts, 0);
  h.partner.assign(ts, 0);
  h.mark.assign(ts, 0);
  h.undecided.assign(3 * ts / 2 + 1, 0);
  h.work.assign(rd::pred::kIncircleScratch, 0.0);
}

// The counters the kernels add with wave_add are added here from the
// bodies' results.
int flip_all(Mesh& m, int64_t* flips, int32_t* round, int32_t* pass) {
  for (;;) {
    const int32_t p = (*pass)++;
    for (int64_t t = 0; t < std::max<int64_t>(m.nt, 3); ++t) rd::dl::reset_body(m, t);
    for (int64_t t = 0; t < m.nt; ++t) {
      const int r = rd::dl::mark_body(m, t, p);
      for (int i = 0; i < 3; ++i) {
        m.count[1] += (r >> i) & 1;
        if ((r >> (4 + i)) & 1) m.undecided[m.count[2]++] = 3 * t + i;
      }
    }
    for (int64_t k = 0; k < m.count[2]; ++k) m.count[1] += rd::dl::exact_body(m, k, m.work);
    if (m.count[1] == 0) return 0;
    ++*round;
    for (int64_t t = 0; t < m.nt; ++t) m.count[0] += rd::dl::flip_body(m, t, *round, p);
    for (int64_t t = 0; t < m.nt; ++t) rd::dl::fix_body(m, t, *round);
    if (m.count[0] < 1) return 3;
    *flips += m.count[0];
  }
}

// Morton renumbering with the library's bodies; the sort is a stable sort
// by key, as the device's radix sort is.
struct Reorder {
  std::vector<uint32_t> key;
  std::vector<int32_t> idx, perm, inv, tt, nb;
  std::vector<double> xt, yt;
  rd::dl::Order o;
};

void sort_perm(Reorder& q, int64_t n) {
  std::vector<int32_t> p(q.idx.begin(), q.idx.begin() + n);
  std::stable_sort(p.begin(), p.end(), [&](int32_t a, int32_t b) { return q.key[a] < q.key[b]; });
  std::copy(p.begin(), p.end(), q.perm.begin());
}

void reorder(Host& h, Mesh& m, Reorder& q, int64_t nv) {
  rd::dl::Order& o = q.o;
  for (int64_t v = 0; v < nv; ++v) rd::dl::vkey_body(m, o, v);
  sort_perm(q, nv);
  for (int64_t i = 0; i < nv; ++i) rd::dl::invert_body(o, i);
  for (int64_t i = 0; i < nv; ++i) rd::dl::vapply_body(m, o, i);
  for (int64_t t = 0; t < m.nt; ++t) rd::dl::vrename_body(m, o, t);
  h.x.swap(q.xt);
  h.y.swap(q.yt);
  m.x = h.x.data();
  m.y = h.y.data();
  o.xt = q.xt.data();
  o.yt = q.yt.data();
  for (int64_t t = 0; t < m.nt; ++t) rd::dl::tkey_body(m, o, t);
  sort_perm(q, m.nt);
  for (int64_t i = 0; i < m.nt; ++i) rd::dl::invert_body(o, i);
  for (int64_t i = 0; i < m.nt; ++i) rd::dl::tapply_body(m, o, i);
  h.tri.swap(q.tt);
  h.nbr.swap(q.nb);
  m.tri = h.tri.data();
  m.nbr = h.nbr.data();
  o.tt = q.tt.data();
  o.nb = q.nb.data();
}

void download(Host& h, int64_t nt, int64_t ts, int32_t* tri) {
  for (int64_t t = 0; t < nt; ++t)
    for (int i = 0; i < 3; ++i) tri[3 * t + i] = h.tri[i * ts + t];
}

}  // namespace

extern "C" {

// rd_delaunay_flip's passes; returns 0, or 3 when a round flips nothing.
int rdl_flip(int64_t nv, const double* x, const double* y, double px, double py, int64_t nt, int32_t* tri,
             int64_t* n_flips, int32_t* n_rounds) {
  Host h;
  h.x.assign(x, x + nv);
  h.y.assign(y, y + nv);
  tables(nv, nt, nt, tri, h);
  alloc(h, nt);
  Mesh m = view(h, nt, nt, px, py);
  int64_t flips = 0;
  int32_t round = 0, pass = 0;
  const int st = flip_all(m, &flips, &round, &pass);
  download(h, nt, nt, tri);
  *n_flips = flips;
  *n_rounds = round;
  return st;
}

// rd_delaunay_refine's passes and driver (status codes as the library's:
// 0 done, 1 iteration limit, 2 capacity, 5 no insertable candidate or a
// circumcentre too far on a periodic axis, 3 flips stuck).
int rdl_refine(int64_t* n_vertices, double* x, double* y, int64_t max_v, double px, double py, int64_t* n_triangles,
               int32_t* tri, int64_t max_t, double max_radius, double max_ratio, const double* size_grid,
               int32_t grid_nx, int32_t grid_ny, int32_t max_iterations, int32_t morton, int32_t* n_iterations,
               int64_t* n_flips) {
  Host h;
  const int64_t ts = max_t;
  int64_t nv = *n_vertices, nt = *n_triangles;
  h.x.assign(max_v, 0.0);
  h.y.assign(max_v, 0.0);
  std::copy(x, x + nv, h.x.begin());
  std::copy(y, y + nv, h.y.begin());
  tables(nv, nt, ts, tri, h);
  alloc(h, ts);
  h.prio.assign(ts, 0);
  h.lock.assign(ts, 0);
  h.px.assign(ts, 0.0);
  h.py.assign(ts, 0.0);
  for (auto* v : {&h.loc, &h.where, &h.win, &h.wpos, &h.tnew, &h.tpos, &h.split}) v->assign(ts, 0);
  h.child.assign(2 * ts, -1);
  Mesh m = view(h, nt, ts, px, py);
  Refine r;
  r.nv = nv;
  r.r2 = max_radius * max_radius;
  r.b2 = max_ratio * max_ratio;
  r.prio = h.prio.data();
  r.px = h.px.data();
  r.py = h.py.data();
  r.loc = h.loc.data();
  r.where = h.where.data();
  r.lock = h.lock.data();
  r.win = h.win.data();
  r.wpos = h.wpos.data();
  r.tnew = h.tnew.data();
  r.tpos = h.tpos.data();
  r.split = h.split.data();
  r.child = h.child.data();
  r.count = h.rcount.data();
  if (size_grid) {  // the library's grid frame
    auto frame = [&](const double* c, double period, int32_t n, double& g0, double& gd) {
      double lo = c[0], hi = c[0];
      for (int64_t v = 1; v < nv; ++v) {
        lo = std::min(lo, c[v]);
        hi = std::max(hi, c[v]);
      }
      g0 = period > 0.0 ? 0.0 : lo;
      gd = period > 0.0 ? period / n : (n > 1 ? (hi - lo) / (n - 1) : 1.0);
    };
    frame(x, px, grid_nx, r.gx0, r.gdx);
    frame(y, py, grid_ny, r.gy0, r.gdy);
    r.sgrid = size_grid;
    r.gnx = grid_nx;
    r.gny = grid_ny;
  }
  Reorder q;
  if (morton) {
    auto frame = [&](const double* c, double period, double& c0, double& sc) {
      double lo = c[0], hi = c[0];
      for (int64_t v = 1; v < nv; ++v) {
        lo = std::min(lo, c[v]);
        hi = std::max(hi, c[v]);
      }
      c0 = period > 0.0 ? 0.0 : lo;
      sc = 4294967296.0 / (period > 0.0 ? period : hi - lo);
    };
    frame(x, px, q.o.x0, q.o.sx);
    frame(y, py, q.o.y0, q.o.sy);
    const int64_t n = std::max(max_v, ts);
    q.key.assign(n, 0);
    q.idx.assign(n, 0);
    q.perm.assign(n, 0);
    q.inv.assign(n, 0);
    q.xt.assign(max_v, 0.0);
    q.yt.assign(max_v, 0.0);
    q.tt.assign(3 * ts, -1);
    q.nb.assign(3 * ts, -1);
    q.o.key = q.key.data();
    q.o.idx = q.idx.data();
    q.o.perm = q.perm.data();
    q.o.inv = q.inv.data();
    q.o.xt = q.xt.data();
    q.o.yt = q.yt.data();
    q.o.tt = q.tt.data();
    q.o.nb = q.nb.data();
  }
  int64_t flips = 0;
  int32_t round = 0, it = 0, pass = 0;
  int64_t nt_ordered = nt;
  int st = flip_all(m, &flips, &round, &pass);
  while (st == 0) {
    r.seed = 0x9e3779b9u * (uint32_t)(it + 1);
    r.count[0] = r.count[1] = r.count[2] = 0;
    for (int64_t t = 0; t < nt; ++t) {
      const int q = rd::dl::quality_body(m, r, t);
      r.count[0] += q == rd::dl::kCandidate;
      r.count[1] += q == rd::dl::kTooFar;
    }
    if (r.count[0] == 0) {
      st = r.count[1] > 0 ? 5 : 0;
      break;
    }
    if (it >= max_iterations) {
      st = 1;
      break;
    }
    ++it;
    for (int64_t t = 0; t < nt; ++t) rd::dl::locate_body(m, r, t);
    for (int64_t t = 0; t < nt; ++t) rd::dl::lock_body(m, r, t);
    for (int64_t t = 0; t < nt; ++t) rd::dl::check_body(m, r, t);
    int64_t nwin = 0, nadd = 0;
    for (int64_t t = 0; t < nt; ++t) {
      r.wpos[t] = (int32_t)nwin;
      r.tpos[t] = (int32_t)nadd;
      nwin += r.win[t];
      nadd += r.tnew[t];
    }
    if (nwin == 0) {
      st = 5;
      break;
    }
    if (nv + nwin > max_v || nt + nadd > max_t) {
      st = 2;
      break;
    }
    r.nv = nv;
    for (int64_t t = 0; t < nt; ++t) rd::dl::insert_body(m, r, t, it, pass);
    m.nt = nt + nadd;
    for (int64_t t = 0; t < nt + nadd; ++t) rd::dl::fixsplit_body(m, r, t, it);
    nv += nwin;
    nt += nadd;
    st = flip_all(m, &flips, &round, &pass);
    if (st == 0 && morton && 4 * nt >= 5 * nt_ordered) {
      reorder(h, m, q, nv);
      nt_ordered = nt;
    }
  }
  if (st == 0 && morton && nt != nt_ordered) reorder(h, m, q, nv);
  std::copy(h.x.begin(), h.x.begin() + nv, x);
  std::copy(h.y.begin(), h.y.begin() + nv, y);
  download(h, nt, ts, tri);
  *n_vertices = nv;
  *n_triangles = nt;
  *n_iterations = it;
  *n_flips = flips;
  return st;
}
}
