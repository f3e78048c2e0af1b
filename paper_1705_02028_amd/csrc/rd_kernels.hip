// gfx950 kernels of the two-pass residual-distribution step, the CFL
// reduction, state conversion and the adjoint, with their launchers.
//
// Launch shapes: one thread per triangle (triangle passes) or per vertex
// (gather, CFL), 256-thread workgroups, block ids renumbered per XCD.
#include "rd_adjoint.h"
#include "rd_kcommon.h"
#include "rd_launch.h"

namespace rd {

// One thread per triangle. (A persistent grid with the next triangle's loads
// software-pipelined was measured slower: fewer waves in flight and, with
// per-workgroup chunks, scattered working sets. So was the adjoint's staged
// form below applied to the FP64 passes, persistent one-wavefront workgroups
// with the next batch's gathered inputs loaded straight to LDS: 0.72-0.87 ms
// against 0.545 ms for the stage-1 pass at 2048^2, 0.51 against 0.50 for
// stage 2; two to three waves per SIMD already overlap these passes' gathers
// with each other's arithmetic.)
template <typename R, int SCHEME, int STAGE, bool SAVE, bool CFL, bool LUMP>
__global__ __launch_bounds__(kBlock, (TriKernelWaves<R, SCHEME, STAGE, SAVE, CFL>::value)) void k_tri(Dev d) {
  const int64_t t = xcd_block() * kBlock + threadIdx.x;
  if (t < d.nt)
    tri_body<R, SCHEME, STAGE, SAVE, CFL, LUMP, TriKernelWaves<R, SCHEME, STAGE, SAVE, CFL>::fast_div>(t, d);
}

template <typename R, int MODE>
__global__ __launch_bounds__(kBlock) void k_gather(Dev d, double* out_soa) {
  const int64_t v = xcd_block() * kBlock + threadIdx.x;
  if (v < d.nv) gather_body<R, MODE>(v, d, out_soa);
}

template <bool STAGE2, bool TILED>
__global__ __launch_bounds__(kBlock) void k_wall(Dev d) {
  const int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (b < d.nwv) wall_body<STAGE2, TILED>(b, d);
}

__global__ __launch_bounds__(kBlock) void k_cfl_tri(Dev d) {
  const int64_t t = xcd_block() * kBlock + threadIdx.x;
  if (t < d.nt) cfl_tri_body(t, d);
}

// Per-vertex CFL bounds 2 V_i / sum l_max lambda_max (summed over the terms of
// the vertex's triangles, or read from the bounds the tiled passes store) and
// their block minima.
template <bool FROM_CFLV, typename R>
__global__ __launch_bounds__(kBlock) void k_cfl_vertex(Dev d, CflPlan p) {
  constexpr int U = kCflSpan / kBlock;
  const int b = blockIdx.x;
  double x = INFINITY;
  int64_t v[U];
  bool in[U];
  for (int u = 0; u < U; ++u) {
    v[u] = (int64_t)p.blk_v0[b] + u * kBlock + threadIdx.x;
    in[u] = v[u] < p.blk_v1[b];
  }
  if (FROM_CFLV) {
    for (int u = 0; u < U; ++u)
      if (in[u]) x = rmin(x, d.cflv[v[u]]);
  } else {
    double bound[U];
    cfl_vertex_bounds<R, U>(v, in, p.blk_v0[b], d, bound);
    for (int u = 0; u < U; ++u)
      if (in[u]) x = rmin(x, bound[u]);
  }
  const double m = block_min(x);
  if (threadIdx.x == 0) p.part[b] = m;
}

// Per-mesh minimum over the mesh's blocks -> dt.
__global__ __launch_bounds__(kBlock) void k_cfl_final(Dev d, CflPlan p, double cfl) {
  const int m = blockIdx.x;
  double x = INFINITY;
  for (int b = p.mesh_b0[m] + threadIdx.x; b < p.mesh_b0[m + 1]; b += kBlock) x = rmin(x, p.part[b]);
  x = block_min(x);
  if (threadIdx.x == 0) d.dt[m] = cfl * x;
}

// Smallest and largest flow speed |v| over each CFL block's vertices (the Bx
// sensor's range), at W^n (MODE 0), at W* held in Ws (MODE 1) or at W*
// formed from the stage-1 residual (MODE 2, tiled form); then per mesh.
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_vrange(Dev d, CflPlan p) {
  const int b = blockIdx.x;
  double lo = INFINITY, hi = 0.0;
#pragma unroll
  for (int u = 0; u < kCflSpan / kBlock; ++u) {
    const int64_t v = (int64_t)p.blk_v0[b] + u * kBlock + threadIdx.x;
    if (v < p.blk_v1[b]) {
      const D4 w = MODE == 0 ? d.W[v] : (MODE == 1 ? d.Ws[v] : star_state(d, v, d.bc ? d.bc[v] : -1,
                                                                            d.vmesh ? d.vmesh[v] : 0));
      const double sp = flow_speed(w);
      lo = rmin(lo, sp);
      hi = rmax(hi, sp);
    }
  }
  lo = block_min(lo);
  __syncthreads();
  hi = -block_min(-hi);
  if (threadIdx.x == 0) {
    p.vpart[2 * b] = lo;
    p.vpart[2 * b + 1] = hi;
  }
}

__global__ __launch_bounds__(kBlock) void k_vrange_final(Dev d, CflPlan p) {
  const int m = blockIdx.x;
  double lo = INFINITY, hi = 0.0;
  for (int b = p.mesh_b0[m] + threadIdx.x; b < p.mesh_b0[m + 1]; b += kBlock) {
    lo = rmin(lo, p.vpart[2 * b]);
    hi = rmax(hi, p.vpart[2 * b + 1]);
  }
  lo = block_min(lo);
  __syncthreads();
  hi = -block_min(-hi);
  if (threadIdx.x == 0) {
    d.vr[3 * m] = lo;
    d.vr[3 * m + 1] = hi;
  }
}

__global__ __launch_bounds__(kBlock) void k_set_state(Dev d, const double* soa, int fp32) {
  const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (v >= d.nv) return;
  const double w[4] = {soa[v], soa[d.nv + v], soa[2 * d.nv + v], soa[3 * d.nv + v]};
  st4<double>(d.W, v, w);
  vertex_epilogue(d, v, w, fp32 != 0);
}

__global__ __launch_bounds__(kBlock) void k_refresh(Dev d, int fp32) {
  const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (v >= d.nv) return;
  const D4 w = d.W[v];
  vertex_epilogue(d, v, w.v, fp32 != 0);
}

__global__ __launch_bounds__(kBlock) void k_aos_to_soa(const D4* src, double* soa, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const D4 w = src[i];
  for (int k = 0; k < 4; ++k) soa[k * n + i] = w.v[k];
}

// FP64 kept triangle residuals (two 16-byte planes: components 0-1, then
// 2-3) to component-major arrays.
__global__ __launch_bounds__(kBlock) void k_keep_to_soa(const double2* src, double* soa, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double2 a = src[i], b = src[n + i];
  soa[i] = a.x;
  soa[n + i] = a.y;
  soa[2 * n + i] = b.x;
  soa[3 * n + i] = b.y;
}

__global__ void k_set_scalar(double* p, double v) { p[0] = v; }
__global__ void k_set_int(int* p, int v) { p[0] = v; }
__global__ void k_or_int(int* dst, const int* src) { dst[0] = dst[0] | src[0]; }
__global__ __launch_bounds__(kBlock) void k_fill_int(int* p, int v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = v;
}


__global__ __launch_bounds__(kBlock) void k_copy4(D4* dst, const D4* src, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// ------------------------------------------------------------- adjoint --

// The reverse triangle kernels run one wavefront per SIMD (their registers
// fill the SIMD), in one-wavefront workgroups.
constexpr int kAdjBlock = 64;

__global__ __launch_bounds__(kBlock) void k_adj_star(Dev d, AdjDev a) {
  const int64_t v = xcd_block() * kBlock + threadIdx.x;
  if (v < d.nv) adj_star_body(v, d, a);
}

__global__ __launch_bounds__(kBlock) void k_adj_euler_prep(Dev d, AdjDev a) {
  const int64_t v = xcd_block() * kBlock + threadIdx.x;
  if (v < d.nv) adj_euler_prep_body(v, d, a);
}

__global__ __launch_bounds__(kBlock) void k_adj_gather2(Dev d, AdjDev a) {
  const int64_t v = xcd_block() * kBlock + threadIdx.x;
  if (v < d.nv) adj_gather2_body(v, d, a);
}

__global__ __launch_bounds__(kBlock) void k_adj_gather1(Dev d, AdjDev a, int rk2, double* out) {
  const int64_t v = xcd_block() * kBlock + threadIdx.x;
  if (v < d.nv) adj_gather1_body(v, d, a, rk2 != 0, out);
}

__global__ __launch_bounds__(kBlock) void k_soa_to_aos(const double* soa, D4* dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double w[4] = {soa[i], soa[n + i], soa[2 * n + i], soa[3 * n + i]};
  st4<double>(dst, i, w);
}

__global__ __launch_bounds__(kBlock) void k_zero4(D4* dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double z[4] = {0.0, 0.0, 0.0, 0.0};
  st4<double>(dst, i, z);
}

// Staged reverse triangle passes. Each one-wavefront workgroup walks a
// contiguous run of 64-triangle batches, its inputs streaming from HBM into
// LDS through direct loads to LDS (16 bytes per lane per instruction,
// landing 16 bytes per lane apart: the staging is laid out [unit][lane]) so
// the wavefront never stalls on the gather of vertex records:
//  - eager inputs (corner ids, slot ranks and slot bases, coordinates,
//    parameter vectors) are loaded one batch ahead, moved to registers at the
//    start of the batch, and their buffer refilled with the next batch's;
//  - the rest (mu; for stage 2 W* - W^n and the kept stage-1 values, for
//    stage 1 their cotangents) is loaded at the start of its own batch and
//    read where the reverse uses it, past the start of the forward
//    recomputation, which covers the load's latency; each read first waits
//    for that batch's loads alone.
// Corner ids two batches ahead also go through LDS.
template <int STAGE>
struct AdjStaged {
  static constexpr int eager = 9;                   // xy (3), Z (6)
  static constexpr int late = STAGE == 2 ? 18 : 12;  // mu (6); stage 2: W* - W^n (6), kept N parts (4), kept residual (2);
                                                     // stage 1: cotangents of the kept values (6)
  // 16-byte stores every triangle's reverse issues unconditionally: stage 2
  // three 64-byte corner records and three 32-byte kept-value cotangents,
  // stage 1 three 32-byte corner records
  static constexpr int stores = STAGE == 2 ? 18 : 6;
  // direct loads issued after a batch's late ones and before its reverse:
  // the next batch's ids (4), slot bases (3) and eager units, the ids two ahead (4)
  static constexpr int after_late = 4 + 3 + eager + 4;
};

// Waits the compiler keeps where they are written (it moves no memory access
// across them). Vector memory operations, direct loads to LDS included,
// complete in issue order, so vmcnt(N) means all but the last N issued have.
// The assembly comments name the waits and loads for the check of their
// counts on the compiled code (tests/test_staged_waits.py): a "late" wait
// waits for the last "late" loads, any other for the last direct loads.
template <int N, bool LATE = false>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt takes 6 bits");
  if constexpr (LATE) asm volatile("s_waitcnt vmcnt(%0) ; staged wait: late" ::"n"(N) : "memory");
  else asm volatile("s_waitcnt vmcnt(%0) ; staged wait" ::"n"(N) : "memory");
}
__device__ __forceinline__ void wait_lgkmcnt0() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// Direct load to LDS: lane l's 16 (4) bytes from src land at dst + 16 l (4 l);
// dst is the same for the whole wavefront (it goes in M0). Written as asm so
// that the compiler does not track these loads: the kernel orders every read
// of the staged data after them with its own waits (its tracking of such
// loads, when it cannot tell the LDS buffers apart, waits on every load in
// flight before any LDS read, which would undo the staging).
__device__ __forceinline__ uint32_t lds_addr(const void* p) {
  return (uint32_t)(uintptr_t)(__attribute__((address_space(3))) const void*)p;
}
template <bool LATE = false>
__device__ __forceinline__ void lds_dma16(const void* src, double2* dst) {
  if constexpr (LATE)
    asm volatile("s_nop 0\n\tglobal_load_lds_dwordx4 %0, off ; staged load: late" ::"v"(src), "{m0}"(lds_addr(dst))
                 : "memory");
  else
    asm volatile("s_nop 0\n\tglobal_load_lds_dwordx4 %0, off ; staged load" ::"v"(src), "{m0}"(lds_addr(dst))
                 : "memory");
}
__device__ __forceinline__ void lds_dma4(const void* src, int32_t* dst) {
  asm volatile("s_nop 0\n\tglobal_load_lds_dword %0, off ; staged load" ::"v"(src), "{m0}"(lds_addr(dst)) : "memory");
}

// A late input in LDS (its two 16-byte halves 64 units apart): each read
// first waits for its batch's loads, issued K direct loads before the last.
// The scheduling barrier keeps the wait where the reverse reads the value
// (the compiler would otherwise hoist it, and its stall, to the top).
template <int K>
struct D4Late {
  const double2* p = nullptr;
  __device__ D4 operator*() const {
    __builtin_amdgcn_sched_barrier(0);
    wait_vmcnt<K, true>();
    return *D4Lds{p};
  }
  __device__ explicit operator bool() const { return p != nullptr; }
};
// mu of the current batch (corner i in rows 2i, 2i+1)
template <int K>
struct MuLate {
  const double2* p;  // this lane's unit in row 0
  __device__ D4 get(int i) const { return *D4Late<K>{p + 128 * i}; }
};

// The eager inputs of one batch held in registers.
struct AdjEager {
  int32_t slot[3];
  double2 p[3];
  D4 z[3];
};

template <int SCHEME, int STAGE>
__global__ __launch_bounds__(kAdjBlock) void k_adj_tri_staged(Dev d, AdjDev a, int rk2, int64_t per) {
  using S = AdjStaged<STAGE>;
  constexpr int K = S::after_late;
  __shared__ __attribute__((aligned(16))) double2 eb[S::eager * 64];  // eager units of the next batch
  __shared__ __attribute__((aligned(16))) double2 lt[S::late * 64];   // late units of the current batch
  __shared__ int32_t ie[7 * 64];  // next batch: corner ids, rank word, slot bases of the corners' vertex slices
  __shared__ int32_t ib[4 * 64];  // corner ids and rank word two batches ahead
  const int l = threadIdx.x;
  const int64_t nb = (d.nt + 63) >> 6;
  const int64_t b0 = xcd_block() * per;
  const int64_t b1 = b0 + per < nb ? b0 + per : nb;
  if (b0 >= b1) return;
  const bool kept = STAGE == 2 || rk2 != 0;
  // this lane's triangle in batch b; batches past the run repeat its last one
  // and lanes past the mesh its last triangle (same inputs, same results)
  auto tri = [&](int64_t b) {
    const int64_t t = (b < b1 ? b : b1 - 1) * 64 + l;
    return (int32_t)(t < d.nt ? t : d.nt - 1);
  };
  auto issue_ids = [&](int32_t t, int32_t* dst) {
    for (int i = 0; i < 3; ++i) lds_dma4(&d.tv[i * d.nt + t], &dst[i * 64]);
    lds_dma4(&d.rk[t], &dst[3 * 64]);
  };
  auto rec = [&](int32_t v) {
    return STAGE == 2 ? reinterpret_cast<const char*>(&a.r2[v]) : reinterpret_cast<const char*>(&a.r1[v]);
  };
  // eager loads of batch b (corner ids iv) into eb and ie
  auto issue_eager = [&](int64_t b, const int32_t iv[3]) {
    issue_ids(tri(b), ie);
    for (int i = 0; i < 3; ++i) lds_dma4(&d.sbase[iv[i] >> 6], &ie[(4 + i) * 64]);
    for (int i = 0; i < 3; ++i) lds_dma16(&d.xy[iv[i]], &eb[i * 64]);
    for (int i = 0; i < 3; ++i)
      for (int c = 0; c < 2; ++c) lds_dma16(rec(iv[i]) + 16 * c, &eb[(3 + 2 * i + c) * 64]);  // Z
  };
  // late loads of batch b (triangle t, corner ids iv) into lt
  auto issue_late = [&](int32_t t, const int32_t iv[3]) {
    for (int i = 0; i < 3; ++i)
      for (int c = 0; c < 2; ++c) lds_dma16<true>(rec(iv[i]) + (STAGE == 2 ? 64 : 32) + 16 * c, &lt[(2 * i + c) * 64]);
    if (STAGE == 2) {
      for (int i = 0; i < 3; ++i)
        for (int c = 0; c < 2; ++c) lds_dma16<true>(rec(iv[i]) + 32 + 16 * c, &lt[(6 + 2 * i + c) * 64]);  // W* - W^n
      // kept stage-1 records: 16-byte planes, chunk c of triangle t at c nt + t
      const char* kn = reinterpret_cast<const char*>(d.keepN) + 16 * (int64_t)t;
      for (int c = 0; c < 4; ++c) lds_dma16<true>(kn + 16 * c * d.nt, &lt[(12 + c) * 64]);
      const char* kt = reinterpret_cast<const char*>(d.keepT) + 16 * (int64_t)t;
      for (int c = 0; c < 2; ++c) lds_dma16<true>(kt + 16 * c * d.nt, &lt[(16 + c) * 64]);
    } else if (kept) {
      // the stage-2 reverse's kept-part cotangents: 16-byte planes as above
      const char* kn = reinterpret_cast<const char*>(a.kN) + 16 * (int64_t)t;
      for (int c = 0; c < 4; ++c) lds_dma16<true>(kn + 16 * c * d.nt, &lt[(6 + c) * 64]);
      const char* kt = reinterpret_cast<const char*>(a.kT) + 16 * (int64_t)t;
      for (int c = 0; c < 2; ++c) lds_dma16<true>(kt + 16 * c * d.nt, &lt[(10 + c) * 64]);
    }
  };
  // Batch b's eager inputs into registers; then its late loads, the eager
  // loads of batch b+1 and the ids of batch b+2. The eager loads of batch b
  // and the ids of b+1 were issued before the previous batch's reverse, whose
  // stores have been issued since: waiting until no more than those stores
  // are outstanding waits for them (the first batch waits for everything).
  AdjEager e;
  auto advance = [&](int64_t b, bool first) {
    if (first) wait_vmcnt<0>();
    else wait_vmcnt<S::stores>();
    const uint32_t rk = (uint32_t)ie[3 * 64 + l];
    int32_t iv[3];
    for (int i = 0; i < 3; ++i) {
      iv[i] = ie[i * 64 + l];
      e.slot[i] = ie[(4 + i) * 64 + l] + (iv[i] & 63) + 64 * (int32_t)((rk >> (10 * i)) & 1023u);
      e.p[i] = eb[i * 64 + l];
      e.z[i] = *D4Lds{&eb[(3 + 2 * i) * 64 + l]};
    }
    const int32_t nx[3] = {ib[l], ib[64 + l], ib[128 + l]};
    // every read of the buffers has returned before new loads overwrite them
    wait_lgkmcnt0();
    issue_late(tri(b), iv);
    issue_eager(b + 1, nx);
    issue_ids(tri(b + 2), ib);
  };
  auto compute = [&](int64_t b) {
    AdjTriIn<D4Late<K>, MuLate<K>> in;
    for (int i = 0; i < 3; ++i) {
      in.slot[i] = e.slot[i];
      in.p[i] = e.p[i];
      in.z[i] = e.z[i];
    }
    in.mu.p = &lt[l];
    if (STAGE == 2) {
      for (int i = 0; i < 3; ++i) in.dw[i].p = &lt[(6 + 2 * i) * 64 + l];
      in.kn[0].p = &lt[12 * 64 + l];
      in.kn[1].p = &lt[14 * 64 + l];
      in.kt.p = &lt[16 * 64 + l];
    } else if (kept) {
      in.kn[0].p = &lt[6 * 64 + l];
      in.kn[1].p = &lt[8 * 64 + l];
      in.kt.p = &lt[10 * 64 + l];
    }
    const int32_t t = tri(b);
    if (STAGE == 2) adj_tri2_compute<SCHEME>(t, d, a, in);
    else adj_tri1_compute<SCHEME>(t, d, a, in);
  };
  {
    const int32_t t = tri(b0);
    const int32_t iv[3] = {d.tv[t], d.tv[d.nt + t], d.tv[2 * d.nt + t]};
    issue_eager(b0, iv);
    issue_ids(tri(b0 + 1), ib);
  }
  advance(b0, true);
  for (int64_t b = b0; b < b1; ++b) {
    compute(b);
    advance(b + 1, false);
  }
  // the last (repeated) loads land before the workgroup's LDS is released
  wait_vmcnt<0>();
}

// a.waves workgroups (one per SIMD the device has), each taking a run of
// ceil(batches / a.waves) batches of 64 triangles
template <int SCHEME>
static void adj_tris(const Dev& d, const AdjDev& a, int stage, int rk2, hipStream_t s) {
  if (d.nt == 0) return;
  const int64_t nb = (d.nt + 63) / 64;
  const int64_t per = (nb + a.waves - 1) / a.waves;
  const unsigned g = (unsigned)((nb + per - 1) / per);
  if (stage == 2) hipLaunchKernelGGL((k_adj_tri_staged<SCHEME, 2>), dim3(g), dim3(kAdjBlock), 0, s, d, a, rk2, per);
  else hipLaunchKernelGGL((k_adj_tri_staged<SCHEME, 1>), dim3(g), dim3(kAdjBlock), 0, s, d, a, rk2, per);
}

hipError_t launch_adjoint(const Dev& d, const AdjDev& a, int scheme, int rk2, double* out, hipStream_t s) {
  if (a.waves <= 0) return hipErrorInvalidValue;
  auto tris = [&](int stage) {
    switch (scheme) {
      case SCH_N: adj_tris<SCH_N>(d, a, stage, rk2, s); break;
      case SCH_LDA: adj_tris<SCH_LDA>(d, a, stage, rk2, s); break;
      case SCH_B: adj_tris<SCH_B>(d, a, stage, rk2, s); break;
      case SCH_BMAX: adj_tris<SCH_BMAX>(d, a, stage, rk2, s); break;
      default: adj_tris<SCH_BMIN>(d, a, stage, rk2, s); break;
    }
  };
  if (rk2) {
    tris(2);
    hipLaunchKernelGGL(k_adj_gather2, dim3(nblk(d.nv)), dim3(kBlock), 0, s, d, a);
  } else {
    hipLaunchKernelGGL(k_adj_euler_prep, dim3(nblk(d.nv)), dim3(kBlock), 0, s, d, a);
  }
  tris(1);
  hipLaunchKernelGGL(k_adj_gather1, dim3(nblk(d.nv)), dim3(kBlock), 0, s, d, a, rk2, out);
  return hipGetLastError();
}

hipError_t launch_adj_star(const Dev& d, const AdjDev& a, hipStream_t s) {
  if (d.nv == 0) return hipSuccess;
  hipLaunchKernelGGL(k_adj_star, dim3(nblk(d.nv)), dim3(kBlock), 0, s, d, a);
  return hipGetLastError();
}

hipError_t launch_soa_to_aos(const double* soa, D4* dst, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_soa_to_aos, dim3(nblk(n)), dim3(kBlock), 0, s, soa, dst, n);
  return hipGetLastError();
}

template <typename R, int SCHEME, int STAGE, bool SAVE, bool CFL, bool LUMP = false>
static hipError_t tri_launch(const Dev& d, hipStream_t s) {
  hipLaunchKernelGGL((k_tri<R, SCHEME, STAGE, SAVE, CFL, LUMP>), dim3(nblk(d.nt)), dim3(kBlock), 0, s, d);
  return hipGetLastError();
}

template <typename R, int SCHEME>
static hipError_t tri_dispatch(const Dev& d, int stage, bool save, bool cfl, hipStream_t s) {
  if (stage == 1 && save && cfl) return tri_launch<R, SCHEME, 1, true, true>(d, s);
  if (stage == 1 && save) return tri_launch<R, SCHEME, 1, true, false>(d, s);
  if (stage == 1 && cfl) return tri_launch<R, SCHEME, 1, false, true>(d, s);
  if (stage == 1) return tri_launch<R, SCHEME, 1, false, false>(d, s);
  if (d.slump) return tri_launch<R, SCHEME, 2, false, false, true>(d, s);
  return tri_launch<R, SCHEME, 2, false, false>(d, s);
}

template <typename R>
static hipError_t tri_scheme(const Dev& d, int scheme, int stage, bool save, bool cfl, hipStream_t s) {
  switch (scheme) {
    case SCH_N: return tri_dispatch<R, SCH_N>(d, stage, save, cfl, s);
    case SCH_LDA: return tri_dispatch<R, SCH_LDA>(d, stage, save, cfl, s);
    case SCH_B: return tri_dispatch<R, SCH_B>(d, stage, save, cfl, s);
    case SCH_BMAX: return tri_dispatch<R, SCH_BMAX>(d, stage, save, cfl, s);
    case SCH_BMIN: return tri_dispatch<R, SCH_BMIN>(d, stage, save, cfl, s);
    case SCH_BX: return tri_dispatch<R, SCH_BX>(d, stage, save, cfl, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_tri(const Dev& d, int fp32, int scheme, int stage, bool save, bool cfl, hipStream_t s) {
  if (d.nt == 0) return hipSuccess;
  return fp32 ? tri_scheme<float>(d, scheme, stage, save, cfl, s)
              : tri_scheme<double>(d, scheme, stage, save, cfl, s);
}

template <typename R>
static hipError_t gather_mode(const Dev& d, int mode, double* out, hipStream_t s) {
  const dim3 g(nblk(d.nv)), b(kBlock);
  switch (mode) {
    case G_EULER: hipLaunchKernelGGL((k_gather<R, G_EULER>), g, b, 0, s, d, out); break;
    case G_STAGE1: hipLaunchKernelGGL((k_gather<R, G_STAGE1>), g, b, 0, s, d, out); break;
    case G_STAGE2: hipLaunchKernelGGL((k_gather<R, G_STAGE2>), g, b, 0, s, d, out); break;
    case G_RESIDUAL: hipLaunchKernelGGL((k_gather<R, G_RESIDUAL>), g, b, 0, s, d, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_gather(const Dev& d, int fp32, int mode, double* out_soa, hipStream_t s) {
  if (d.nv == 0) return hipSuccess;
  return fp32 ? gather_mode<float>(d, mode, out_soa, s) : gather_mode<double>(d, mode, out_soa, s);
}

hipError_t launch_wall(const Dev& d, bool stage2, hipStream_t s, bool tiled) {
  if (d.nwv == 0) return hipSuccess;
  if (stage2 && tiled) hipLaunchKernelGGL((k_wall<true, true>), dim3(nblk(d.nwv)), dim3(kBlock), 0, s, d);
  else if (stage2) hipLaunchKernelGGL((k_wall<true, false>), dim3(nblk(d.nwv)), dim3(kBlock), 0, s, d);
  else hipLaunchKernelGGL((k_wall<false, false>), dim3(nblk(d.nwv)), dim3(kBlock), 0, s, d);
  return hipGetLastError();
}

hipError_t launch_cfl_part(const Dev& d, const CflPlan& p, double cfl, int part, hipStream_t s, int fp32) {
  if (part == 0) hipLaunchKernelGGL(k_cfl_tri, dim3(nblk(d.nt)), dim3(kBlock), 0, s, d);
  else if (part == 1 && fp32) hipLaunchKernelGGL((k_cfl_vertex<false, float>), dim3(p.nblocks), dim3(kBlock), 0, s, d, p);
  else if (part == 1) hipLaunchKernelGGL((k_cfl_vertex<false, double>), dim3(p.nblocks), dim3(kBlock), 0, s, d, p);
  else if (part == 3) hipLaunchKernelGGL((k_cfl_vertex<true, double>), dim3(p.nblocks), dim3(kBlock), 0, s, d, p);
  else hipLaunchKernelGGL(k_cfl_final, dim3(p.nmesh), dim3(kBlock), 0, s, d, p, cfl);
  return hipGetLastError();
}

hipError_t launch_vrange(const Dev& d, const CflPlan& p, int mode, hipStream_t s) {
  if (p.nblocks == 0) return hipSuccess;
  if (mode == 0) hipLaunchKernelGGL(k_vrange<0>, dim3(p.nblocks), dim3(kBlock), 0, s, d, p);
  else if (mode == 1) hipLaunchKernelGGL(k_vrange<1>, dim3(p.nblocks), dim3(kBlock), 0, s, d, p);
  else if (mode == 2) hipLaunchKernelGGL(k_vrange<2>, dim3(p.nblocks), dim3(kBlock), 0, s, d, p);
  else return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_vrange_final, dim3(p.nmesh), dim3(kBlock), 0, s, d, p);
  return hipGetLastError();
}

hipError_t launch_cfl(const Dev& d, const CflPlan& p, double cfl, hipStream_t s) {
  for (int part = 0; part < 3; ++part) {
    hipError_t e = launch_cfl_part(d, p, cfl, part, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_set_state(const Dev& d, const double* soa, int fp32, hipStream_t s) {
  hipLaunchKernelGGL(k_set_state, dim3(nblk(d.nv)), dim3(kBlock), 0, s, d, soa, fp32);
  return hipGetLastError();
}

hipError_t launch_refresh(const Dev& d, int fp32, hipStream_t s) {
  hipLaunchKernelGGL(k_refresh, dim3(nblk(d.nv)), dim3(kBlock), 0, s, d, fp32);
  return hipGetLastError();
}

hipError_t launch_get_state(const Dev& d, const D4* src, double* soa, hipStream_t s) {
  hipLaunchKernelGGL(k_aos_to_soa, dim3(nblk(d.nv)), dim3(kBlock), 0, s, src, soa, d.nv);
  return hipGetLastError();
}

hipError_t launch_aos_to_soa(const D4* src, double* soa, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_aos_to_soa, dim3(nblk(n)), dim3(kBlock), 0, s, src, soa, n);
  return hipGetLastError();
}

hipError_t launch_keep_to_soa(const void* keep, double* soa, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_keep_to_soa, dim3(nblk(n)), dim3(kBlock), 0, s, static_cast<const double2*>(keep), soa, n);
  return hipGetLastError();
}

hipError_t launch_set_scalar(double* p, double v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(1), 0, s, p, v);
  return hipGetLastError();
}

hipError_t launch_set_int(int* p, int v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, p, v);
  return hipGetLastError();
}

hipError_t launch_fill_int(int* p, int v, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_int, dim3(nblk(n)), dim3(kBlock), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_or_int(int* dst, const int* src, hipStream_t s) {
  hipLaunchKernelGGL(k_or_int, dim3(1), dim3(1), 0, s, dst, src);
  return hipGetLastError();
}

hipError_t launch_copy4(D4* dst, const D4* src, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy4, dim3(nblk(n)), dim3(kBlock), 0, s, dst, src, n);
  return hipGetLastError();
}

}  // namespace rd
