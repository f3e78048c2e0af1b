// gfx950 kernels of the three-dimensional path (bodies in rd3_device.h):
// the per-vertex parameter vector, the per-tetrahedron distribution (stage 1
// or Euler, stage 2), the per-vertex sums in a fixed order (no float
// atomics) with the update, and the CFL limit (per-corner parts summed per
// vertex, then a two-level minimum). One step = Z -> tetrahedra -> vertices
// (-> tetrahedra -> vertices for RK2); the time step is read on the device.
#include "rd3_launch.h"

namespace rd3 {

__global__ __launch_bounds__(kBlock) void k3_z(Dev3 d, const double* src) {
  const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (v >= d.nv) return;
  double w[5], z[5], sg;
  for (int k = 0; k < 5; ++k) w[k] = src[k * d.nv + v];
  if (!to_z(w, d.gamma, z, sg)) d.flag[0] = 1;
  for (int k = 0; k < 5; ++k) d.Z[k * d.nv + v] = z[k];
  d.sig[v] = sg;
}

// At most 256 registers per lane (two waves per SIMD): the second stage's
// extra terms would otherwise take it just past that, to one wave.
template <int STAGE, int SCHEME>
__global__ __launch_bounds__(kBlock, 2) void k3_tet(Dev3 d, int keep) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t < d.nt) tet_body<STAGE, SCHEME>(d, t, keep != 0);
}

// mode 0: Euler (W <- W - dt/V R, then Z, sig of W); 1: first stage
// (Ws <- W - dt/V R, then Z of Ws); 2: second stage (W <- Ws - dt/V R, then
// Z, sig of W).
template <int MODE>
__global__ __launch_bounds__(kBlock) void k3_gather(Dev3 d) {
  const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (v >= d.nv) return;
  const int64_t nv = d.nv;
  double r[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const int64_t first = d.sbase[v >> 6] + (v & 63);
  const int32_t n = d.deg[v];
  // J ranks of parts loaded before any is summed (slot order kept; ranks
  // past the degree reload its last rank and are left out of the sums)
  constexpr int J = 4;
  for (int32_t j0 = 0; j0 < n; j0 += J) {
    double x[J][5];
    for (int u = 0; u < J; ++u) {
      const int64_t q = first + 64 * (int64_t)(j0 + u < n ? j0 + u : n - 1);
      for (int k = 0; k < 5; ++k) x[u][k] = d.part[k * d.ns + q];
    }
    for (int u = 0; u < J; ++u)
      for (int k = 0; k < 5; ++k) r[k] = j0 + u < n ? r[k] + x[u][k] : r[k];
  }
  const double f = *d.dt / d.V[v];
  const double* src = MODE == 2 ? d.Ws : d.W;
  double* dst = MODE == 1 ? d.Ws : d.W;
  double w[5], z[5], sg;
  const double idt = 1.0 / *d.dt;
  for (int k = 0; k < 5; ++k) {
    const double old = src[k * nv + v];
    w[k] = old - f * r[k];
    dst[k * nv + v] = w[k];
    if (MODE == 1) d.rate[k * nv + v] = (w[k] - old) * idt;  // read by the second tetrahedron pass
  }
  if (!to_z(w, d.gamma, z, sg)) d.flag[0] = 1;
  for (int k = 0; k < 5; ++k) d.Z[k * nv + v] = z[k];
  if (MODE != 1) d.sig[v] = sg;
}

// CFL parts: S_T lambda_T at each corner's slot (lambda_T the largest
// |u| + c at the corners).
__global__ __launch_bounds__(kBlock) void k3_cfl_tet(Dev3 d) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= d.nt) return;
  double lam = 0.0;
  for (int i = 0; i < 4; ++i) lam = fmax(lam, d.sig[d.tet[i * d.nt + t]]);
  const double c = d.smax[t] * lam;
  for (int i = 0; i < 4; ++i) d.cpart[d.slot[i * d.nt + t]] = c;
}

// Per vertex 3 V / sum of its parts; block minima.
__global__ __launch_bounds__(kBlock) void k3_cfl_vertex(Dev3 d) {
  __shared__ double red[kBlock];
  const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double best = INFINITY;
  if (v < d.nv) {
    // The parts are loaded J at a time before any of them is summed (in
    // slot order, as one sequential sum), so that a thread keeps J loads in
    // flight; ranks past the degree reload its last rank (every vertex has
    // a tetrahedron) and are left out of the sum.
    constexpr int J = 8;
    double acc = 0.0;
    const int64_t base = d.sbase[v >> 6] + (v & 63);
    const int32_t n = d.deg[v];
    const double vol = d.V[v];
    for (int32_t j0 = 0; j0 < n; j0 += J) {
      double x[J];
      for (int u = 0; u < J; ++u) x[u] = d.cpart[base + 64 * (int64_t)(j0 + u < n ? j0 + u : n - 1)];
      for (int u = 0; u < J; ++u) acc = j0 + u < n ? acc + x[u] : acc;
    }
    best = 3.0 * vol / acc;
  }
  red[threadIdx.x] = best;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) d.bmin[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kBlock) void k3_cfl_final(Dev3 d, int nblocks, double cfl) {
  __shared__ double red[kBlock];
  double best = INFINITY;
  for (int b = threadIdx.x; b < nblocks; b += kBlock) best = fmin(best, d.bmin[b]);
  red[threadIdx.x] = best;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *d.dt = cfl * red[0];
}

__global__ void k3_set(double* p, double v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

static unsigned blocks(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

hipError_t launch3_z(const Dev3& d, const double* src, hipStream_t s) {
  hipLaunchKernelGGL(k3_z, dim3(blocks(d.nv)), dim3(kBlock), 0, s, d, src);
  return hipGetLastError();
}

template <int SCHEME>
static void tet_launch(const Dev3& d, int stage, bool keep, hipStream_t s) {
  if (stage == 1)
    hipLaunchKernelGGL((k3_tet<1, SCHEME>), dim3(blocks(d.nt)), dim3(kBlock), 0, s, d, keep ? 1 : 0);
  else
    hipLaunchKernelGGL((k3_tet<2, SCHEME>), dim3(blocks(d.nt)), dim3(kBlock), 0, s, d, 0);
}

hipError_t launch3_tet(const Dev3& d, int stage, int scheme, bool keep, hipStream_t s) {
  switch (scheme) {
    case S_N: tet_launch<S_N>(d, stage, keep, s); break;
    case S_LDA: tet_launch<S_LDA>(d, stage, keep, s); break;
    case S_B: tet_launch<S_B>(d, stage, keep, s); break;
    case S_BMAX: tet_launch<S_BMAX>(d, stage, keep, s); break;
    case S_BMIN: tet_launch<S_BMIN>(d, stage, keep, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch3_gather(const Dev3& d, int mode, hipStream_t s) {
  if (mode == 0)
    hipLaunchKernelGGL(k3_gather<0>, dim3(blocks(d.nv)), dim3(kBlock), 0, s, d);
  else if (mode == 1)
    hipLaunchKernelGGL(k3_gather<1>, dim3(blocks(d.nv)), dim3(kBlock), 0, s, d);
  else
    hipLaunchKernelGGL(k3_gather<2>, dim3(blocks(d.nv)), dim3(kBlock), 0, s, d);
  return hipGetLastError();
}

int cfl_blocks(int64_t nv) { return (int)blocks(nv); }

hipError_t launch3_cfl(const Dev3& d, double cfl, hipStream_t s) {
  hipLaunchKernelGGL(k3_cfl_tet, dim3(blocks(d.nt)), dim3(kBlock), 0, s, d);
  hipLaunchKernelGGL(k3_cfl_vertex, dim3(blocks(d.nv)), dim3(kBlock), 0, s, d);
  hipLaunchKernelGGL(k3_cfl_final, dim3(1), dim3(kBlock), 0, s, d, (int)blocks(d.nv), cfl);
  return hipGetLastError();
}

hipError_t launch3_set_dt(const Dev3& d, double dt, hipStream_t s) {
  hipLaunchKernelGGL(k3_set, dim3(1), dim3(64), 0, s, d.dt, dt);
  return hipGetLastError();
}

}  // namespace rd3
