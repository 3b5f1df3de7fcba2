// HIP kernels of the ionisation updates around the trace: the equilibrium
// iteration (moray_equilibrate) and the time-stepped evolution
// (moray_evolve), per-cell updates, the step limit and their reductions.
#include "moray_device.h"
#include "moray_internal.h"

#include <hip/hip_runtime.h>
#include <cmath>

namespace moray {

// ---------------------------------------------------------------------------
// Photo-ionisation equilibrium update (section 2.2, Eq. dndt with dn/dt = 0,
// hydrogen only, n_e = n_p = (1 - x) n_H): per cell the root in [0, 1] of
// alpha n (1 - x)^2 = k x, written without cancellation as
// 2a / ((2a + k) + sqrt(k^2 + 4ak)) with a = alpha n (x = 1 where n = 0),
// then the damped step x <- (1 - w) x + w root. The float64 iterate and its
// float32 copy (the field the next trace reads) are both written.
//
// The pass streams 20 bytes in and 12 out per cell. Each thread loads
// kEqUnroll cells (one grid stride apart, so every load of a wave is one
// coalesced 256- or 512-byte line set) before it computes any, so a wave
// has 3 kEqUnroll loads in flight. The largest change of the pass is
// reduced per block into part[block] (no atomics: thousands of blocks
// updating one address would serialise at the memory side), and one
// block then reduces the partials into dx[0].
// ---------------------------------------------------------------------------
constexpr int kEqBlock = 256;
constexpr int kEqUnroll = 4;

__device__ __forceinline__ double block_max(double m) {
  for (int o = kWave / 2; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  __shared__ double wmax[1024 / kWave];
  if ((threadIdx.x & (kWave - 1)) == 0) wmax[threadIdx.x / kWave] = m;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int v = 1; v < (int)(blockDim.x / kWave); ++v) m = fmax(m, wmax[v]);
  return m;                                   // valid in thread 0
}

// skip (or NULL): cells that keep their x (root cells under a child grid)
__global__ __launch_bounds__(kEqBlock) void equilibrium_update_kernel(const double* __restrict__ kph,
                                                                      const float* __restrict__ n_h,
                                                                      double* __restrict__ x64,
                                                                      float* __restrict__ x32, long long n,
                                                                      double alpha_b, double w,
                                                                      const unsigned char* __restrict__ skip,
                                                                      double* __restrict__ part) {
  const long long stride = (long long)gridDim.x * kEqBlock;
  double dmax = 0.0;
  for (long long base = blockIdx.x * (long long)kEqBlock + threadIdx.x; base < n; base += kEqUnroll * stride) {
    double k[kEqUnroll], x[kEqUnroll];
    float nh[kEqUnroll];
#pragma unroll
    for (int u = 0; u < kEqUnroll; ++u) {
      const long long i = base + u * stride;
      const bool in = i < n;
      k[u] = in ? kph[i] : 0.0;
      x[u] = in ? x64[i] : 0.0;
      nh[u] = in ? n_h[i] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < kEqUnroll; ++u) {
      const long long i = base + u * stride;
      if (i < n && !(skip && skip[i])) {
        const double a = alpha_b * (double)nh[u];
        const double root = a > 0.0 ? 2.0 * a / ((2.0 * a + k[u]) + sqrt(k[u] * k[u] + 4.0 * a * k[u])) : 1.0;
        const double xn = (1.0 - w) * x[u] + w * root;
        dmax = fmax(dmax, fabs(xn - x[u]));
        x64[i] = xn;
        x32[i] = (float)xn;
      }
    }
  }
  dmax = block_max(dmax);
  if (threadIdx.x == 0) part[blockIdx.x] = dmax;
}

__global__ __launch_bounds__(1024) void max_partials_kernel(const double* __restrict__ part, int n,
                                                            double* __restrict__ out) {
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, part[i]);
  m = block_max(m);
  if (threadIdx.x == 0) *out = m;
}

// ---------------------------------------------------------------------------
// Time-stepped evolution (section 3.4.1 for the step, section 2.2 Eq. dndt
// for the update), three passes per step after the trace:
//
// step_limit_kernel: per cell the limit of Eq. dtelec with n_e = (1 - x) n_H
//   and no collisional term, dt_cell = eps / (k + n_e alpha), in cells of the
//   ionisation front (own optical depth sigma_bar n_H x dx above tau_front),
//   dt_max elsewhere and at most dt_max everywhere. 20 bytes read, 8 written.
// smooth_min_kernel: the 3^3 smoothing of that field with binomial weights
//   (1/4, 1/2, 1/4) per axis, normalised by the weight of the neighbours
//   inside the grid (a product of per-axis sums), then its minimum per block.
//   Neighbour offsets are summed in the same (z, y, x) order as a plain
//   triple loop. The 26 neighbour reads of a cell hit the caches: 8 bytes
//   per cell from HBM.
// evolve_update_kernel: with k_ph and a = alpha n_H held over dt, the exact
//   solution of dx/dt = a (1 - x)^2 - k x: u = x - x1 (x1 the root in [0, 1])
//   obeys du/dt = a u^2 - D u with D = sqrt(k^2 + 4ak), so
//   u(dt) = u0 e^{-D dt} / (1 - a u0 g), g = (1 - e^{-D dt}) / D (dt at D = 0);
//   cells without gas keep x. 20 bytes read, 12 written.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_min(double m) {
  for (int o = kWave / 2; o > 0; o >>= 1) m = fmin(m, __shfl_xor(m, o));
  __shared__ double wmin[1024 / kWave];
  if ((threadIdx.x & (kWave - 1)) == 0) wmin[threadIdx.x / kWave] = m;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int v = 1; v < (int)(blockDim.x / kWave); ++v) m = fmin(m, wmin[v]);
  return m;                                   // valid in thread 0
}

__global__ __launch_bounds__(kEqBlock) void step_limit_kernel(const double* __restrict__ kph,
                                                              const float* __restrict__ n_h,
                                                              const double* __restrict__ x64, long long n,
                                                              double alpha_b, double sigma_bar, double dx_cm,
                                                              double eps, double tau_front, double dt_max,
                                                              const unsigned char* __restrict__ skip,
                                                              double* __restrict__ lim) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const double x = x64[i], nh = (double)n_h[i];
    const double rate = kph[i] + (1.0 - x) * nh * alpha_b;
    const bool front = sigma_bar * nh * x * dx_cm > tau_front;
    double v = dt_max;
    if (front && rate > 0.0 && !(skip && skip[i])) v = fmin(eps / rate, dt_max);
    lim[i] = v;
  }
}

__global__ __launch_bounds__(kEqBlock) void smooth_min_kernel(const double* __restrict__ lim, int nx, int ny, int nz,
                                                              double* __restrict__ part) {
  const long long n = (long long)nx * ny * nz;
  double m = __builtin_huge_val();
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n; c += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(c % nx);
    const long long r = c / nx;
    const int j = (int)(r % ny), k = (int)(r / ny);
    double num = 0.0;
    for (int dz = -1; dz <= 1; ++dz) {
      const int z = k + dz;
      if ((unsigned)z >= (unsigned)nz) continue;
      const double wz = dz == 0 ? 0.5 : 0.25;
      for (int dy = -1; dy <= 1; ++dy) {
        const int y = j + dy;
        if ((unsigned)y >= (unsigned)ny) continue;
        const double wzy = wz * (dy == 0 ? 0.5 : 0.25);
        const double* row = lim + ((long long)z * ny + y) * nx;
        for (int dx = -1; dx <= 1; ++dx) {
          const int x = i + dx;
          if ((unsigned)x >= (unsigned)nx) continue;
          num += (wzy * (dx == 0 ? 0.5 : 0.25)) * row[x];
        }
      }
    }
    const double sx = 0.5 + (i > 0 ? 0.25 : 0.0) + (i + 1 < nx ? 0.25 : 0.0);
    const double sy = 0.5 + (j > 0 ? 0.25 : 0.0) + (j + 1 < ny ? 0.25 : 0.0);
    const double sz = 0.5 + (k > 0 ? 0.25 : 0.0) + (k + 1 < nz ? 0.25 : 0.0);
    m = fmin(m, num / (sz * sy * sx));
  }
  m = block_min(m);
  if (threadIdx.x == 0) part[blockIdx.x] = m;
}

__global__ __launch_bounds__(1024) void min_partials_kernel(const double* __restrict__ part, int n,
                                                            double* __restrict__ out) {
  double m = __builtin_huge_val();
  for (int i = threadIdx.x; i < n; i += blockDim.x) m = fmin(m, part[i]);
  m = block_min(m);
  if (threadIdx.x == 0) *out = m;
}

__global__ __launch_bounds__(kEqBlock) void evolve_update_kernel(const double* __restrict__ kph,
                                                                 const float* __restrict__ n_h,
                                                                 double* __restrict__ x64, float* __restrict__ x32,
                                                                 long long n, double alpha_b, double dt,
                                                                 const unsigned char* __restrict__ skip) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const double a = alpha_b * (double)n_h[i];
    const double k = kph[i];
    const double x0 = x64[i];
    double x = x0;
    if (a > 0.0 && !(skip && skip[i])) {
      const double d = sqrt(k * k + 4.0 * a * k);
      const double x1 = 2.0 * a / ((2.0 * a + k) + d);
      const double g = d > 0.0 ? -expm1(-d * dt) / d : dt;
      const double u0 = x0 - x1;
      x = fmin(fmax(x1 + u0 * exp(-d * dt) / (1.0 - a * u0 * g), 0.0), 1.0);
    }
    x64[i] = x;
    x32[i] = (float)x;
  }
}

__global__ void widen_kernel(const float* __restrict__ x32, double* __restrict__ x64, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    x64[i] = (double)x32[i];
}

static int equilibrium_blocks(long long n) {
  const long long per = (long long)kEqBlock * kEqUnroll;
  const long long b = (n + per - 1) / per;
  return (int)(b < 1 ? 1 : (b > kEqMaxBlocks ? kEqMaxBlocks : b));
}

hipError_t launch_equilibrium_update(hipStream_t s, const double* kph, const float* n_h, double* x64, float* x32,
                                     long long n, double alpha_b, double w, const unsigned char* skip, double* dx) {
  const int blocks = equilibrium_blocks(n);
  hipLaunchKernelGGL(equilibrium_update_kernel, dim3(blocks), dim3(kEqBlock), 0, s, kph, n_h, x64, x32, n, alpha_b,
                     w, skip, dx + 1);
  hipLaunchKernelGGL(max_partials_kernel, dim3(1), dim3(1024), 0, s, (const double*)(dx + 1), blocks, dx);
  return hipGetLastError();
}

static int grid_blocks(int num_cu, long long n) {
  long long blocks = (n + kEqBlock - 1) / kEqBlock;
  if (blocks > 16LL * num_cu) blocks = 16LL * num_cu;
  if (blocks > kEqMaxBlocks) blocks = kEqMaxBlocks;
  return (int)(blocks < 1 ? 1 : blocks);
}

hipError_t launch_step_limit(hipStream_t s, int num_cu, const double* kph, const float* n_h, const double* x64,
                             int nx, int ny, int nz, double alpha_b, double sigma_bar, double dx_cm, double eps,
                             double tau_front, double dt_max, const unsigned char* skip, double* lim, double* dmin) {
  const long long n = (long long)nx * ny * nz;
  const int blocks = grid_blocks(num_cu, n);
  hipLaunchKernelGGL(step_limit_kernel, dim3(blocks), dim3(kEqBlock), 0, s, kph, n_h, x64, n, alpha_b, sigma_bar,
                     dx_cm, eps, tau_front, dt_max, skip, lim);
  hipLaunchKernelGGL(smooth_min_kernel, dim3(blocks), dim3(kEqBlock), 0, s, (const double*)lim, nx, ny, nz, dmin + 1);
  hipLaunchKernelGGL(min_partials_kernel, dim3(1), dim3(1024), 0, s, (const double*)(dmin + 1), blocks, dmin);
  return hipGetLastError();
}

hipError_t launch_evolve_update(hipStream_t s, int num_cu, const double* kph, const float* n_h, double* x64,
                                float* x32, long long n, double alpha_b, double dt, const unsigned char* skip) {
  hipLaunchKernelGGL(evolve_update_kernel, dim3(grid_blocks(num_cu, n)), dim3(kEqBlock), 0, s, kph, n_h, x64, x32, n,
                     alpha_b, dt, skip);
  return hipGetLastError();
}

hipError_t launch_widen(hipStream_t s, int num_cu, const float* x32, double* x64, long long n) {
  long long blocks = (n + 255) / 256;
  if (blocks > 16LL * num_cu) blocks = 16LL * num_cu;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(widen_kernel, dim3((unsigned)blocks), dim3(256), 0, s, x32, x64, n);
  return hipGetLastError();
}

}  // namespace moray
