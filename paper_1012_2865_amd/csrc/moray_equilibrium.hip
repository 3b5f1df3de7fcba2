// HIP kernels of the photo-ionisation equilibrium iteration around the trace
// (moray_equilibrate): the per-cell update and its helpers.
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

__global__ __launch_bounds__(kEqBlock) void equilibrium_update_kernel(const double* __restrict__ kph,
                                                                      const float* __restrict__ n_h,
                                                                      double* __restrict__ x64,
                                                                      float* __restrict__ x32, long long n,
                                                                      double alpha_b, double w,
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
      if (i < n) {
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
                                     long long n, double alpha_b, double w, double* dx) {
  const int blocks = equilibrium_blocks(n);
  hipLaunchKernelGGL(equilibrium_update_kernel, dim3(blocks), dim3(kEqBlock), 0, s, kph, n_h, x64, x32, n, alpha_b,
                     w, dx + 1);
  hipLaunchKernelGGL(max_partials_kernel, dim3(1), dim3(1024), 0, s, (const double*)(dx + 1), blocks, dx);
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
