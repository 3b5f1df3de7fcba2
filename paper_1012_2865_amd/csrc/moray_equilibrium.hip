// HIP kernels of the photo-ionisation equilibrium iteration around the trace
// (moray_equilibrate): the per-cell update and its helpers.
#include "moray_device.h"

#include <hip/hip_runtime.h>
#include <cmath>

namespace moray {

// ---------------------------------------------------------------------------
// Photo-ionisation equilibrium update (section 2.2, Eq. dndt with dn/dt = 0,
// hydrogen only, n_e = n_p = (1 - x) n_H): per cell the root in [0, 1] of
// alpha n (1 - x)^2 = k x, written without cancellation as
// 2a / ((2a + k) + sqrt(k^2 + 4ak)) with a = alpha n (x = 1 where n = 0),
// then the damped step x <- (1 - w) x + w root. The float64 iterate and its
// float32 copy (the field the next trace reads) are both written; the largest
// change of the launch goes to *dxmax (non-negative doubles order like their
// bit patterns, so an integer maximum serves).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void equilibrium_update_kernel(const double* kph, const float* n_h, double* x64,
                                                                 float* x32, long long n, double alpha_b, double w,
                                                                 unsigned long long* dxmax) {
  double dmax = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const double a = alpha_b * (double)n_h[i];
    const double k = kph[i];
    const double root = a > 0.0 ? 2.0 * a / ((2.0 * a + k) + sqrt(k * k + 4.0 * a * k)) : 1.0;
    const double x = x64[i];
    const double xn = (1.0 - w) * x + w * root;
    dmax = fmax(dmax, fabs(xn - x));
    x64[i] = xn;
    x32[i] = (float)xn;
  }
  for (int o = kWave / 2; o > 0; o >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, o));
  __shared__ double wmax[256 / kWave];
  if ((threadIdx.x & (kWave - 1)) == 0) wmax[threadIdx.x / kWave] = dmax;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = wmax[0];
    for (int v = 1; v < (int)(blockDim.x / kWave); ++v) m = fmax(m, wmax[v]);
    atomicMax(dxmax, (unsigned long long)__double_as_longlong(m));
  }
}

__global__ void widen_kernel(const float* x32, double* x64, long long n, unsigned long long* dxmax) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    x64[i] = (double)x32[i];
  if (blockIdx.x == 0 && threadIdx.x == 0) *dxmax = 0ull;
}

__global__ void clear_u64_kernel(unsigned long long* p) { *p = 0ull; }

hipError_t launch_equilibrium_update(hipStream_t s, int num_cu, const double* kph, const float* n_h, double* x64,
                                     float* x32, long long n, double alpha_b, double w, unsigned long long* dxmax) {
  long long blocks = (n + 255) / 256;
  if (blocks > 16LL * num_cu) blocks = 16LL * num_cu;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(clear_u64_kernel, dim3(1), dim3(1), 0, s, dxmax);
  hipLaunchKernelGGL(equilibrium_update_kernel, dim3((unsigned)blocks), dim3(256), 0, s, kph, n_h, x64, x32, n,
                     alpha_b, w, dxmax);
  return hipGetLastError();
}

hipError_t launch_widen(hipStream_t s, int num_cu, const float* x32, double* x64, long long n,
                        unsigned long long* dxmax) {
  long long blocks = (n + 255) / 256;
  if (blocks > 16LL * num_cu) blocks = 16LL * num_cu;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(widen_kernel, dim3((unsigned)blocks), dim3(256), 0, s, x32, x64, n, dxmax);
  return hipGetLastError();
}

}  // namespace moray
