// Device peaks the trace kernel's rooflines are priced against, measured on
// the device itself (a separate library, not part of the tracer's ABI):
//
//   * float64 atomic adds scattered over a 256^3 float64 array (every lane a
//     hashed cell), the pattern of evicted deposit sums;
//   * the same with spatially coherent lanes (64 neighbouring cells per wave);
//   * a streaming device-to-device copy (HBM read + write).
//
//   int moray_microbench(int device, double* out);
//     out[0] scattered float64 atomics per second, out[1] coherent float64
//     atomics per second, out[2] copy bandwidth in GB/s (bytes read + written).
//     Returns 0, or a HIP error code; allocates and frees its own buffers.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

__device__ __forceinline__ unsigned mix32(unsigned x) {
  x ^= x >> 16;
  x *= 0x7feb352dU;
  x ^= x >> 15;
  x *= 0x846ca68bU;
  x ^= x >> 16;
  return x;
}

__global__ void atomics_scattered(double* acc, unsigned mask, int iters) {
  const unsigned tid = blockIdx.x * blockDim.x + threadIdx.x;
  for (int k = 0; k < iters; ++k) unsafeAtomicAdd(&acc[mix32(tid * 2654435761u + (unsigned)k * 40503u) & mask], 1.0);
}

__global__ void atomics_coherent(double* acc, unsigned mask, int iters) {
  const unsigned tid = blockIdx.x * blockDim.x + threadIdx.x;
  const unsigned wave = tid >> 6, lane = tid & 63u;
  for (int k = 0; k < iters; ++k) {
    const unsigned base = mix32(wave * 977u + (unsigned)k * 131u) & mask;
    unsafeAtomicAdd(&acc[(base + lane * 3u) & mask], 1.0);
  }
}

__global__ void zero(double* p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0.0;
}

__global__ void copy(const float4* __restrict__ a, float4* __restrict__ b, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) b[i] = a[i];
}

}  // namespace

extern "C" int moray_microbench(int device, double* out) {
  hipError_t e = hipSetDevice(device);
  int cus = 0;
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  if (e != hipSuccess) return (int)e;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  double* acc = nullptr;
  float4 *a = nullptr, *b = nullptr;
  const unsigned n = 1u << 24;                        // 256^3 cells
  const size_t copy_bytes = (size_t)1 << 30;
  const int blocks = cus * 8, threads = 256, iters = 64;
  const double total = (double)blocks * threads * iters;
  auto timed = [&](int which, float& ms) -> hipError_t {
    for (int rep = 0; rep < 2; ++rep) {             // the second run is timed
      hipError_t r = hipEventRecord(e0, s);
      if (r != hipSuccess) return r;
      if (which == 0) hipLaunchKernelGGL(atomics_scattered, dim3(blocks), dim3(threads), 0, s, acc, n - 1, iters);
      else if (which == 1) hipLaunchKernelGGL(atomics_coherent, dim3(blocks), dim3(threads), 0, s, acc, n - 1, iters);
      else hipLaunchKernelGGL(copy, dim3(cus * 16), dim3(256), 0, s, a, b, copy_bytes / sizeof(float4));
      if ((r = hipGetLastError()) != hipSuccess || (r = hipEventRecord(e1, s)) != hipSuccess ||
          (r = hipEventSynchronize(e1)) != hipSuccess || (r = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess)
        return r;
    }
    return hipSuccess;
  };
  float ms[3] = {0.f, 0.f, 0.f};
  if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) == hipSuccess &&
      (e = hipEventCreate(&e0)) == hipSuccess && (e = hipEventCreate(&e1)) == hipSuccess &&
      (e = hipMalloc(&acc, (size_t)n * sizeof(double))) == hipSuccess &&
      (e = hipMalloc(&a, copy_bytes)) == hipSuccess && (e = hipMalloc(&b, copy_bytes)) == hipSuccess) {
    hipLaunchKernelGGL(zero, dim3(cus * 8), dim3(256), 0, s, acc, (size_t)n);
    hipLaunchKernelGGL(zero, dim3(cus * 8), dim3(256), 0, s, (double*)a, copy_bytes / sizeof(double));
    e = hipGetLastError();
    for (int w = 0; w < 3 && e == hipSuccess; ++w) e = timed(w, ms[w]);
  }
  if (e == hipSuccess) {
    out[0] = total / (ms[0] * 1e-3);
    out[1] = total / (ms[1] * 1e-3);
    out[2] = 2.0 * (double)copy_bytes / (ms[2] * 1e-3) / 1e9;
  }
  if (s) (void)hipStreamSynchronize(s);
  if (acc) (void)hipFree(acc);
  if (a) (void)hipFree(a);
  if (b) (void)hipFree(b);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) (void)hipStreamDestroy(s);
  return (int)e;
}
