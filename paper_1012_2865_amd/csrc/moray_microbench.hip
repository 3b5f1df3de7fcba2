// Device peaks the trace kernel's rooflines are priced against, measured on
// the device itself (a separate library, not part of the tracer's ABI).
//
//   int moray_microbench(int device, double* out);
//     One fixed shape of each pattern, kept for counter calibration (its
//     scattered-atomics dispatch issues exactly 64 float64 atomics per thread
//     of its grid): out[0] scattered float64 atomics per second, out[1]
//     coherent float64 atomics per second, out[2] copy bandwidth in GB/s
//     (bytes read + written). Returns 0, or a HIP error code.
//
//   int moray_microbench_case(int device, int kind, unsigned long long bytes,
//                             int blocks_per_cu, int per_thread, int group,
//                             double* rate);
//     One point of a sweep. kind MB_ATOMICS: float64 atomic adds into an array
//     of `bytes` (a power of two, 1 KiB .. 8 GiB); each thread issues
//     `per_thread` adds (1 .. 4096); lanes come in runs of `group` (a power of
//     two, 1 .. 64) consecutive cells at a hashed base, so group 1 scatters
//     every lane and group 64 gives each wave one contiguous 512-byte run;
//     *rate = atomics per second. kind MB_COPY / MB_COPY_NT: a streaming copy
//     of `bytes` (a multiple of 16, at most 8 GiB) with `per_thread` 16-byte
//     loads in flight per lane (1, 2, 4 or 8), plain or non-temporal loads and
//     stores; *rate = GB/s read + written. kind MB_READ / MB_READ_NT: a
//     streaming sum of `bytes`; *rate = GB/s read. Every case runs on
//     blocks_per_cu (1 .. 64) blocks of 256 threads per compute unit, once to
//     warm up and three times timed; the best of the three is reported.
//     Returns 0, -1 for arguments outside those ranges, or a HIP error code.
//     Allocates and frees its own buffers.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

enum { MB_ATOMICS = 0, MB_COPY = 1, MB_COPY_NT = 2, MB_READ = 3, MB_READ_NT = 4 };

typedef float f4 __attribute__((ext_vector_type(4)));

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

// Runs of 2^gshift consecutive cells at hashed bases (the base is aligned to
// the run, so a run never straddles more lines than it must).
__global__ void atomics_grouped(double* acc, unsigned long long mask, int iters, unsigned gshift) {
  const unsigned tid = blockIdx.x * blockDim.x + threadIdx.x;
  const unsigned g = tid >> gshift, r = tid & ((1u << gshift) - 1u);
  for (int k = 0; k < iters; ++k) {
    const unsigned long long h = ((unsigned long long)mix32(g * 2654435761u + (unsigned)k * 40503u) << 20) ^
                                 (unsigned long long)mix32(g ^ ((unsigned)k << 16));
    unsafeAtomicAdd(&acc[(((h >> gshift) << gshift) | r) & mask], 1.0);
  }
}

__global__ void zero(double* p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0.0;
}

__global__ void copy(const float4* __restrict__ a, float4* __restrict__ b, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) b[i] = a[i];
}

// Each block moves U * 256 consecutive 16-byte words per round: all U loads
// are issued before the first store, so U loads per lane are in flight.
template <int U, bool NT>
__global__ __launch_bounds__(256) void copy_unrolled(const f4* __restrict__ a, f4* __restrict__ b, size_t n) {
  const size_t stride = (size_t)gridDim.x * 256u * U;
  for (size_t base = (size_t)blockIdx.x * 256u * U + threadIdx.x; base < n; base += stride) {
    f4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t i = base + (size_t)u * 256u;
      if (i < n) v[u] = NT ? __builtin_nontemporal_load(&a[i]) : a[i];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t i = base + (size_t)u * 256u;
      if (i < n) {
        if (NT) __builtin_nontemporal_store(v[u], &b[i]);
        else b[i] = v[u];
      }
    }
  }
}

// A streaming sum; the (never taken) store keeps the loads alive.
template <int U, bool NT>
__global__ __launch_bounds__(256) void read_unrolled(const f4* __restrict__ a, size_t n, float* sink) {
  const size_t stride = (size_t)gridDim.x * 256u * U;
  f4 acc = {0.f, 0.f, 0.f, 0.f};
  for (size_t base = (size_t)blockIdx.x * 256u * U + threadIdx.x; base < n; base += stride) {
    f4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t i = base + (size_t)u * 256u;
      v[u] = i < n ? (NT ? __builtin_nontemporal_load(&a[i]) : a[i]) : f4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int u = 0; u < U; ++u) acc += v[u];
  }
  const float s = acc.x + acc.y + acc.z + acc.w;
  if (s == -1.0f) sink[blockIdx.x & 255u] = s;
}

template <bool NT>
hipError_t launch_stream(int kind_copy, int u, int blocks, hipStream_t s, const f4* a, f4* b, size_t n,
                         float* sink) {
  if (kind_copy) {
    switch (u) {
      case 1: hipLaunchKernelGGL((copy_unrolled<1, NT>), dim3(blocks), dim3(256), 0, s, a, b, n); break;
      case 2: hipLaunchKernelGGL((copy_unrolled<2, NT>), dim3(blocks), dim3(256), 0, s, a, b, n); break;
      case 4: hipLaunchKernelGGL((copy_unrolled<4, NT>), dim3(blocks), dim3(256), 0, s, a, b, n); break;
      default: hipLaunchKernelGGL((copy_unrolled<8, NT>), dim3(blocks), dim3(256), 0, s, a, b, n); break;
    }
  } else {
    switch (u) {
      case 1: hipLaunchKernelGGL((read_unrolled<1, NT>), dim3(blocks), dim3(256), 0, s, a, n, sink); break;
      case 2: hipLaunchKernelGGL((read_unrolled<2, NT>), dim3(blocks), dim3(256), 0, s, a, n, sink); break;
      case 4: hipLaunchKernelGGL((read_unrolled<4, NT>), dim3(blocks), dim3(256), 0, s, a, n, sink); break;
      default: hipLaunchKernelGGL((read_unrolled<8, NT>), dim3(blocks), dim3(256), 0, s, a, n, sink); break;
    }
  }
  return hipGetLastError();
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

extern "C" int moray_microbench_case(int device, int kind, unsigned long long bytes, int blocks_per_cu,
                                     int per_thread, int group, double* rate) {
  const unsigned long long kMaxBytes = 1ull << 33;
  if (!rate || kind < MB_ATOMICS || kind > MB_READ_NT || blocks_per_cu < 1 || blocks_per_cu > 64) return -1;
  unsigned gshift = 0;
  if (kind == MB_ATOMICS) {
    if (bytes < 1024 || bytes > kMaxBytes || (bytes & (bytes - 1)) || per_thread < 1 || per_thread > 4096 ||
        group < 1 || group > 64 || (group & (group - 1)))
      return -1;
    while ((1 << gshift) < group) ++gshift;
  } else {
    if (bytes < 16 || bytes > kMaxBytes || (bytes & 15) ||
        (per_thread != 1 && per_thread != 2 && per_thread != 4 && per_thread != 8))
      return -1;
  }
  hipError_t e = hipSetDevice(device);
  int cus = 0;
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  if (e != hipSuccess) return (int)e;
  const int blocks = cus * blocks_per_cu;
  const bool is_copy = kind == MB_COPY || kind == MB_COPY_NT;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  void *a = nullptr, *b = nullptr;
  float best = 0.f;
  if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) == hipSuccess &&
      (e = hipEventCreate(&e0)) == hipSuccess && (e = hipEventCreate(&e1)) == hipSuccess &&
      (e = hipMalloc(&a, bytes)) == hipSuccess &&
      (e = hipMalloc(&b, is_copy ? bytes : (size_t)1024)) == hipSuccess) {
    hipLaunchKernelGGL(zero, dim3(cus * 8), dim3(256), 0, s, (double*)a, (size_t)(bytes / sizeof(double)));
    e = hipGetLastError();
    const size_t words = bytes / 16;
    for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {   // one warm-up, three timed
      if ((e = hipEventRecord(e0, s)) != hipSuccess) break;
      if (kind == MB_ATOMICS) {
        hipLaunchKernelGGL(atomics_grouped, dim3(blocks), dim3(256), 0, s, (double*)a,
                           (unsigned long long)(bytes / sizeof(double) - 1), per_thread, gshift);
        e = hipGetLastError();
      } else if (kind == MB_COPY || kind == MB_READ) {
        e = launch_stream<false>(is_copy, per_thread, blocks, s, (const f4*)a, (f4*)b, words, (float*)b);
      } else {
        e = launch_stream<true>(is_copy, per_thread, blocks, s, (const f4*)a, (f4*)b, words, (float*)b);
      }
      float ms = 0.f;
      if (e != hipSuccess || (e = hipEventRecord(e1, s)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess ||
          (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess)
        break;
      if (rep > 0 && (best == 0.f || ms < best)) best = ms;
    }
  }
  if (e == hipSuccess) {
    const double sec = (double)best * 1e-3;
    if (kind == MB_ATOMICS) *rate = (double)blocks * 256.0 * per_thread / sec;
    else *rate = (is_copy ? 2.0 : 1.0) * (double)bytes / sec / 1e9;
  }
  if (s) (void)hipStreamSynchronize(s);
  if (a) (void)hipFree(a);
  if (b) (void)hipFree(b);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) (void)hipStreamDestroy(s);
  return (int)e;
}
