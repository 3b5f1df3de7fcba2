// Kernels that order the rays held between the steps of a time-dependent
// trace (moray_td_step). The rays halt in whatever order the waves reach
// their halting radius, so a wave that resumed them in that order would hold
// 64 unrelated rays whose deposits seldom fall in the same cells. Sorting the
// halt list by (level, tree, pixel) before the next step puts every level's
// rays in one contiguous run, in which neighbouring records are neighbouring
// pixels of one tree, as in the single pass's queues.
#include "moray_device.h"
#include "moray_internal.h"

#include <hip/hip_runtime.h>
#include <rocprim/device/device_radix_sort.hpp>

namespace moray {

__device__ __forceinline__ unsigned long long lane0_u64(unsigned long long v) {
  const unsigned lo = __shfl((unsigned)v, 0), hi = __shfl((unsigned)(v >> 32), 0);
  return ((unsigned long long)hi << 32) | lo;
}

// key = level << (tree_bits + pix_bits) | tree << pix_bits | pixel; value = record index
__global__ __launch_bounds__(256) void td_keys_kernel(const uint32_t* __restrict__ sg,
                                                      const uint64_t* __restrict__ pix,
                                                      const int* __restrict__ lev, unsigned long long n,
                                                      int tree_bits, int pix_bits,
                                                      unsigned long long* __restrict__ keys,
                                                      uint32_t* __restrict__ idx) {
  for (unsigned long long i = blockIdx.x * 256ull + threadIdx.x; i < n; i += (unsigned long long)gridDim.x * 256ull) {
    keys[i] = ((unsigned long long)lev[i] << (tree_bits + pix_bits)) | ((unsigned long long)sg[i] << pix_bits) |
              pix[i];
    idx[i] = (uint32_t)i;
  }
}

// Records [first, first + count) of the sorted order join level queue q
// (counter row `row`): each 64 consecutive records go, with one atomic, to
// the end of one of the nseg segments (a power of two).
__global__ __launch_bounds__(256) void prefill_sorted_kernel(RayQueue pool, const uint32_t* __restrict__ order,
                                                             unsigned long long first, unsigned long long count,
                                                             RayQueue q, unsigned long long seg_cap, int nseg,
                                                             Counters* ctr, int row) {
  const int lane = threadIdx.x & (kWave - 1);
  const unsigned long long waves = (unsigned long long)gridDim.x * (blockDim.x / kWave);
  const unsigned long long wave = blockIdx.x * (unsigned long long)(blockDim.x / kWave) + threadIdx.x / kWave;
  for (unsigned long long w = wave; w * kWave < count; w += waves) {
    const unsigned long long j = w * kWave + lane;
    const unsigned long long live = count - w * kWave;
    const int take = live < (unsigned long long)kWave ? (int)live : kWave;
    const int seg = (int)(w & (unsigned long long)(nseg - 1));
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(&ctr->count[row][seg], (unsigned long long)take);
    base = lane0_u64(base);
    if (lane < take) {
      const unsigned long long pos = base + (unsigned long long)lane;
      if (pos < seg_cap) {
        const uint32_t i = order[first + j];
        const unsigned long long o = (unsigned long long)seg * seg_cap + pos;
        q.pix[o] = pool.pix[i];
        q.sg[o] = pool.sg[i];
        q.r[o] = pool.r[i];
        q.P[o] = pool.P[i];
      } else {
        atomicOr(&ctr->err, kErrOverflow);
      }
    }
  }
}

hipError_t td_sort_temp_bytes(unsigned long long cap, size_t* bytes) {
  *bytes = 0;
  return rocprim::radix_sort_pairs(nullptr, *bytes, (const unsigned long long*)nullptr, (unsigned long long*)nullptr,
                                   (const uint32_t*)nullptr, (uint32_t*)nullptr, cap, 0u, 64u, (hipStream_t)0);
}

hipError_t launch_td_sort(hipStream_t s, int num_cu, const RayQueue& pool, const int* lev, unsigned long long n,
                          int tree_bits, int pix_bits, unsigned long long* keys_in, unsigned long long* keys_out,
                          uint32_t* idx_in, uint32_t* idx_out, void* temp, size_t temp_bytes) {
  if (n == 0) return hipSuccess;
  const int end_bit = 5 + tree_bits + pix_bits;
  size_t need = 0;
  hipError_t e = rocprim::radix_sort_pairs(nullptr, need, (const unsigned long long*)nullptr,
                                           (unsigned long long*)nullptr, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                           n, 0u, (unsigned)end_bit, s);
  if (e != hipSuccess) return e;
  if (need > temp_bytes) return hipErrorInvalidValue;
  unsigned long long blocks = (n + 255) / 256;
  if (blocks > 16ull * (unsigned long long)num_cu) blocks = 16ull * (unsigned long long)num_cu;
  hipLaunchKernelGGL(td_keys_kernel, dim3((unsigned)blocks), dim3(256), 0, s, pool.sg, pool.pix, lev, n, tree_bits,
                     pix_bits, keys_in, idx_in);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  size_t tb = temp_bytes;
  return rocprim::radix_sort_pairs(temp, tb, (const unsigned long long*)keys_in, keys_out, (const uint32_t*)idx_in,
                                   idx_out, n, 0u, (unsigned)end_bit, s);
}

hipError_t launch_prefill_sorted(hipStream_t s, int num_cu, const RayQueue& pool, const uint32_t* order,
                                 unsigned long long first, unsigned long long count, const RayQueue& q,
                                 unsigned long long seg_cap, int nseg, Counters* ctr, int row) {
  if (count == 0) return hipSuccess;
  unsigned long long blocks = (count + 255) / 256;
  if (blocks > 16ull * (unsigned long long)num_cu) blocks = 16ull * (unsigned long long)num_cu;
  hipLaunchKernelGGL(prefill_sorted_kernel, dim3((unsigned)blocks), dim3(256), 0, s, pool, order, first, count, q,
                     seg_cap, nseg, ctr, row);
  return hipGetLastError();
}

}  // namespace moray
