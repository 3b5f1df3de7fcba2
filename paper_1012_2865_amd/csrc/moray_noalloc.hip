// The library's fixed scratch array for moray_trace_noalloc (include/moray.h):
// callers that cannot allocate device memory (code under graph capture,
// tight serving loops) get every scratch buffer of a trace carved from this
// file-scope array instead of from hipMalloc. The array lives in the loaded
// code object, so each GPU the library runs on holds its own copy for the
// life of the process. Host code must not use the array's name as a device
// address: its address on a device comes from hipGetSymbolAddress, taken
// once per device (at moray_init, with that device current) and kept here.
#include "moray_internal.h"

#include <hip/hip_runtime.h>

#include <mutex>

namespace {

constexpr size_t kScratchBytes = size_t(256) << 20;     // 256 MiB per device
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};
hipError_t g_err[kMaxDevices] = {};
bool g_done[kMaxDevices] = {};

}  // namespace

namespace moray {

size_t scratch_bytes() { return kScratchBytes; }

// The array's device address on `device`, which must be the current device.
// Looked up once per device; later calls return the kept address (or the
// error of the lookup).
hipError_t scratch_address(int device, void** ptr) {
  *ptr = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_done[device]) {
    void* p = nullptr;
    g_err[device] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_ptr[device] = g_err[device] == hipSuccess ? p : nullptr;
    g_done[device] = true;
  }
  *ptr = g_ptr[device];
  return g_err[device];
}

}  // namespace moray
