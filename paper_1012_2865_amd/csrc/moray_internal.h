// Host-side internals shared by the one-shot runtime (moray_runtime.cpp) and
// the serving engine (moray_serve.cpp). Not part of the public ABI.
#pragma once
#include "moray.h"
#include "moray_device.h"

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

namespace moray {

// ---- kernel launchers (moray_kernels.hip) ----
hipError_t launch_reset(hipStream_t, Counters*, SgStats*, int);
hipError_t launch_reset_levels(hipStream_t, Counters*);
hipError_t launch_reset_generation(hipStream_t, Counters*, int cin, int cout);
hipError_t launch_reset_stats(hipStream_t, SgStats*, int first, int count);
// mark: the optically-thin marks the prep pass clears (NULL: none);
// kappa64: where it also writes the columns in float64 (NULL: nowhere)
template <typename R>
hipError_t launch_prep(hipStream_t, int, const GridDev*, int, int, const ProblemDev*, long long, long long, R*, double*,
                       Counters*, uint8_t* mark = nullptr, double* kappa64 = nullptr);
template <typename R>
hipError_t launch_trace_level(hipStream_t, int, const TraceArgs<R>&, bool cache, bool cover, bool radp,
                              bool thin = false);
template <typename R>
hipError_t launch_trace_level_halt(hipStream_t, int, const TraceArgs<R>&, bool cache);
hipError_t launch_prefill_level(hipStream_t, int num_cu, const RayQueue& pool, const int* pool_lev,
                                unsigned long long n_pool, int level, const RayQueue& q, unsigned long long seg_cap,
                                int nseg, Counters* ctr, int row);
// Serving: empty the queued rays (counter row `row`, nseg segments) whose
// tree index lies in one of the n ranges [lo[i], hi[i]) (n <= kDropRanges).
hipError_t launch_drop_trees(hipStream_t, uint32_t* sg, const Counters* ctr, int row, unsigned long long seg_cap,
                             int nseg, const int* lo, const int* hi, int n);
hipError_t launch_sum_blocks(hipStream_t, int blocks, const double* v, unsigned long long n, double* part);
// moray_td_kernels.hip: the halt list sorted by (level, tree, pixel), and its per-level runs as queue input
hipError_t td_sort_temp_bytes(unsigned long long cap, size_t* bytes);
hipError_t launch_td_sort(hipStream_t, int num_cu, const RayQueue& pool, const int* lev, unsigned long long n,
                          int tree_bits, int pix_bits, unsigned long long* keys_in, unsigned long long* keys_out,
                          uint32_t* idx_in, uint32_t* idx_out, void* temp, size_t temp_bytes);
hipError_t launch_prefill_sorted(hipStream_t, int num_cu, const RayQueue& pool, const uint32_t* order,
                                 unsigned long long first, unsigned long long count, const RayQueue& q,
                                 unsigned long long seg_cap, int nseg, Counters* ctr, int row);
// sgs, mark: the tree table and the optically-thin marks (NULL when no problem uses them)
hipError_t launch_finalize(hipStream_t, int, const GridDev*, const ProblemDev*, const FinalBlock*, const double*,
                           const double*, double*, const Counters*, const SgDev* sgs = nullptr,
                           const uint8_t* mark = nullptr);
hipError_t trace_occupancy(int precision, bool cache, int* blocks_per_cu);
// photo-ionisation equilibrium (moray_equilibrium.hip)
// dx: 1 + kEqMaxBlocks doubles; dx[0] receives the largest change of the pass
constexpr int kEqMaxBlocks = 2048;
hipError_t launch_equilibrium_update(hipStream_t, const double* kph, const float* n_h, double* x64, float* x32,
                                     long long n, double alpha_b, double w, const unsigned char* skip, double* dx);
hipError_t launch_widen(hipStream_t, int num_cu, const float* x32, double* x64, long long n);
// moray_evolve: lim receives the per-cell limits, dmin (1 + kEqMaxBlocks doubles) their smoothed minimum in dmin[0]
hipError_t launch_step_limit(hipStream_t, int num_cu, const double* kph, const float* n_h, const double* x64, int nx,
                             int ny, int nz, double alpha_b, double sigma_bar, double dx_cm, double eps,
                             double tau_front, double dt_max, const unsigned char* skip, double* lim, double* dmin);
hipError_t launch_evolve_update(hipStream_t, int num_cu, const double* kph, const float* n_h, double* x64, float* x32,
                                long long n, double alpha_b, double dt, const unsigned char* skip);

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

// moray_noalloc.hip: the fixed scratch array of moray_trace_noalloc and its
// address on a device (looked up once per device, with that device current)
size_t scratch_bytes();
hipError_t scratch_address(int device, void** ptr);

struct Engine;     // serving engine of a context (moray_serve.cpp)
struct PlanHost;   // last one-shot solve and its captured launch sequence (moray_runtime.cpp)

}  // namespace moray

struct moray_ctx {
  int device = 0;
  int precision = MORAY_FP32_ACC64;
  hipStream_t stream = nullptr;
  size_t budget = 0;
  size_t queue_cap_user = 0;
  int waves_per_cu = 0, refill = 0, chunk = 0, profile = 0;
  int reserve_user = 0;          // next-level slots a wave reserves at once; 0 = from the queue size
  bool cache = true;
  int num_cu = 0;
  int blocks_per_cu = 1;
  std::string err = "no error";
  // moray_trace_noalloc: the device address of the library's fixed scratch
  // array on this context's device (null if its lookup failed: scratch_err),
  // and while such a call runs, the part of it the call has carved so far
  char* scratch = nullptr;
  std::string scratch_err;
  bool arena = false;
  size_t arena_used = 0;
  bool fail_capture_once = false;  // test hook (MORAY_INJECT_CAPTURE_FAILURE=1 at moray_init): the next capture
                                   // of a launch sequence fails as if HIP had refused it
  bool overflow_serve_once = false;  // test hook (MORAY_INJECT_SERVE_OVERFLOW=1 at moray_init): the serving
                                     // engine's first launch with two or more problems reports a queue overflow
  size_t allocated = 0;
  moray::DevBuf grids, probs, sgs, stats, ctr, kappa, kappa64, acc, mark, eexc, fblocks, partial, fields, outs;
  moray::DevBuf q_pix[2], q_sg[2], q_r[2], q_P[2];
  size_t q_cap = 0;
  void* h_stage = nullptr;
  size_t h_stage_bytes = 0;
  std::vector<hipEvent_t> evs;
  moray::Engine* engine = nullptr;
  moray::PlanHost* plan = nullptr;
  hipStream_t gstream = nullptr;   // stream of captured launch sequences
  hipEvent_t gev = nullptr;
  moray::DevBuf eq_x, eq_kph, eq_heat, eq_dx;   // moray_equilibrate / moray_evolve: float64 iterate, rates,
                                                 // reduction partials
  moray::DevBuf ev_lim;                          // moray_evolve: per-cell step limits
  moray::DevBuf eq_skip;                         // both: root cells under a child grid (1) or not (0)
};

namespace moray {

moray_status fail(moray_ctx* c, moray_status s, const std::string& msg);
bool hip_ok(moray_ctx* c, hipError_t e, const char* what);
void release(moray_ctx* c, DevBuf& b);
moray_status ensure(moray_ctx* c, DevBuf& b, size_t bytes, const char* what);
moray_status validate(moray_ctx* c, const moray_problem& P, int pi);
int reach_level(const moray_problem& P);
double level_rays_bound(const moray_problem& P);

// Segments of a level queue of `cap` slots: a power of two up to kSegMax, so
// the trace kernel splits a launch's seeds among them with shifts.
inline int queue_segments(size_t cap) {
  int n = 1;
  while (n < kSegMax && (size_t)(2 * n) * 65536 <= cap) n *= 2;
  return n;
}

// serving engine (moray_serve.cpp)
bool engine_busy(moray_ctx* c);
void engine_stop(moray_ctx* c);

constexpr double kEvErgConst = 1.602176634e-12;
constexpr double kPiConst = 3.14159265358979323846;

}  // namespace moray
