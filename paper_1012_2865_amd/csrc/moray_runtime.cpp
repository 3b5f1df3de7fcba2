// Host runtime of the adaptive ray tracer: the C ABI declared in moray.h.
//
// A call validates the problems on the host, lays every problem of the batch
// out in one cell numbering (grid, problem and (source, group) tables), sizes
// the ping-pong ray queue from a geometric bound on the rays one HEALPix level
// can hold, and enqueues reset -> prep -> trace_level(l0..l_reach) -> finalize
// on the context's stream. Trees whose queue estimate exceeds the capacity
// are traced in chunks sharing the same accumulators; a device overflow flag
// triggers a retry with smaller chunks.
#include "moray_internal.h"

#include <algorithm>
#include <cfloat>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

using namespace moray;

namespace {

struct ChunkPlan {
  int sg_begin, sg_end;
};

// (source, group) tree of a one-shot solve: its seed level, problem, source and group.
struct SgKey {
  int l0, prob, src, grp;
};

}  // namespace

// What a one-shot solve needs to turn the staged counters into results, kept
// with the launch sequence captured for the same descriptors.
struct moray::PlanHost {
  std::string key;                  // descriptors, settings and buffer pointers of the solve
  std::vector<SgKey> keys;
  std::vector<int> fblock_first;
  int n_sg = 0;
  size_t nfb = 0;
  int nseg = 1;
  unsigned long long seg_cap = 0;
  int launches = 0;
  bool valid = false;               // the device tables hold this solve
  bool no_graph = false;            // capture failed once: run it directly
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

void drop_graph(PlanHost* ph) {
  if (ph->exec) (void)hipGraphExecDestroy(ph->exec);
  if (ph->graph) (void)hipGraphDestroy(ph->graph);
  ph->exec = nullptr;
  ph->graph = nullptr;
}

template <typename T>
void put(std::string& k, const T& v) {
  k.append(reinterpret_cast<const char*>(&v), sizeof v);
}

// Everything a captured launch sequence depends on: problem descriptors,
// field and output pointers, flags and the context's launch settings.
std::string plan_key(const moray_ctx* c, const moray_problem* probs, int n, unsigned flags, const moray_result* outs) {
  std::string k;
  put(k, n); put(k, flags); put(k, c->precision); put(k, c->chunk); put(k, c->refill); put(k, c->blocks_per_cu);
  put(k, c->cache); put(k, c->reserve_user); put(k, c->queue_cap_user);
  for (int i = 0; i < n; ++i) {
    const moray_problem& P = probs[i];
    put(k, P.n_grids); put(k, P.n_sources); put(k, P.params);
    for (int q = 0; q < P.n_grids; ++q) {
      const moray_grid& G = P.grids[q];
      put(k, G.nx); put(k, G.ny); put(k, G.nz); put(k, G.dx_cm); put(k, G.parent); put(k, G.offset);
      put(k, G.n_h); put(k, G.x_hi);
    }
    for (int j = 0; j < P.n_sources; ++j) put(k, P.sources[j]);
    const moray_spectrum& S = *P.spectrum;
    put(k, S.n_groups); put(k, S.e_ion_ev);
    for (int g = 0; g < S.n_groups; ++g) {
      put(k, S.energy_ev[g]); put(k, S.sigma_cm2[g]); put(k, S.photon_frac[g]);
    }
    put(k, outs[i].k_ph); put(k, outs[i].heating); put(k, outs[i].accel);
  }
  return k;
}

// Results of a finished solve from the pinned staging area.
void collect(moray_ctx* c, const PlanHost& ph, const moray_problem* probs, int n_probs, moray_result* outs,
             double trace_ms) {
  char* hs = (char*)c->h_stage;
  const Counters* hctr = (const Counters*)hs;
  const SgStats* hst = (const SgStats*)(hs + sizeof(Counters));
  const double* hpart = (const double*)(hs + sizeof(Counters) + ph.n_sg * sizeof(SgStats));
  unsigned long long peak = 0;
  for (int l = 0; l < kLevels; ++l) {
    unsigned long long n = 0;
    for (int s = 0; s < ph.nseg; ++s) n += std::min<unsigned long long>(hctr->count[l][s], ph.seg_cap);
    peak = std::max(peak, n);
  }
  for (int i = 0; i < n_probs; ++i) {
    moray_result& R = outs[i];
    R.emitted = R.absorbed = R.escaped = R.truncated = 0.0;
    R.segments = R.rays_seeded = R.splits = R.rays_escaped = R.rays_truncated = 0;
    R.thin_segments = 0;
    R.peak_level_rays = peak;
    R.trace_ms = trace_ms;
    R.trace_launches = ph.launches;
    R.t_admit = R.t_done = 0.0;
    R.from_graph = 0;
    for (int b = ph.fblock_first[i]; b < ph.fblock_first[i + 1]; ++b) R.absorbed += hpart[b];
  }
  for (int k = 0; k < ph.n_sg; ++k) {
    const SgKey& K = ph.keys[k];
    moray_result& R = outs[K.prob];
    const moray_problem& P = probs[K.prob];
    const SgStats& S = hst[k];
    R.emitted += P.spectrum->photon_frac[K.grp] * P.sources[K.src].ndot;
    R.escaped += S.esc_P;
    R.truncated += S.trunc_P;
    R.segments += S.segs;
    R.splits += S.splits;
    R.rays_escaped += S.n_esc;
    R.rays_truncated += S.n_trunc;
    R.thin_segments += S.thin_segs;
    R.rays_seeded += (unsigned long long)std::ldexp(12.0, 2 * P.params.level_init);
    if (R.escaped_sg) R.escaped_sg[K.src * P.spectrum->n_groups + K.grp] = S.esc_P;
  }
}

// Replay of the captured launch sequence. Returns MORAY_EQUEUE (and drops the
// plan) when the replay overflowed, so the caller traces afresh.
moray_status replay(moray_ctx* c, PlanHost& ph, const moray_problem* probs, int n_probs, moray_result* outs) {
  if (!hip_ok(c, hipEventRecord(c->gev, c->stream), "event") ||
      !hip_ok(c, hipStreamWaitEvent(c->gstream, c->gev, 0), "event") ||
      !hip_ok(c, hipGraphLaunch(ph.exec, c->gstream), "graph launch") ||
      !hip_ok(c, hipStreamSynchronize(c->gstream), "synchronize"))
    return MORAY_EDEVICE;
  const Counters* hctr = (const Counters*)c->h_stage;
  if (hctr->err & kErrBadInput) return fail(c, MORAY_EINVAL, "a density or neutral fraction is negative, non-finite or x_HI > 1");
  if (hctr->err & kErrInternal) return fail(c, MORAY_EINTERNAL, "a ray exceeded its step bound");
  if (hctr->err & kErrOverflow) {
    drop_graph(&ph);
    ph.valid = false;
    return MORAY_EQUEUE;
  }
  collect(c, ph, probs, n_probs, outs, 0.0);
  for (int i = 0; i < n_probs; ++i) outs[i].from_graph = 1;
  c->err = "no error";
  return MORAY_OK;
}

}  // namespace

namespace moray {

moray_status fail(moray_ctx* c, moray_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

bool hip_ok(moray_ctx* c, hipError_t e, const char* what) {
  if (e == hipSuccess) return true;
  c->err = std::string(what) + ": " + hipGetErrorString(e);
  return false;
}

void release(moray_ctx* c, DevBuf& b) {
  if (b.p) {
    (void)hipFree(b.p);
    c->allocated -= b.bytes;
  }
  b.p = nullptr;
  b.bytes = 0;
}

// Grow-only device buffer inside the context's HBM budget. During a
// moray_trace_noalloc call the buffer is carved from the library's fixed
// scratch array instead (nothing is allocated; too little room is an error).
moray_status ensure(moray_ctx* c, DevBuf& b, size_t bytes, const char* what) {
  if (c->arena) {
    bytes = (bytes + 255) & ~size_t(255);
    if (bytes > scratch_bytes() - c->arena_used)
      return fail(c, MORAY_ENOMEM, std::string("moray_trace_noalloc: the ") + what + " do not fit the library's " +
                                       std::to_string(scratch_bytes() >> 20) + " MiB scratch array (" +
                                       std::to_string(c->arena_used >> 20) + " MiB already in use by this call)");
    b.p = c->scratch + c->arena_used;
    b.bytes = bytes;
    c->arena_used += bytes;
    return MORAY_OK;
  }
  if (bytes <= b.bytes) return MORAY_OK;
  bytes = (bytes + 255) & ~size_t(255);
  if (c->allocated - b.bytes + bytes > c->budget)
    return fail(c, MORAY_ENOMEM, std::string("HBM budget exceeded allocating ") + what);
  release(c, b);
  if (hipMalloc(&b.p, bytes) != hipSuccess) {
    b.p = nullptr;
    return fail(c, MORAY_ENOMEM, std::string("hipMalloc failed for ") + what);
  }
  b.bytes = bytes;
  c->allocated += bytes;
  return MORAY_OK;
}

static bool finite_nonneg(double x) { return std::isfinite(x) && x >= 0.0; }

// Host-side checks of everything except field values (checked on the device).
moray_status validate(moray_ctx* c, const moray_problem& P, int pi) {
  char buf[256];
  auto bad = [&](const char* m) {
    std::snprintf(buf, sizeof buf, "problem %d: %s", pi, m);
    return fail(c, MORAY_EINVAL, buf);
  };
  if (!P.grids || P.n_grids < 1) return bad("needs at least one grid");
  if (!P.spectrum) return bad("spectrum is NULL");
  if (P.n_sources < 0 || (P.n_sources > 0 && !P.sources)) return bad("bad source list");
  const moray_grid& R = P.grids[0];
  if (R.parent != -1) return bad("grid 0 must be the root (parent -1)");
  for (int q = 0; q < P.n_grids; ++q) {
    const moray_grid& G = P.grids[q];
    if (G.nx < 1 || G.ny < 1 || G.nz < 1) return bad("grid dimensions must be positive");
    if (!(G.dx_cm > 0.0) || !std::isfinite(G.dx_cm)) return bad("dx_cm must be positive and finite");
    if (!G.n_h || !G.x_hi) return bad("field pointer is NULL");
    if ((double)G.nx * G.ny * G.nz > 1.0e9) return bad("grid too large");
    if (q > 0) {
      if (G.parent != 0) return bad("only children of the root grid are supported");
      if ((G.nx | G.ny | G.nz) & 1) return bad("child dimensions must be even");
      if (G.dx_cm != 0.5 * R.dx_cm) return bad("child cell width must be half the root's");
      if (G.offset[0] < 0 || G.offset[1] < 0 || G.offset[2] < 0 || G.offset[0] + G.nx / 2 > R.nx ||
          G.offset[1] + G.ny / 2 > R.ny || G.offset[2] + G.nz / 2 > R.nz)
        return bad("child grid not inside the root");
      for (int o = 1; o < q; ++o) {
        const moray_grid& H = P.grids[o];
        bool sep = false;
        const int lo1[3] = {G.offset[0], G.offset[1], G.offset[2]};
        const int hi1[3] = {G.offset[0] + G.nx / 2, G.offset[1] + G.ny / 2, G.offset[2] + G.nz / 2};
        const int lo2[3] = {H.offset[0], H.offset[1], H.offset[2]};
        const int hi2[3] = {H.offset[0] + H.nx / 2, H.offset[1] + H.ny / 2, H.offset[2] + H.nz / 2};
        for (int k = 0; k < 3; ++k) sep = sep || hi1[k] <= lo2[k] || hi2[k] <= lo1[k];
        if (!sep) return bad("child grids overlap");
      }
    }
  }
  for (int s = 0; s < P.n_sources; ++s) {
    const moray_source& S = P.sources[s];
    if (!(S.x >= 0.0 && S.x < R.nx && S.y >= 0.0 && S.y < R.ny && S.z >= 0.0 && S.z < R.nz))
      return bad("source outside the root grid");
    if (!(S.ndot > 0.0) || !std::isfinite(S.ndot)) return bad("source rate must be positive and finite");
  }
  const moray_spectrum& Sp = *P.spectrum;
  if (Sp.n_groups < 1 || !Sp.energy_ev || !Sp.sigma_cm2 || !Sp.photon_frac) return bad("bad spectrum");
  if (!std::isfinite(Sp.e_ion_ev) || Sp.e_ion_ev < 0.0) return bad("bad ionisation energy");
  double fs = 0.0;
  for (int g = 0; g < Sp.n_groups; ++g) {
    if (!finite_nonneg(Sp.sigma_cm2[g]) || !finite_nonneg(Sp.photon_frac[g])) return bad("bad group");
    if (!(Sp.energy_ev[g] >= Sp.e_ion_ev) || !std::isfinite(Sp.energy_ev[g]))
      return bad("group energy below the ionisation energy");
    fs += Sp.photon_frac[g];
  }
  if (std::fabs(fs - 1.0) > 1e-12) return bad("photon fractions must sum to 1");
  const moray_trace_params& T = P.params;
  if (!finite_nonneg(T.phi_c)) return bad("phi_c must be finite and >= 0");
  if (T.level_init < 0 || T.level_init > T.level_max || T.level_max > kMaxLevel)
    return bad("need 0 <= level_init <= level_max <= 29");
  if (!(T.p_min_frac >= 0.0 && T.p_min_frac < 1.0)) return bad("p_min_frac must be in [0, 1)");
  if (!finite_nonneg(T.tau_thin)) return bad("tau_thin must be finite and >= 0");
  return MORAY_OK;
}

// Highest level that can hold rays: rays of level l exist only if a level l-1
// ray split, which needs 12 * 4^(l-1) < 4 pi phi_c u^2 with u at most the
// largest distance inside the problem in local cells.
int reach_level(const moray_problem& P) {
  const moray_trace_params& T = P.params;
  if (T.phi_c <= 0.0) return T.level_init;
  const moray_grid& R = P.grids[0];
  double umax = std::sqrt((double)R.nx * R.nx + (double)R.ny * R.ny + (double)R.nz * R.nz) + 2.0;
  if (P.n_grids > 1) umax *= 2.0;
  const double k = 4.0 * kPiConst * T.phi_c * umax * umax;
  int l = T.level_init;
  while (l < T.level_max && std::ldexp(12.0, 2 * l) < k) ++l;
  return l;
}

// Upper estimate of the rays one level of one (source, group) tree can hold:
// children are created at ray densities of at most ~4 phi_c per local cell
// face, on a sphere whose part inside a grid is bounded by the grid's surface.
double level_rays_bound(const moray_problem& P) {
  const int lr = reach_level(P);
  double area = 0.0;
  for (int q = 0; q < P.n_grids; ++q) {
    const moray_grid& G = P.grids[q];
    area += 2.0 * ((double)G.nx * G.ny + (double)G.ny * G.nz + (double)G.nz * G.nx);
  }
  const double geo = 5.0 * std::max(P.params.phi_c, 1.0) * area + 256.0;
  return std::min(std::ldexp(12.0, 2 * lr), geo);
}

}  // namespace moray

extern "C" {

const char* moray_version(void) { return "0.2.0"; }

namespace {
// why the last moray_init on this thread returned no context
thread_local std::string g_init_err = "context is NULL";

moray_status init_fail(moray_status s, const std::string& msg) {
  g_init_err = msg;
  return s;
}
}  // namespace

const char* moray_last_error(const moray_ctx* ctx) { return ctx ? ctx->err.c_str() : g_init_err.c_str(); }

moray_status moray_init(moray_ctx** out, const moray_init_params* p) {
  if (!out) return init_fail(MORAY_EINVAL, "context pointer is NULL");
  *out = nullptr;
  if (!p) return init_fail(MORAY_EINVAL, "parameters are NULL");
  if (p->precision != MORAY_FP64 && p->precision != MORAY_FP32_ACC64) return init_fail(MORAY_EINVAL, "unknown precision");
  if (p->waves_per_cu < 0 || p->refill_lanes < 0 || p->refill_lanes > kWave || p->chunk_rays < 0 || p->reserve_rays < 0)
    return init_fail(MORAY_EINVAL, "negative or out-of-range launch setting");
  int n = 0;
  hipError_t he = hipGetDeviceCount(&n);
  if (he != hipSuccess || n < 1)
    return init_fail(MORAY_EDEVICE, std::string("no usable GPU: hipGetDeviceCount: ") + hipGetErrorString(he) +
                                        " (a process that loads a second HIP runtime, such as PyTorch's, after this "
                                        "library's leaves one of them without a device: load the other one first)");
  if (p->device < 0 || p->device >= n) return init_fail(MORAY_EINVAL, "device ordinal out of range");
  if ((he = hipSetDevice(p->device)) != hipSuccess)
    return init_fail(MORAY_EDEVICE, std::string("hipSetDevice: ") + hipGetErrorString(he));
  moray_ctx* c = new moray_ctx();
  c->device = p->device;
  c->precision = p->precision;
  c->stream = (hipStream_t)p->hip_stream;
  c->queue_cap_user = p->queue_capacity;
  c->profile = p->profile;
  if (const char* inj = std::getenv("MORAY_INJECT_CAPTURE_FAILURE")) c->fail_capture_once = inj[0] == '1';
  if (const char* inj = std::getenv("MORAY_INJECT_SERVE_OVERFLOW")) c->overflow_serve_once = inj[0] == '1';
  c->refill = p->refill_lanes ? p->refill_lanes : 64;
  c->chunk = p->chunk_rays ? p->chunk_rays : 256;
  c->reserve_user = p->reserve_rays;
  if ((he = hipDeviceGetAttribute(&c->num_cu, hipDeviceAttributeMultiprocessorCount, p->device)) != hipSuccess ||
      c->num_cu < 1) {
    delete c;
    return init_fail(MORAY_EDEVICE, std::string("hipDeviceGetAttribute: ") + hipGetErrorString(he));
  }
  c->cache = p->deposit_cache >= 0;
  int bpc = 1;
  if (trace_occupancy(c->precision, c->cache, &bpc) != hipSuccess || bpc < 1) bpc = 1;
  c->blocks_per_cu = bpc;
  if (p->waves_per_cu) {
    const int want = std::max(1, p->waves_per_cu / (kTraceBlock / kWave));
    c->blocks_per_cu = std::min(want, bpc);
  }
  size_t free_b = 0, total_b = 0;
  if ((he = hipMemGetInfo(&free_b, &total_b)) != hipSuccess) {
    delete c;
    return init_fail(MORAY_EDEVICE, std::string("hipMemGetInfo: ") + hipGetErrorString(he));
  }
  c->budget = p->hbm_budget_bytes ? p->hbm_budget_bytes : free_b / 2;
  if ((he = hipHostMalloc(&c->h_stage, 1 << 20, hipHostMallocDefault)) != hipSuccess) {
    delete c;
    return init_fail(MORAY_EDEVICE, std::string("hipHostMalloc: ") + hipGetErrorString(he));
  }
  c->h_stage_bytes = 1 << 20;
  // the fixed scratch array of moray_trace_noalloc: its address on this
  // device, looked up once per device with the device current
  void* sp = nullptr;
  if ((he = scratch_address(c->device, &sp)) == hipSuccess) c->scratch = (char*)sp;
  else c->scratch_err = std::string("hipGetSymbolAddress of the scratch array: ") + hipGetErrorString(he);
  *out = c;
  return MORAY_OK;
}

void moray_free(moray_ctx* c) {
  if (!c) return;
  engine_stop(c);
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  DevBuf* all[] = {&c->grids,   &c->probs,  &c->sgs,   &c->stats,  &c->ctr,     &c->kappa,  &c->kappa64,
                   &c->acc,     &c->mark,   &c->eexc,   &c->fblocks, &c->partial, &c->fields, &c->outs,
                   &c->eq_x,    &c->eq_kph, &c->eq_heat, &c->eq_dx,  &c->ev_lim, &c->eq_skip};
  for (DevBuf* b : all) release(c, *b);
  for (int i = 0; i < 2; ++i) {
    release(c, c->q_pix[i]);
    release(c, c->q_sg[i]);
    release(c, c->q_r[i]);
    release(c, c->q_P[i]);
  }
  for (hipEvent_t e : c->evs) (void)hipEventDestroy(e);
  if (c->plan) {
    drop_graph(c->plan);
    delete c->plan;
  }
  if (c->gstream) (void)hipStreamSynchronize(c->gstream), (void)hipStreamDestroy(c->gstream);
  if (c->gev) (void)hipEventDestroy(c->gev);
  if (c->h_stage) (void)hipHostFree(c->h_stage);
  delete c;
}

}  // extern "C"

namespace {

// The one-shot solve behind moray_trace and moray_trace_noalloc (c->arena:
// buffers carved from the scratch array, no graphs, no profiling, no staging
// growth).
moray_status trace_impl(moray_ctx* c, const moray_problem* probs, int n_probs, unsigned flags, moray_result* outs) {
  if (!c) return MORAY_EINVAL;
  if (!probs || n_probs < 1 || !outs) return fail(c, MORAY_EINVAL, "need n_probs >= 1 problems and results");
  if (flags & ~(MORAY_FIELDS_ON_DEVICE | MORAY_OUT_ON_DEVICE)) return fail(c, MORAY_EINVAL, "unknown flags");
  for (int i = 0; i < n_probs; ++i) {
    const moray_status s = validate(c, probs[i], i);
    if (s != MORAY_OK) return s;
    if (!outs[i].k_ph || !outs[i].heating) return fail(c, MORAY_EINVAL, "result buffers are NULL");
  }
  if (engine_busy(c)) return fail(c, MORAY_EBUSY, "asynchronous solves are still running on this context");
  if (!hip_ok(c, hipSetDevice(c->device), "hipSetDevice")) return MORAY_EDEVICE;

  // Repeated solves of the same descriptors with device-resident fields and
  // results: the second call captures its launch sequence in a graph, later
  // calls replay it (fields may change in place between calls).
  const bool graphable = (flags & MORAY_FIELDS_ON_DEVICE) && (flags & MORAY_OUT_ON_DEVICE) && !c->profile && !c->arena;
  std::string key;
  bool capture = false;
  if (graphable) {
    key = plan_key(c, probs, n_probs, flags, outs);
    if (!c->plan) c->plan = new PlanHost();
    PlanHost& ph = *c->plan;
    if (ph.valid && ph.key == key) {
      if (ph.exec) {
        const moray_status st = replay(c, ph, probs, n_probs, outs);
        if (st != MORAY_EQUEUE) return st;
      } else if (!ph.no_graph) {
        capture = true;
      }
    }
  }
  if (c->plan && !c->arena && !(capture && c->plan->key == key)) {
    drop_graph(c->plan);
    c->plan->valid = false;
    c->plan->no_graph = false;
  }
  const bool fdev = flags & MORAY_FIELDS_ON_DEVICE, odev = flags & MORAY_OUT_ON_DEVICE;
  const bool fp32 = c->precision == MORAY_FP32_ACC64;
  const size_t rsz = fp32 ? sizeof(float) : sizeof(double);

  // ---- tables: grids, problems, per-group energies ----
  std::vector<GridDev> grids;
  std::vector<ProblemDev> pdev(n_probs);
  std::vector<double> eexc;
  long long n_cells = 0, n_acc = 0;
  int max_reach = 0, min_l0 = kMaxLevel;
  unsigned max_steps = 64;
  for (int i = 0; i < n_probs; ++i) {
    const moray_problem& P = probs[i];
    ProblemDev& pd = pdev[i];
    pd.root_grid = (int)grids.size();
    pd.n_groups = P.spectrum->n_groups;
    pd.cell_off = n_cells;
    pd.eexc_off = (int)eexc.size();
    for (int g = 0; g < P.spectrum->n_groups; ++g)
      eexc.push_back((P.spectrum->energy_ev[g] - P.spectrum->e_ion_ev) * kEvErgConst);
    long long steps = 16;
    for (int q = 0; q < P.n_grids; ++q) {
      const moray_grid& G = P.grids[q];
      GridDev d{};
      d.nx = G.nx; d.ny = G.ny; d.nz = G.nz;
      d.is_child = q > 0;
      d.ox = q > 0 ? G.offset[0] : 0;
      d.oy = q > 0 ? G.offset[1] : 0;
      d.oz = q > 0 ? G.offset[2] : 0;
      d.problem = i;
      d.cell_off = n_cells;
      d.dx_cm = G.dx_cm;
      grids.push_back(d);
      n_cells += (long long)G.nx * G.ny * G.nz;
      steps += 2LL * (G.nx + G.ny + G.nz);
    }
    pd.n_cells = n_cells - pd.cell_off;
    pd.acc_off = n_acc;
    n_acc += pd.n_cells * pd.n_groups;
    max_steps = std::max<unsigned>(max_steps, (unsigned)std::min<long long>(steps * 2, 1u << 30));
    max_reach = std::max(max_reach, reach_level(P));
    min_l0 = std::min(min_l0, P.params.level_init);
  }
  if (n_cells >= (1LL << 31) - 1) return fail(c, MORAY_EINVAL, "batch exceeds 2^31 cells");
  // Accumulators: one float64 sum per (group, cell) for the problems that do
  // not ask for the radiation-pressure acceleration; after them, from the
  // first 64-byte boundary (rec_base), a 32-byte record per (group, cell)
  // (absorbed rate and momentum x, y, z) for those that do.
  // Problems with the optically-thin approximation keep a second sum per
  // (group, cell) among the plain ones (stride 2), for the deposits of thin
  // rays in cells that hold their source.
  bool thin = false;
  long long n_plain = 0, n_rec = 0;
  for (int i = 0; i < n_probs; ++i)
    if (!outs[i].accel) {
      const int stride = probs[i].params.tau_thin > 0.0 ? 2 : 1;
      thin = thin || stride == 2;
      pdev[i].acc_stride = stride;
      pdev[i].acc_off = n_plain;
      n_plain += stride * pdev[i].n_cells * pdev[i].n_groups;
    }
  const long long rec_base = (n_plain + 7) & ~7LL;
  for (int i = 0; i < n_probs; ++i)
    if (outs[i].accel) {
      pdev[i].acc_stride = 4;
      pdev[i].acc_off = rec_base + n_rec;
      n_rec += 4 * pdev[i].n_cells * pdev[i].n_groups;
    }
  const bool radp = n_rec > 0;
  const long long n_sums = radp ? rec_base + n_rec : n_plain;
  for (int i = 0; i < n_probs; ++i)
    if (outs[i].accel && probs[i].params.tau_thin > 0.0)
      return fail(c, MORAY_EINVAL, "problem " + std::to_string(i) +
                                       ": the optically-thin approximation does not take radiation pressure");
  if (thin && radp)
    return fail(c, MORAY_EINVAL, "a batch cannot mix the optically-thin approximation with radiation pressure");
  // optically-thin marks: one byte per (source, group) tree and cell, per
  // problem that uses the approximation (the paper's marker field holds a
  // bit per source; a byte takes a plain store where a bit needs an atomic)
  long long n_mark = 0;
  for (int i = 0; i < n_probs; ++i)
    if (probs[i].params.tau_thin > 0.0) {
      pdev[i].mark_trees = probs[i].n_sources * probs[i].spectrum->n_groups;
      pdev[i].mark_off = n_mark;
      n_mark += pdev[i].mark_trees * pdev[i].n_cells;
    }
  (void)n_acc;
  // the trace kernel addresses accumulators with 32-bit indices
  if (n_sums >= (long long)kNoSlot)
    return fail(c, MORAY_EINVAL, "a batch needs fewer than 2^32 - 1 accumulators (cells x groups, 4 times that "
                                 "with radiation pressure)");
  bool cover = false;                                   // some problem scales its deposits by the covering factor
  for (int i = 0; i < n_probs; ++i) cover = cover || probs[i].params.covering != 0;

  // finalize blocks: each covers up to kFinalBlock*kFinalCellsPerThread cells of one grid
  std::vector<FinalBlock> fblocks;
  std::vector<int> fblock_first(n_probs + 1, 0);
  {
    const long long per = (long long)kFinalBlock * kFinalCellsPerThread;
    for (size_t q = 0; q < grids.size(); ++q) {
      const GridDev& G = grids[q];
      if (q == 0 || grids[q - 1].problem != G.problem) fblock_first[G.problem] = (int)fblocks.size();
      const long long nc = (long long)G.nx * G.ny * G.nz;
      for (long long f = 0; f < nc; f += per)
        fblocks.push_back({(int)q, (int)std::min(per, nc - f), f});
    }
    fblock_first[n_probs] = (int)fblocks.size();
  }

  // (source, group) trees ordered by seed level, then problem, source, group
  std::vector<SgKey> keys;
  for (int i = 0; i < n_probs; ++i)
    for (int s = 0; s < probs[i].n_sources; ++s)
      for (int g = 0; g < probs[i].spectrum->n_groups; ++g) keys.push_back({probs[i].params.level_init, i, s, g});
  std::stable_sort(keys.begin(), keys.end(), [](const SgKey& a, const SgKey& b) { return a.l0 < b.l0; });
  const int n_sg = (int)keys.size();
  std::vector<SgDev> sgs(n_sg);
  std::vector<double> sg_bound(n_sg);
  for (int k = 0; k < n_sg; ++k) {
    const SgKey& K = keys[k];
    const moray_problem& P = probs[K.prob];
    const moray_source& S = P.sources[K.src];
    const moray_spectrum& Sp = *P.spectrum;
    const ProblemDev& pd = pdev[K.prob];
    SgDev& d = sgs[k];
    d.sx = S.x; d.sy = S.y; d.sz = S.z;
    const double npix0 = std::ldexp(12.0, 2 * P.params.level_init);
    d.P0 = Sp.photon_frac[K.grp] * S.ndot / npix0;
    d.pmin0 = P.params.p_min_frac * d.P0;
    d.sigma64 = Sp.sigma_cm2[K.grp];
    d.sigma32 = (float)Sp.sigma_cm2[K.grp];
    d.four_pi_phi_c = 4.0 * kPiConst * P.params.phi_c;
    d.split_t2_base = P.params.phi_c > 0.0 ? (float)(12.0 / (4.0 * kPiConst * P.params.phi_c)) : FLT_MAX;
    d.acc_stride = (uint32_t)pd.acc_stride;
    d.acc_slot = pd.acc_off + (long long)pd.acc_stride * ((long long)K.grp * pd.n_cells - pd.cell_off);
    d.problem = K.prob;
    d.covering = P.params.covering != 0;
    if (pd.acc_stride == 4) d.mom_scale = Sp.energy_ev[K.grp] * kEvErgConst / kLightCms;
    d.root_grid = pd.root_grid;
    d.rnx = grids[pd.root_grid].nx; d.rny = grids[pd.root_grid].ny; d.rnz = grids[pd.root_grid].nz;
    d.rcell_off = grids[pd.root_grid].cell_off;
    d.level_init = P.params.level_init;
    d.gen0 = P.params.level_init;     // one-shot solve: the launch generation is the HEALPix level
    d.level_max = P.params.phi_c > 0.0 ? P.params.level_max : P.params.level_init;
    if (k == 0 || keys[k - 1].prob != K.prob) pdev[K.prob].sg_first = k;
    if (P.params.tau_thin > 0.0) {
      const double phi_thin = std::min(1.0, P.params.phi_c);
      const int t = K.src * Sp.n_groups + K.grp;                  // the tree within its problem
      const double dx_root = P.grids[0].dx_cm;
      d.tau_thin = P.params.tau_thin;
      d.four_pi_phi_thin = 4.0 * kPiConst * phi_thin;
      d.split_t2_thin = phi_thin > 0.0 ? (float)(12.0 / (4.0 * kPiConst * phi_thin)) : FLT_MAX;
      d.mark_base = pd.mark_off + (long long)t * pd.n_cells - pd.cell_off;
      d.thin_coef = d.sigma64 * (d.P0 * npix0) / (4.0 * kPiConst * dx_root * dx_root);
    }
    sg_bound[k] = level_rays_bound(P);
  }

  // ---- queue capacity ----
  double need = 0.0;
  for (double b : sg_bound) need += b;
  size_t cap = c->queue_cap_user;
  const size_t per_ray = 2 * (sizeof(uint64_t) + sizeof(uint32_t) + 2 * sizeof(double));
  const size_t out_stage = odev ? 0 : (size_t)n_cells * (radp ? 40 : 16);
  const size_t fixed = (size_t)n_cells * rsz + (size_t)n_sums * 8 + (size_t)n_mark +
                       (thin && fp32 ? (size_t)n_cells * 8 : 0) + (fdev ? 0 : (size_t)n_cells * 8) + out_stage + (size_t)n_sg * (sizeof(SgDev) + sizeof(SgStats)) +
                       grids.size() * sizeof(GridDev) + fblocks.size() * (sizeof(FinalBlock) + 8) +
                       (c->arena ? (size_t)(1 << 20) : (size_t)(64 << 20));
  if (!cap) {
    const size_t room = c->budget > c->allocated + fixed ? c->budget - fixed : 0;
    const double fit = (double)room / (double)per_ray;
    const double slack = (double)std::max(1, c->num_cu * c->blocks_per_cu) * (kTraceBlock / kWave) * kReserveMax;
    cap = (size_t)std::max(4096.0, std::min({need + slack, fit, 2.0e9}));
  }
  cap = std::max<size_t>(cap, 256);

  // ---- device memory ----
  moray_status st;
  if ((st = ensure(c, c->grids, grids.size() * sizeof(GridDev), "grid table")) ||
      (st = ensure(c, c->probs, pdev.size() * sizeof(ProblemDev), "problem table")) ||
      (st = ensure(c, c->sgs, std::max<size_t>(1, n_sg) * sizeof(SgDev), "source table")) ||
      (st = ensure(c, c->stats, std::max<size_t>(1, n_sg) * sizeof(SgStats), "statistics")) ||
      (st = ensure(c, c->ctr, sizeof(Counters), "counters")) ||
      (st = ensure(c, c->kappa, (size_t)n_cells * rsz, "absorber columns")) ||
      (st = ensure(c, c->acc, (size_t)std::max<long long>(1, n_sums) * 8, "accumulators")) ||
      (n_mark && (st = ensure(c, c->mark, (size_t)n_mark, "optically-thin marks"))) ||
      (thin && fp32 && (st = ensure(c, c->kappa64, (size_t)n_cells * 8, "float64 absorber columns"))) ||
      (st = ensure(c, c->eexc, eexc.size() * 8, "group energies")) ||
      (st = ensure(c, c->fblocks, fblocks.size() * sizeof(FinalBlock), "finalize blocks")) ||
      (st = ensure(c, c->partial, fblocks.size() * 8, "partial sums")))
    return st;
  if (!fdev && (st = ensure(c, c->fields, (size_t)n_cells * 8, "field upload"))) return st;
  if (!odev && (st = ensure(c, c->outs, out_stage, "result staging"))) return st;
  for (int i = 0; i < 2; ++i) {
    if ((st = ensure(c, c->q_pix[i], cap * 8, "ray queue")) || (st = ensure(c, c->q_sg[i], cap * 4, "ray queue")) ||
        (st = ensure(c, c->q_r[i], cap * 8, "ray queue")) || (st = ensure(c, c->q_P[i], cap * 8, "ray queue")))
      return st;
  }
  c->q_cap = cap;

  // field and output pointers
  float* fbuf = (float*)c->fields.p;
  double* obuf = (double*)c->outs.p;
  {
    size_t gi = 0;
    for (int i = 0; i < n_probs; ++i) {
      long long within = 0;
      for (int q = 0; q < probs[i].n_grids; ++q, ++gi) {
        const moray_grid& G = probs[i].grids[q];
        GridDev& d = grids[gi];
        const long long nc = (long long)G.nx * G.ny * G.nz;
        if (fdev) {
          d.n_h = G.n_h;
          d.x_hi = G.x_hi;
        } else {
          d.n_h = fbuf + d.cell_off;
          d.x_hi = fbuf + n_cells + d.cell_off;
          if (!hip_ok(c, hipMemcpyAsync((void*)d.n_h, G.n_h, nc * 4, hipMemcpyHostToDevice, c->stream), "upload") ||
              !hip_ok(c, hipMemcpyAsync((void*)d.x_hi, G.x_hi, nc * 4, hipMemcpyHostToDevice, c->stream), "upload"))
            return MORAY_EDEVICE;
        }
        if (odev) {
          d.out_kph = outs[i].k_ph + within;
          d.out_heat = outs[i].heating + within;
          d.out_acc = outs[i].accel ? outs[i].accel + within : nullptr;
        } else {
          d.out_kph = obuf + d.cell_off;
          d.out_heat = obuf + n_cells + d.cell_off;
          // the problem's three planes follow one another in the staging area
          d.out_acc = outs[i].accel ? obuf + 2 * n_cells + 3 * pdev[i].cell_off + within : nullptr;
        }
        within += nc;
      }
    }
  }
  auto up = [&](DevBuf& b, const void* src, size_t bytes) {
    return bytes == 0 || hip_ok(c, hipMemcpyAsync(b.p, src, bytes, hipMemcpyHostToDevice, c->stream), "upload");
  };
  if (!up(c->grids, grids.data(), grids.size() * sizeof(GridDev)) ||
      !up(c->probs, pdev.data(), pdev.size() * sizeof(ProblemDev)) ||
      !up(c->sgs, sgs.data(), n_sg * sizeof(SgDev)) || !up(c->eexc, eexc.data(), eexc.size() * 8) ||
      !up(c->fblocks, fblocks.data(), fblocks.size() * sizeof(FinalBlock)))
    return MORAY_EDEVICE;

  // seed ranges per level
  std::vector<int> seed_lo(kLevels, 0), seed_hi(kLevels, 0);
  for (int l = 0; l <= kMaxLevel; ++l) {
    int lo = n_sg, hi = n_sg;
    for (int k = 0; k < n_sg; ++k)
      if (keys[k].l0 == l) { lo = std::min(lo, k); hi = k + 1; }
    if (lo >= hi) lo = hi = 0;
    seed_lo[l] = lo;
    seed_hi[l] = hi;
  }

  const int blocks = std::max(1, c->num_cu * c->blocks_per_cu);
  const int n_grids_tot = (int)grids.size();
  Counters* ctr = (Counters*)c->ctr.p;
  SgStats* stats = (SgStats*)c->stats.p;
  // each wave may leave up to one reserved block unused per level: keep that
  // under an eighth of the queue and plan the trees against the rest
  const double waves = (double)blocks * (kTraceBlock / kWave);
  // level queues in nseg segments (one claim and one write counter each); a
  // segment serves about waves/nseg waves, so the reserve fraction holds per segment
  const int nseg = queue_segments(cap);
  const unsigned long long seg_cap = cap / (size_t)nseg;
  unsigned long long reserve = (unsigned long long)std::min<double>((double)kReserveMax, (double)cap / (8.0 * waves));
  if (c->reserve_user > 0) reserve = std::min<unsigned long long>((unsigned long long)c->reserve_user, kReserveMax);
  reserve = std::max<unsigned long long>(4, reserve & ~3ull);
  double chunk_limit = std::max(1.0, (double)cap - waves * (double)reserve);
  const int max_launches = (max_reach - min_l0 + 1);

  // pinned staging for the counters, the tree statistics and the partial sums
  const size_t need_stage = sizeof(Counters) + n_sg * sizeof(SgStats) + fblocks.size() * 8;
  if (need_stage > c->h_stage_bytes && c->arena)
    return fail(c, MORAY_ENOMEM, "moray_trace_noalloc: the batch has more (source, group) trees and finalize blocks "
                                 "than the context's 1 MiB read-back staging holds");
  if (need_stage > c->h_stage_bytes) {
    (void)hipHostFree(c->h_stage);
    c->h_stage = nullptr;
    if (hipHostMalloc(&c->h_stage, need_stage, hipHostMallocDefault) != hipSuccess) {
      c->h_stage_bytes = 0;
      return fail(c, MORAY_ENOMEM, "pinned staging allocation failed");
    }
    c->h_stage_bytes = need_stage;
  }
  char* hs = (char*)c->h_stage;
  Counters* hctr = (Counters*)hs;
  SgStats* hst = (SgStats*)(hs + sizeof(Counters));
  double* hpart = (double*)(hs + sizeof(Counters) + n_sg * sizeof(SgStats));
  if (capture) {
    if (!c->gstream && (!hip_ok(c, hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking), "stream") ||
                        !hip_ok(c, hipEventCreateWithFlags(&c->gev, hipEventDisableTiming), "event")))
      return MORAY_EDEVICE;
    // the tables above were uploaded on the context's stream
    if (!hip_ok(c, hipStreamSynchronize(c->stream), "synchronize")) return MORAY_EDEVICE;
  }

  // A failure while the launch sequence is being captured (or instantiating
  // or launching the graph) ends the capture, drops the graph and reruns the
  // solve eagerly on the context's stream: the call still succeeds.
  auto abandon_capture = [&](hipStream_t s) {
    hipGraph_t g = nullptr;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
      (void)hipStreamEndCapture(s, &g);
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    drop_graph(c->plan);
    c->plan->no_graph = true;
  };
  for (int attempt = 0;; ++attempt) {
    const bool capturing = capture && attempt == 0 && !c->plan->no_graph;
    hipStream_t strm = capturing ? c->gstream : c->stream;
    if (capturing && (c->fail_capture_once || !hip_ok(c, hipStreamBeginCapture(strm, hipStreamCaptureModeThreadLocal), "capture"))) {
      c->fail_capture_once = false;
      abandon_capture(strm);
      continue;
    }
    // chunks: consecutive trees whose bounds fit the capacity
    std::vector<ChunkPlan> chunks;
    {
      int b = 0;
      double acc = 0.0;
      for (int k = 0; k < n_sg; ++k) {
        if (k > b && acc + sg_bound[k] > chunk_limit) {
          chunks.push_back({b, k});
          b = k;
          acc = 0.0;
        }
        acc += sg_bound[k];
      }
      if (n_sg > b) chunks.push_back({b, n_sg});
    }
    const int n_launch_total = (int)chunks.size() * max_launches;
    if (c->profile && (int)c->evs.size() < 2 * n_launch_total) {
      while ((int)c->evs.size() < 2 * n_launch_total) {
        hipEvent_t e;
        if (!hip_ok(c, hipEventCreate(&e), "hipEventCreate")) return MORAY_EDEVICE;
        c->evs.push_back(e);
      }
    }
    if (!hip_ok(c, launch_reset(strm, ctr, stats, n_sg), "reset")) {
      if (capturing) { abandon_capture(strm); continue; }
      return MORAY_EDEVICE;
    }
    uint8_t* mark = n_mark ? (uint8_t*)c->mark.p : nullptr;
    double* kappa64 = thin && fp32 ? (double*)c->kappa64.p : nullptr;
    hipError_t e = fp32 ? launch_prep<float>(strm, c->num_cu, (GridDev*)c->grids.p, n_grids_tot, 0,
                                             (ProblemDev*)c->probs.p, 0, n_cells, (float*)c->kappa.p, (double*)c->acc.p, ctr,
                                             mark, kappa64)
                        : launch_prep<double>(strm, c->num_cu, (GridDev*)c->grids.p, n_grids_tot, 0,
                                              (ProblemDev*)c->probs.p, 0, n_cells, (double*)c->kappa.p,
                                              (double*)c->acc.p, ctr, mark);
    if (!hip_ok(c, e, "prep")) {
      if (capturing) { abandon_capture(strm); continue; }
      return MORAY_EDEVICE;
    }
    int launches = 0;
    bool launch_failed = false;
    for (const ChunkPlan& ch : chunks) {
      if (chunks.size() > 1 && !hip_ok(c, launch_reset_levels(strm, ctr), "reset levels")) {
        launch_failed = true;
        break;
      }
      for (int l = min_l0; l <= max_reach; ++l) {
        const int lo = std::max(seed_lo[l], ch.sg_begin), hi = std::min(seed_hi[l], ch.sg_end);
        const RayQueue qin{(uint64_t*)c->q_pix[l & 1].p, (uint32_t*)c->q_sg[l & 1].p, (double*)c->q_r[l & 1].p,
                           (double*)c->q_P[l & 1].p};
        const RayQueue qout{(uint64_t*)c->q_pix[(l + 1) & 1].p, (uint32_t*)c->q_sg[(l + 1) & 1].p,
                            (double*)c->q_r[(l + 1) & 1].p, (double*)c->q_P[(l + 1) & 1].p};
        if (c->profile) (void)hipEventRecord(c->evs[2 * launches], strm);
        if (fp32) {
          TraceArgs<float> A{};
          A.grids = (GridDev*)c->grids.p; A.probs = (ProblemDev*)c->probs.p; A.sgs = (SgDev*)c->sgs.p;
          A.kappa = (float*)c->kappa.p; A.acc = (double*)c->acc.p; A.rec_base = (uint32_t)rec_base; A.in = qin; A.out = qout;
          A.seg_cap = seg_cap; A.nseg = nseg; A.ctr = ctr; A.stats = stats; A.gen = l; A.cin = l; A.cout = l + 1;
          A.seed_level = l;
          A.seed_sg_begin = lo < hi ? lo : 0; A.seed_sg_end = lo < hi ? hi : 0;
          A.chunk = c->chunk; A.refill = c->refill; A.max_steps = max_steps; A.reserve = reserve;
          A.mark = mark;
          A.kappa64 = kappa64;
          e = launch_trace_level<float>(strm, blocks, A, c->cache, cover, radp, thin);
        } else {
          TraceArgs<double> A{};
          A.grids = (GridDev*)c->grids.p; A.probs = (ProblemDev*)c->probs.p; A.sgs = (SgDev*)c->sgs.p;
          A.kappa = (double*)c->kappa.p; A.acc = (double*)c->acc.p; A.rec_base = (uint32_t)rec_base; A.in = qin; A.out = qout;
          A.seg_cap = seg_cap; A.nseg = nseg; A.ctr = ctr; A.stats = stats; A.gen = l; A.cin = l; A.cout = l + 1;
          A.seed_level = l;
          A.seed_sg_begin = lo < hi ? lo : 0; A.seed_sg_end = lo < hi ? hi : 0;
          A.chunk = c->chunk; A.refill = c->refill; A.max_steps = max_steps; A.reserve = reserve;
          A.mark = mark;
          e = launch_trace_level<double>(strm, blocks, A, c->cache, cover, radp, thin);
        }
        if (!hip_ok(c, e, "trace")) {
          launch_failed = true;
          break;
        }
        if (c->profile) (void)hipEventRecord(c->evs[2 * launches + 1], strm);
        ++launches;
      }
      if (launch_failed) break;
    }
    if (launch_failed) {
      if (capturing) { abandon_capture(strm); continue; }
      return MORAY_EDEVICE;
    }
    if (!hip_ok(c, launch_finalize(strm, (int)fblocks.size(), (GridDev*)c->grids.p, (ProblemDev*)c->probs.p,
                                   (FinalBlock*)c->fblocks.p, (double*)c->acc.p, (double*)c->eexc.p,
                                   (double*)c->partial.p, ctr, (SgDev*)c->sgs.p, mark),
                "finalize")) {
      if (capturing) { abandon_capture(strm); continue; }
      return MORAY_EDEVICE;
    }

    // ---- results ----
    if (!hip_ok(c, hipMemcpyAsync(hctr, ctr, sizeof(Counters), hipMemcpyDeviceToHost, strm), "copy") ||
        (n_sg && !hip_ok(c, hipMemcpyAsync(hst, stats, n_sg * sizeof(SgStats), hipMemcpyDeviceToHost, strm), "copy")) ||
        (!fblocks.empty() &&
         !hip_ok(c, hipMemcpyAsync(hpart, c->partial.p, fblocks.size() * 8, hipMemcpyDeviceToHost, strm), "copy"))) {
      if (capturing) { abandon_capture(strm); continue; }
      return MORAY_EDEVICE;
    }
    if (capturing) {
      PlanHost& ph = *c->plan;
      if (!hip_ok(c, hipStreamEndCapture(strm, &ph.graph), "capture") ||
          !hip_ok(c, hipGraphInstantiate(&ph.exec, ph.graph, nullptr, nullptr, 0), "graph instantiate") ||
          !hip_ok(c, hipGraphLaunch(ph.exec, strm), "graph launch")) {
        abandon_capture(strm);
        continue;
      }
    }
    if (!hip_ok(c, hipStreamSynchronize(strm), "synchronize")) return MORAY_EDEVICE;
    if (hctr->err & kErrBadInput) return fail(c, MORAY_EINVAL, "a density or neutral fraction is negative, non-finite or x_HI > 1");
    if (hctr->err & kErrInternal) return fail(c, MORAY_EINTERNAL, "a ray exceeded its step bound");
    if (hctr->err & kErrOverflow) {
      bool single = true;
      for (const ChunkPlan& ch : chunks) single = single && ch.sg_end - ch.sg_begin <= 1;
      if (c->plan) {
        drop_graph(c->plan);
        c->plan->no_graph = true;
      }
      if (single || attempt >= 6)
        return fail(c, MORAY_EQUEUE, "ray queue overflowed; raise queue_capacity or the HBM budget");
      chunk_limit *= 0.25;   // retry with smaller chunks of trees
      continue;
    }
    double trace_ms = 0.0;
    if (c->profile) {
      for (int k = 0; k < launches; ++k) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c->evs[2 * k], c->evs[2 * k + 1]) == hipSuccess) trace_ms += ms;
      }
    }
    PlanHost local;
    PlanHost& ph = graphable ? *c->plan : local;
    ph.keys = keys;
    ph.fblock_first = fblock_first;
    ph.n_sg = n_sg;
    ph.nfb = fblocks.size();
    ph.nseg = nseg;
    ph.seg_cap = seg_cap;
    ph.launches = launches;
    if (graphable) {
      ph.key = key;
      ph.valid = true;
    }
    collect(c, ph, probs, n_probs, outs, trace_ms);
    if (!odev) {
      for (int i = 0; i < n_probs; ++i) {
        const long long off = pdev[i].cell_off, nc = pdev[i].n_cells;
        if (!hip_ok(c, hipMemcpy(outs[i].k_ph, obuf + off, nc * 8, hipMemcpyDeviceToHost), "copy results") ||
            !hip_ok(c, hipMemcpy(outs[i].heating, obuf + n_cells + off, nc * 8, hipMemcpyDeviceToHost), "copy results") ||
            (outs[i].accel && !hip_ok(c, hipMemcpy(outs[i].accel, obuf + 2 * n_cells + 3 * off, 3 * nc * 8,
                                                   hipMemcpyDeviceToHost), "copy results")))
          return MORAY_EDEVICE;
      }
    }
    c->err = "no error";
    return MORAY_OK;
  }
}

}  // namespace

extern "C" {

moray_status moray_trace(moray_ctx* c, const moray_problem* probs, int n_probs, unsigned flags, moray_result* outs) {
  return trace_impl(c, probs, n_probs, flags, outs);
}

moray_status moray_trace_noalloc(moray_ctx* c, const moray_problem* probs, int n_probs, unsigned flags,
                                 moray_result* outs) {
  if (!c) return MORAY_EINVAL;
  if (!c->scratch)
    return fail(c, MORAY_EDEVICE, c->scratch_err.empty() ? "no scratch array on this device" : c->scratch_err);
  // The context's own buffers step aside for the call (they stay allocated
  // for later moray_trace calls); every buffer of this call is carved from
  // the scratch array, from its start, and graphs and profiling are off.
  DevBuf* bufs[] = {&c->grids,    &c->probs,    &c->sgs,      &c->stats,    &c->ctr,      &c->kappa,    &c->kappa64,
                    &c->acc,      &c->mark,     &c->eexc,     &c->fblocks,  &c->partial,  &c->fields,   &c->outs,
                    &c->q_pix[0], &c->q_sg[0],  &c->q_r[0],   &c->q_P[0],   &c->q_pix[1], &c->q_sg[1],
                    &c->q_r[1],   &c->q_P[1]};
  constexpr int nb = (int)(sizeof(bufs) / sizeof(bufs[0]));
  DevBuf saved[nb];
  for (int i = 0; i < nb; ++i) {
    saved[i] = *bufs[i];
    *bufs[i] = DevBuf{};
  }
  const size_t budget = c->budget, allocated = c->allocated, q_cap = c->q_cap;
  const int profile = c->profile;
  c->budget = scratch_bytes();
  c->allocated = 0;
  c->profile = 0;
  c->arena = true;
  c->arena_used = 0;
  const moray_status st = trace_impl(c, probs, n_probs, flags, outs);
  c->arena = false;
  c->arena_used = 0;
  c->profile = profile;
  c->budget = budget;
  c->allocated = allocated;
  c->q_cap = q_cap;
  for (int i = 0; i < nb; ++i) *bufs[i] = saved[i];
  return st;
}

// Cells of the ionisation updates: every grid of the problem in order
// (their offsets in the concatenated results), and a mask of the root cells a
// child covers, which keep their neutral fraction (their field lives in the
// child), uploaded to c->eq_skip.
struct UpdateGrids {
  std::vector<long long> off;      // first cell of each grid; off.back() = all cells
};

static moray_status update_grids(moray_ctx* c, const moray_problem& P, UpdateGrids& U) {
  U.off.assign(1, 0);
  for (int q = 0; q < P.n_grids; ++q)
    U.off.push_back(U.off.back() + (long long)P.grids[q].nx * P.grids[q].ny * P.grids[q].nz);
  if (P.n_grids == 1) return MORAY_OK;
  const moray_grid& R = P.grids[0];
  std::vector<unsigned char> skip((size_t)U.off[1], 0);
  for (int q = 1; q < P.n_grids; ++q) {
    const moray_grid& G = P.grids[q];
    for (int k = 0; k < G.nz / 2; ++k)
      for (int j = 0; j < G.ny / 2; ++j)
        for (int i = 0; i < G.nx / 2; ++i)
          skip[(size_t)(G.offset[0] + i) + (size_t)R.nx * ((size_t)(G.offset[1] + j) + (size_t)R.ny * (G.offset[2] + k))] = 1;
  }
  moray_status st = ensure(c, c->eq_skip, skip.size(), "covered cells");
  if (st != MORAY_OK) return st;
  if (!hip_ok(c, hipMemcpyAsync(c->eq_skip.p, skip.data(), skip.size(), hipMemcpyHostToDevice, c->stream), "upload") ||
      !hip_ok(c, hipStreamSynchronize(c->stream), "synchronize"))
    return MORAY_EDEVICE;
  return MORAY_OK;
}

moray_status moray_equilibrate(moray_ctx* c, const moray_problem* prob, unsigned flags,
                               const moray_equilibrium_params* ep, double* x_out, moray_result* out, int* iterations) {
  if (!c) return MORAY_EINVAL;
  if (!prob || !ep || !out) return fail(c, MORAY_EINVAL, "NULL problem, parameters or result");
  if (!(ep->alpha_b > 0.0) || !(ep->damping > 0.0 && ep->damping <= 1.0) || !(ep->tol > 0.0) || ep->max_iter < 1)
    return fail(c, MORAY_EINVAL, "alpha_b, damping, tol or max_iter out of range");
  if (!(flags & MORAY_FIELDS_ON_DEVICE)) return fail(c, MORAY_EINVAL, "the equilibrium iteration needs device fields");
  if (engine_busy(c)) return fail(c, MORAY_EBUSY, "the context is serving asynchronous solves");
  moray_status st = validate(c, *prob, 0);
  if (st != MORAY_OK) return st;
  if (!hip_ok(c, hipSetDevice(c->device), "hipSetDevice")) return MORAY_EDEVICE;
  UpdateGrids U;
  if ((st = update_grids(c, *prob, U)) != MORAY_OK) return st;
  const int ng = prob->n_grids;
  const long long n = U.off.back();
  const size_t stride = 1 + kEqMaxBlocks;      // one reduction area per grid
  if ((st = ensure(c, c->eq_x, (size_t)n * 8, "equilibrium iterate")) ||
      (st = ensure(c, c->eq_kph, (size_t)n * 8, "equilibrium rates")) ||
      (st = ensure(c, c->eq_heat, (size_t)n * 8, "equilibrium rates")) ||
      (st = ensure(c, c->eq_dx, (size_t)ng * stride * 8, "equilibrium change")))
    return st;
  // the caller's x_hi arrays are the iterate the trace reads (updated in place, see moray.h)
  double* x64 = (double*)c->eq_x.p;
  double* dx = (double*)c->eq_dx.p;
  const unsigned char* skip = ng > 1 ? (const unsigned char*)c->eq_skip.p : nullptr;
  for (int q = 0; q < ng; ++q)
    if (!hip_ok(c, launch_widen(c->stream, c->num_cu, prob->grids[q].x_hi, x64 + U.off[q], U.off[q + 1] - U.off[q]),
                "equilibrium start"))
      return MORAY_EDEVICE;
  moray_result mid{};
  mid.k_ph = (double*)c->eq_kph.p;
  mid.heating = (double*)c->eq_heat.p;
  const unsigned mid_flags = flags | MORAY_OUT_ON_DEVICE;
  std::vector<double> change(ng);
  int it = 0;
  while (it < ep->max_iter) {
    if ((st = moray_trace(c, prob, 1, mid_flags, &mid)) != MORAY_OK) return st;
    ++it;
    for (int q = 0; q < ng; ++q) {
      const moray_grid& G = prob->grids[q];
      if (!hip_ok(c, launch_equilibrium_update(c->stream, mid.k_ph + U.off[q], G.n_h, x64 + U.off[q],
                                               const_cast<float*>(G.x_hi), U.off[q + 1] - U.off[q], ep->alpha_b,
                                               ep->damping, q == 0 ? skip : nullptr, dx + q * stride),
                  "equilibrium update") ||
          !hip_ok(c, hipMemcpyAsync(&change[q], dx + q * stride, 8, hipMemcpyDeviceToHost, c->stream), "copy"))
        return MORAY_EDEVICE;
    }
    if (!hip_ok(c, hipStreamSynchronize(c->stream), "synchronize")) return MORAY_EDEVICE;
    if (*std::max_element(change.begin(), change.end()) < ep->tol) break;
  }
  if ((st = moray_trace(c, prob, 1, flags, out)) != MORAY_OK) return st;
  if (x_out && (!hip_ok(c, hipMemcpyAsync(x_out, x64, (size_t)n * 8, hipMemcpyDeviceToDevice, c->stream), "copy") ||
                !hip_ok(c, hipStreamSynchronize(c->stream), "synchronize")))
    return MORAY_EDEVICE;
  if (iterations) *iterations = it;
  return MORAY_OK;
}

moray_status moray_evolve(moray_ctx* c, const moray_problem* prob, unsigned flags, const moray_evolve_params* ep,
                          double* x_out, moray_result* out, int* steps, double* t_reached, double* dt_steps) {
  if (!c) return MORAY_EINVAL;
  if (!prob || !ep || !out) return fail(c, MORAY_EINVAL, "NULL problem, parameters or result");
  if (!(ep->alpha_b > 0.0) || !(ep->eps_ion > 0.0) || !(ep->tau_front >= 0.0) || !(ep->dt_max > 0.0) ||
      !(ep->t_end > 0.0) || !std::isfinite(ep->t_end) || !std::isfinite(ep->dt_max) || ep->max_steps < 1)
    return fail(c, MORAY_EINVAL, "alpha_b, eps_ion, tau_front, dt_max, t_end or max_steps out of range");
  if (!(flags & MORAY_FIELDS_ON_DEVICE)) return fail(c, MORAY_EINVAL, "the time-stepped evolution needs device fields");
  if (engine_busy(c)) return fail(c, MORAY_EBUSY, "the context is serving asynchronous solves");
  moray_status st = validate(c, *prob, 0);
  if (st != MORAY_OK) return st;
  if (!hip_ok(c, hipSetDevice(c->device), "hipSetDevice")) return MORAY_EDEVICE;
  UpdateGrids U;
  if ((st = update_grids(c, *prob, U)) != MORAY_OK) return st;
  const int ng = prob->n_grids;
  const long long n = U.off.back();
  const size_t stride = 1 + kEqMaxBlocks;      // one reduction area per grid
  if ((st = ensure(c, c->eq_x, (size_t)n * 8, "evolution iterate")) ||
      (st = ensure(c, c->eq_kph, (size_t)n * 8, "evolution rates")) ||
      (st = ensure(c, c->eq_heat, (size_t)n * 8, "evolution rates")) ||
      (st = ensure(c, c->ev_lim, (size_t)n * 8, "evolution step limits")) ||
      (st = ensure(c, c->eq_dx, (size_t)ng * stride * 8, "evolution step")))
    return st;
  // photon-weighted cross-section of the spectrum: the front test's sigma
  const moray_spectrum& Sp = *prob->spectrum;
  double sigma_bar = 0.0;
  for (int g = 0; g < Sp.n_groups; ++g) sigma_bar += Sp.photon_frac[g] * Sp.sigma_cm2[g];
  // the caller's x_hi arrays are the field the trace reads (updated in place, see moray.h)
  double* x64 = (double*)c->eq_x.p;
  double* dmin = (double*)c->eq_dx.p;
  double* lim = (double*)c->ev_lim.p;
  const unsigned char* skip = ng > 1 ? (const unsigned char*)c->eq_skip.p : nullptr;
  for (int q = 0; q < ng; ++q)
    if (!hip_ok(c, launch_widen(c->stream, c->num_cu, prob->grids[q].x_hi, x64 + U.off[q], U.off[q + 1] - U.off[q]),
                "evolution start"))
      return MORAY_EDEVICE;
  moray_result mid{};
  mid.k_ph = (double*)c->eq_kph.p;
  mid.heating = (double*)c->eq_heat.p;
  const unsigned mid_flags = flags | MORAY_OUT_ON_DEVICE;
  std::vector<double> gmin(ng);
  double t = 0.0, dt_prev = 0.0;
  int k = 0;
  while (t < ep->t_end && k < ep->max_steps) {
    if ((st = moray_trace(c, prob, 1, mid_flags, &mid)) != MORAY_OK) return st;
    // each grid's limits, smoothed within the grid; the step is the smallest
    for (int q = 0; q < ng; ++q) {
      const moray_grid& G = prob->grids[q];
      if (!hip_ok(c, launch_step_limit(c->stream, c->num_cu, mid.k_ph + U.off[q], G.n_h, x64 + U.off[q], G.nx, G.ny,
                                       G.nz, ep->alpha_b, sigma_bar, G.dx_cm, ep->eps_ion, ep->tau_front, ep->dt_max,
                                       q == 0 ? skip : nullptr, lim + U.off[q], dmin + q * stride),
                  "evolution step") ||
          !hip_ok(c, hipMemcpyAsync(&gmin[q], dmin + q * stride, 8, hipMemcpyDeviceToHost, c->stream), "copy"))
        return MORAY_EDEVICE;
    }
    if (!hip_ok(c, hipStreamSynchronize(c->stream), "synchronize")) return MORAY_EDEVICE;
    double dt = *std::min_element(gmin.begin(), gmin.end());
    if (k > 0) dt = std::min(dt, 2.0 * dt_prev);          // Eq. dtchange
    dt = std::min(dt, std::min(ep->dt_max, ep->t_end - t));
    for (int q = 0; q < ng; ++q) {
      const moray_grid& G = prob->grids[q];
      if (!hip_ok(c, launch_evolve_update(c->stream, c->num_cu, mid.k_ph + U.off[q], G.n_h, x64 + U.off[q],
                                          const_cast<float*>(G.x_hi), U.off[q + 1] - U.off[q], ep->alpha_b, dt,
                                          q == 0 ? skip : nullptr),
                  "evolution update"))
        return MORAY_EDEVICE;
    }
    t += dt;
    dt_prev = dt;
    if (dt_steps) dt_steps[k] = dt;
    ++k;
  }
  if ((st = moray_trace(c, prob, 1, flags, out)) != MORAY_OK) return st;
  if (x_out && (!hip_ok(c, hipMemcpyAsync(x_out, x64, (size_t)n * 8, hipMemcpyDeviceToDevice, c->stream), "copy") ||
                !hip_ok(c, hipStreamSynchronize(c->stream), "synchronize")))
    return MORAY_EDEVICE;
  if (steps) *steps = k;
  if (t_reached) *t_reached = t;
  return MORAY_OK;
}

moray_status moray_autotune(moray_ctx* c, const moray_problem* probs, int n_probs, unsigned flags, int max_trials,
                            moray_tune_result* out) {
  if (!c) return MORAY_EINVAL;
  if (!probs || n_probs < 1) return fail(c, MORAY_EINVAL, "need n_probs >= 1 problems");
  if (flags & ~(MORAY_FIELDS_ON_DEVICE | MORAY_OUT_ON_DEVICE)) return fail(c, MORAY_EINVAL, "unknown flags");
  for (int i = 0; i < n_probs; ++i) {
    const moray_status s = validate(c, probs[i], i);
    if (s != MORAY_OK) return s;
  }
  if (engine_busy(c)) return fail(c, MORAY_EBUSY, "asynchronous solves are still running on this context");
  if (!hip_ok(c, hipSetDevice(c->device), "hipSetDevice")) return MORAY_EDEVICE;
  // scratch results on the device
  long long cells = 0;
  for (int i = 0; i < n_probs; ++i)
    for (int q = 0; q < probs[i].n_grids; ++q)
      cells += (long long)probs[i].grids[q].nx * probs[i].grids[q].ny * probs[i].grids[q].nz;
  DevBuf scratch;
  moray_status st = ensure(c, scratch, (size_t)cells * 16, "autotune results");
  if (st != MORAY_OK) return st;
  std::vector<moray_result> res(n_probs);
  {
    long long off = 0;
    for (int i = 0; i < n_probs; ++i) {
      long long nc = 0;
      for (int q = 0; q < probs[i].n_grids; ++q)
        nc += (long long)probs[i].grids[q].nx * probs[i].grids[q].ny * probs[i].grids[q].nz;
      res[i] = moray_result{};
      res[i].k_ph = (double*)scratch.p + off;
      res[i].heating = (double*)scratch.p + cells + off;
      off += nc;
    }
  }
  const unsigned fl = flags | MORAY_OUT_ON_DEVICE;
  const int keep_chunk = c->chunk, keep_refill = c->refill, keep_reserve = c->reserve_user, keep_bpc = c->blocks_per_cu;
  int trials = 0;
  // fastest of three solves (the second captures a graph, the third replays it)
  auto timed = [&](double& ms) -> moray_status {
    ms = 1e300;
    for (int r = 0; r < 3; ++r) {
      const auto t0 = std::chrono::steady_clock::now();
      const moray_status s = moray_trace(c, probs, n_probs, fl, res.data());
      if (s != MORAY_OK) return s;
      ms = std::min(ms, std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
    }
    ++trials;
    return MORAY_OK;
  };
  double first = 0.0;
  st = timed(first);
  double best = first;
  int bpc_max = 1;
  if (st == MORAY_OK && (trace_occupancy(c->precision, c->cache, &bpc_max) != hipSuccess || bpc_max < 1)) bpc_max = 1;
  struct Knob {
    int* field;
    std::vector<int> values;
  };
  std::vector<int> bpcs;
  for (int b = 1; b <= bpc_max; ++b) bpcs.push_back(b);
  std::vector<Knob> knobs = {{&c->chunk, {128, 256, 512, 1024}},
                             {&c->refill, {8, 16, 24, 64}},
                             {&c->reserve_user, {64, 128, 256}},
                             {&c->blocks_per_cu, bpcs}};
  for (Knob& k : knobs) {
    if (st != MORAY_OK) break;
    const int start = *k.field;
    int pick = start;
    for (int v : k.values) {
      if (v == start) continue;
      if (max_trials > 0 && trials >= max_trials) break;
      *k.field = v;
      double ms = 0.0;
      st = timed(ms);
      if (st != MORAY_OK) break;
      if (ms < best) {
        best = ms;
        pick = v;
      }
    }
    *k.field = pick;
  }
  release(c, scratch);
  if (st != MORAY_OK) {
    c->chunk = keep_chunk;
    c->refill = keep_refill;
    c->reserve_user = keep_reserve;
    c->blocks_per_cu = keep_bpc;
    return st;
  }
  if (out) {
    out->chunk_rays = c->chunk;
    out->refill_lanes = c->refill;
    out->reserve_rays = c->reserve_user;
    out->waves_per_cu = c->blocks_per_cu * (kTraceBlock / kWave);
    out->first_ms = first;
    out->best_ms = best;
    out->trials = trials;
  }
  c->err = "no error";
  return MORAY_OK;
}

}  // extern "C"
