// Serving engine: continuous batching of trace requests on one context.
//
// moray_trace_async queues problems; a host thread per context runs the
// launch loop. Every trip is one launch generation of the trace kernel: rays
// of every running problem advance by one HEALPix level, and problems that
// were admitted since the last trip start with their seed rays in the same
// launch (a ray's level is its tree's seed level plus the generations since
// the tree was admitted). Between launches the engine
//   * admits pending problems in arrival order while their cells, absorber
//     columns, accumulators, table slots and their share of the ray queue fit
//     the context's HBM budget (all problems admitted together share one seed
//     level and one contiguous block of tree slots);
//   * retires every problem none of whose trees split in the last launch (it
//     has no rays left): finalize writes its k_ph and heating, its totals are
//     filled in, its ticket is released and its memory returns to the pools.
// Problems therefore join and leave a running batch at launch boundaries, and
// their rays share every launch. A queue overflow restarts the problems that
// were running (their partial results are discarded) with a smaller share of
// the queue; results never depend on what else is in the batch beyond the
// order of floating-point additions into each cell.
#include "moray_internal.h"

#include <time.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>

using namespace moray;

namespace moray {
namespace {

constexpr int kServeMaxGroups = 64;
constexpr double kLoadFrac = 0.75;         // share of the ray queue admitted problems may claim

double now_s() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

// First-fit allocator of integer ranges inside [0, cap).
class RangeAlloc {
 public:
  void reset(long long cap) {
    free_.clear();
    if (cap > 0) free_[0] = cap;
  }
  long long alloc(long long n) {
    if (n <= 0) return 0;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      const long long start = it->first, len = it->second;
      free_.erase(it);
      if (len > n) free_[start + n] = len - n;
      return start;
    }
    return -1;
  }
  void release(long long start, long long n) {
    if (n <= 0 || start < 0) return;
    auto next = free_.lower_bound(start);
    if (next != free_.end() && start + n == next->first) {
      n += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == start) {
        prev->second += n;
        return;
      }
    }
    free_[start] = n;
  }

 private:
  std::map<long long, long long> free_;
};

struct Ticket {
  int remaining = 0;
  moray_status status = MORAY_OK;
  std::string err;
  double deadline = HUGE_VAL;    // CLOCK_MONOTONIC seconds (moray_set_deadline)
  bool cancel = false;           // moray_cancel
};

// One problem of an asynchronous call, with its own copies of the descriptors.
struct ServeProblem {
  unsigned long long ticket = 0;
  unsigned flags = 0;
  moray_result* out = nullptr;
  std::vector<moray_grid> grids;
  std::vector<moray_source> sources;
  std::vector<double> energy, sigma, frac;
  moray_spectrum spec{};
  moray_problem prob{};
  double bound = 0.0;            // ray-queue share: rays one level of all its trees can hold
  long long ncells = 0, nacc = 0;
  int ngroups = 0, ntrees = 0, l0 = 0;
  unsigned max_steps = 64;
  // placement while admitted
  int pslot = -1, gbase = -1, tbase = -1;
  long long cbase = -1, abase = -1;
  int gen0 = 0, launches = 0;
  DevBuf fields, outs;           // device copies of host fields / host results
  std::vector<unsigned long long> splits_seen;
  unsigned long long peak = 0;
  double t_admit = 0.0;
  int restarts = 0;
};

// Ray-queue share of a problem for admission: the largest level population
// of one tree measured on lognormal grids of 64^3..256^3 is 6-14 rays per
// unit of face area (N^2); 4 phi_c per unit, capped by the pixel count,
// covers it. An underestimate only costs a restart.
double serve_rays_estimate(const moray_problem& P) {
  const int lr = reach_level(P);
  double face = 0.0;
  for (int q = 0; q < P.n_grids; ++q) {
    const moray_grid& G = P.grids[q];
    face += ((double)G.nx * G.ny + (double)G.ny * G.nz + (double)G.nz * G.nx) / 3.0;
  }
  const double per_tree = std::min(std::ldexp(12.0, 2 * lr), 4.0 * std::max(P.params.phi_c, 1.0) * face + 256.0);
  return per_tree * (double)P.n_sources * (double)P.spectrum->n_groups;
}

}  // namespace

struct Engine {
  moray_ctx* c = nullptr;
  std::thread th;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  moray_status fatal = MORAY_OK;
  std::string fatal_msg;
  std::deque<ServeProblem*> pending;       // under mu
  std::map<unsigned long long, Ticket> tickets;
  unsigned long long next_ticket = 1;
  int in_flight = 0;                        // pending + running problems, under mu

  // engine thread only
  std::vector<ServeProblem*> running;
  bool fp32 = true;
  size_t rsz = 4;
  long long cells_cap = 0, acc_cap = 0;
  int grid_cap = 4096, prob_cap = 1024, tree_cap = 1 << 16;
  RangeAlloc cells, accs, gslots, pslots, tslots;
  DevBuf kappa, acc, grids, probs, sgs, stats, ctr, eexc, fblocks, partial;
  DevBuf qpix[2], qsg[2], qr[2], qP[2];
  size_t qcap = 0;
  int nseg = 1;
  unsigned long long seg_cap = 0, reserve = 4;
  GridDev* hgrids = nullptr;
  ProblemDev* hprobs = nullptr;
  SgDev* hsgs = nullptr;
  double* heexc = nullptr;
  SgStats* hstats = nullptr;
  Counters* hctr = nullptr;
  void* hfin = nullptr;                     // finalize blocks out, partial sums back
  size_t hfin_bytes = 0;
  int gen = 0;
  double load = 0.0, load_frac = 0.75;     // queue share in use, and the admission limit (kLoadFrac when
                                           // clean; halved by overflows, restored by clean generations)
  std::string err;                          // last engine-side error (engine thread only)
};

namespace {

// Error helpers of the engine thread: they write the engine's own message,
// which reaches the caller through its ticket.
bool eok(Engine* E, hipError_t e, const char* what) {
  if (e == hipSuccess) return true;
  E->err = std::string(what) + ": " + hipGetErrorString(e);
  return false;
}

moray_status efail(Engine* E, moray_status s, const std::string& msg) {
  E->err = msg;
  return s;
}

// Grow-only device buffer inside the context's budget (engine thread; the
// caller cannot allocate on this context while the engine has work).
moray_status eensure(Engine* E, DevBuf& b, size_t bytes, const char* what) {
  moray_ctx* c = E->c;
  if (bytes <= b.bytes) return MORAY_OK;
  bytes = (bytes + 255) & ~size_t(255);
  if (c->allocated - b.bytes + bytes > c->budget)
    return efail(E, MORAY_ENOMEM, std::string("HBM budget exceeded allocating ") + what);
  release(c, b);
  if (hipMalloc(&b.p, bytes) != hipSuccess) {
    b.p = nullptr;
    return efail(E, MORAY_ENOMEM, std::string("hipMalloc failed for ") + what);
  }
  b.bytes = bytes;
  c->allocated += bytes;
  return MORAY_OK;
}

void free_pinned(void*& p) {
  if (p) (void)hipHostFree(p);
  p = nullptr;
}

void engine_release_device(Engine* E) {
  moray_ctx* c = E->c;
  DevBuf* all[] = {&E->kappa, &E->acc, &E->grids, &E->probs, &E->sgs, &E->stats, &E->ctr, &E->eexc, &E->fblocks,
                   &E->partial};
  for (DevBuf* b : all) release(c, *b);
  for (int i = 0; i < 2; ++i) {
    release(c, E->qpix[i]);
    release(c, E->qsg[i]);
    release(c, E->qr[i]);
    release(c, E->qP[i]);
  }
  void* pins[] = {E->hgrids, E->hprobs, E->hsgs, E->heexc, E->hstats, E->hctr, E->hfin};
  for (void* p : pins) free_pinned(p);
  E->hgrids = nullptr; E->hprobs = nullptr; E->hsgs = nullptr; E->heexc = nullptr;
  E->hstats = nullptr; E->hctr = nullptr; E->hfin = nullptr;
}

// Device pools of the engine, sized from what the context's budget has left.
moray_status engine_setup(moray_ctx* c, Engine* E) {
  E->fp32 = c->precision == MORAY_FP32_ACC64;
  E->rsz = E->fp32 ? sizeof(float) : sizeof(double);
  const double avail = c->budget > c->allocated ? (double)(c->budget - c->allocated) : 0.0;
  const double per_ray = 2.0 * (sizeof(uint64_t) + sizeof(uint32_t) + 2 * sizeof(double));
  E->qcap = c->queue_cap_user ? c->queue_cap_user
                              : (size_t)std::min(std::max(avail * 0.3 / per_ray, 65536.0), (double)(1u << 28));
  E->qcap = std::max<size_t>(E->qcap, 256);
  E->cells_cap = (long long)std::min(std::max(avail * 0.15 / (double)E->rsz, 65536.0), (double)(1 << 28));
  E->acc_cap = (long long)std::min(std::max(avail * 0.3 / 8.0, 262144.0), (double)(1u << 31));
  E->cells.reset(E->cells_cap);
  E->accs.reset(E->acc_cap);
  E->gslots.reset(E->grid_cap);
  E->pslots.reset(E->prob_cap);
  E->tslots.reset(E->tree_cap);
  moray_status st;
  if ((st = ensure(c, E->kappa, (size_t)E->cells_cap * E->rsz, "serving absorber columns")) ||
      (st = ensure(c, E->acc, (size_t)E->acc_cap * 8, "serving accumulators")) ||
      (st = ensure(c, E->grids, (size_t)E->grid_cap * sizeof(GridDev), "serving grid table")) ||
      (st = ensure(c, E->probs, (size_t)E->prob_cap * sizeof(ProblemDev), "serving problem table")) ||
      (st = ensure(c, E->sgs, (size_t)E->tree_cap * sizeof(SgDev), "serving tree table")) ||
      (st = ensure(c, E->stats, (size_t)E->tree_cap * sizeof(SgStats), "serving statistics")) ||
      (st = ensure(c, E->ctr, sizeof(Counters), "serving counters")) ||
      (st = ensure(c, E->eexc, (size_t)E->prob_cap * kServeMaxGroups * 8, "serving group energies")))
    return st;
  for (int i = 0; i < 2; ++i) {
    if ((st = ensure(c, E->qpix[i], E->qcap * 8, "serving ray queue")) ||
        (st = ensure(c, E->qsg[i], E->qcap * 4, "serving ray queue")) ||
        (st = ensure(c, E->qr[i], E->qcap * 8, "serving ray queue")) ||
        (st = ensure(c, E->qP[i], E->qcap * 8, "serving ray queue")))
      return st;
  }
  auto pin = [&](void** p, size_t bytes) { return hipHostMalloc(p, bytes, hipHostMallocDefault) == hipSuccess; };
  if (!pin((void**)&E->hgrids, (size_t)E->grid_cap * sizeof(GridDev)) ||
      !pin((void**)&E->hprobs, (size_t)E->prob_cap * sizeof(ProblemDev)) ||
      !pin((void**)&E->hsgs, (size_t)E->tree_cap * sizeof(SgDev)) ||
      !pin((void**)&E->heexc, (size_t)E->prob_cap * kServeMaxGroups * 8) ||
      !pin((void**)&E->hstats, (size_t)E->tree_cap * sizeof(SgStats)) || !pin((void**)&E->hctr, sizeof(Counters)))
    return fail(c, MORAY_ENOMEM, "pinned host allocation failed");
  E->nseg = queue_segments(E->qcap);
  E->seg_cap = E->qcap / (size_t)E->nseg;
  const double waves = (double)std::max(1, c->num_cu * c->blocks_per_cu) * (kTraceBlock / kWave);
  E->reserve = (unsigned long long)std::min<double>((double)kReserveMax, (double)E->qcap / (8.0 * waves));
  E->reserve = std::max<unsigned long long>(4, E->reserve & ~3ull);
  if (!hip_ok(c, launch_reset(c->stream, (Counters*)E->ctr.p, (SgStats*)E->stats.p, 0), "reset") ||
      !hip_ok(c, hipStreamSynchronize(c->stream), "synchronize"))
    return MORAY_EDEVICE;
  return MORAY_OK;
}

void finish_ticket(Engine* E, ServeProblem* p, moray_status st, const std::string& msg) {
  std::lock_guard<std::mutex> lk(E->mu);
  auto it = E->tickets.find(p->ticket);
  if (it != E->tickets.end()) {
    Ticket& t = it->second;
    if (st != MORAY_OK && t.status == MORAY_OK) {
      t.status = st;
      t.err = msg;
    }
    --t.remaining;
  }
  --E->in_flight;
  E->cv_done.notify_all();
}

void unplace(Engine* E, ServeProblem* p) {
  moray_ctx* c = E->c;
  if (p->cbase >= 0) E->cells.release(p->cbase, p->ncells);
  if (p->abase >= 0) E->accs.release(p->abase, p->nacc);
  if (p->gbase >= 0) E->gslots.release(p->gbase, (long long)p->grids.size());
  if (p->pslot >= 0) E->pslots.release(p->pslot, 1);
  if (p->tbase >= 0) E->tslots.release(p->tbase, p->ntrees);
  p->cbase = p->abase = -1;
  p->gbase = p->pslot = p->tbase = -1;
  release(c, p->fields);
  release(c, p->outs);
}

// Cells, accumulators, table slots and staging for one problem (not its trees).
// (A problem alone is always tried, whatever its queue share.)
bool place(Engine* E, ServeProblem* p) {
  if (E->load > 0.0 && E->load + p->bound > E->load_frac * (double)E->qcap) return false;
  p->cbase = E->cells.alloc(p->ncells);
  p->abase = E->accs.alloc(p->nacc);
  p->gbase = (int)E->gslots.alloc((long long)p->grids.size());
  p->pslot = (int)E->pslots.alloc(1);
  bool ok = p->cbase >= 0 && p->abase >= 0 && p->gbase >= 0 && p->pslot >= 0;
  if (ok && !(p->flags & MORAY_FIELDS_ON_DEVICE))
    ok = eensure(E, p->fields, (size_t)p->ncells * 8, "request fields") == MORAY_OK;
  if (ok && !(p->flags & MORAY_OUT_ON_DEVICE))
    ok = eensure(E, p->outs, (size_t)p->ncells * 16, "request results") == MORAY_OK;
  if (!ok) unplace(E, p);     // releases only what was obtained (failed pools hold -1)
  return ok;
}

// Table entries of an admitted problem whose trees start at slot tbase, seeded in generation gen.
moray_status write_tables(Engine* E, ServeProblem* p) {
  moray_ctx* c = E->c;
  hipStream_t s = c->stream;
  const moray_problem& P = p->prob;
  ProblemDev& pd = E->hprobs[p->pslot];
  pd = ProblemDev{};
  pd.root_grid = p->gbase;
  pd.n_groups = p->ngroups;
  pd.cell_off = p->cbase;
  pd.n_cells = p->ncells;
  pd.acc_off = p->abase;
  pd.eexc_off = p->pslot * kServeMaxGroups;
  for (int g = 0; g < p->ngroups; ++g)
    E->heexc[pd.eexc_off + g] = (p->energy[g] - p->spec.e_ion_ev) * kEvErgConst;
  long long off = p->cbase;
  const float* fbuf = (const float*)p->fields.p;
  double* obuf = (double*)p->outs.p;
  long long within = 0;
  for (size_t q = 0; q < p->grids.size(); ++q) {
    const moray_grid& G = p->grids[q];
    GridDev& d = E->hgrids[p->gbase + q];
    d = GridDev{};
    d.nx = G.nx; d.ny = G.ny; d.nz = G.nz;
    d.is_child = q > 0;
    d.ox = q > 0 ? G.offset[0] : 0;
    d.oy = q > 0 ? G.offset[1] : 0;
    d.oz = q > 0 ? G.offset[2] : 0;
    d.problem = p->pslot;
    d.cell_off = off;
    d.dx_cm = G.dx_cm;
    const long long nc = (long long)G.nx * G.ny * G.nz;
    if (p->flags & MORAY_FIELDS_ON_DEVICE) {
      d.n_h = G.n_h;
      d.x_hi = G.x_hi;
    } else {
      d.n_h = fbuf + within;
      d.x_hi = fbuf + p->ncells + within;
      if (!eok(E, hipMemcpyAsync((void*)d.n_h, G.n_h, nc * 4, hipMemcpyHostToDevice, s), "upload") ||
          !eok(E, hipMemcpyAsync((void*)d.x_hi, G.x_hi, nc * 4, hipMemcpyHostToDevice, s), "upload"))
        return MORAY_EDEVICE;
    }
    if (p->flags & MORAY_OUT_ON_DEVICE) {
      d.out_kph = p->out->k_ph + within;
      d.out_heat = p->out->heating + within;
    } else {
      d.out_kph = obuf + within;
      d.out_heat = obuf + p->ncells + within;
    }
    off += nc;
    within += nc;
  }
  const double npix0 = std::ldexp(12.0, 2 * P.params.level_init);
  const GridDev& rg = E->hgrids[p->gbase];
  int k = 0;
  for (int si = 0; si < P.n_sources; ++si) {
    for (int g = 0; g < p->ngroups; ++g, ++k) {
      SgDev& d = E->hsgs[p->tbase + k];
      d = SgDev{};
      const moray_source& S = P.sources[si];
      d.sx = S.x; d.sy = S.y; d.sz = S.z;
      d.P0 = p->frac[g] * S.ndot / npix0;
      d.pmin0 = P.params.p_min_frac * d.P0;
      d.sigma64 = p->sigma[g];
      d.sigma32 = (float)p->sigma[g];
      d.four_pi_phi_c = 4.0 * kPiConst * P.params.phi_c;
      d.split_t2_base = P.params.phi_c > 0.0 ? (float)(12.0 / (4.0 * kPiConst * P.params.phi_c)) : FLT_MAX;
      d.acc_slot = pd.acc_off + (long long)g * pd.n_cells - pd.cell_off;
      d.problem = p->pslot;
      d.covering = P.params.covering != 0;
      d.root_grid = p->gbase;
      d.rnx = rg.nx; d.rny = rg.ny; d.rnz = rg.nz;
      d.rcell_off = rg.cell_off;
      d.level_init = P.params.level_init;
      d.level_max = P.params.phi_c > 0.0 ? P.params.level_max : P.params.level_init;
      d.gen0 = p->gen0;
    }
  }
  auto up = [&](DevBuf& b, size_t first, const void* src, size_t bytes) {
    return bytes == 0 ||
           eok(E, hipMemcpyAsync((char*)b.p + first, src, bytes, hipMemcpyHostToDevice, s), "table upload");
  };
  if (!up(E->grids, (size_t)p->gbase * sizeof(GridDev), E->hgrids + p->gbase, p->grids.size() * sizeof(GridDev)) ||
      !up(E->probs, (size_t)p->pslot * sizeof(ProblemDev), E->hprobs + p->pslot, sizeof(ProblemDev)) ||
      !up(E->eexc, (size_t)pd.eexc_off * 8, E->heexc + pd.eexc_off, (size_t)p->ngroups * 8) ||
      !up(E->sgs, (size_t)p->tbase * sizeof(SgDev), E->hsgs + p->tbase, (size_t)p->ntrees * sizeof(SgDev)))
    return MORAY_EDEVICE;
  hipError_t e =
      E->fp32 ? launch_prep<float>(s, c->num_cu, (GridDev*)E->grids.p + p->gbase, (int)p->grids.size(), p->gbase,
                                   (ProblemDev*)E->probs.p, p->cbase, p->cbase + p->ncells, (float*)E->kappa.p,
                                   (double*)E->acc.p, (Counters*)E->ctr.p)
              : launch_prep<double>(s, c->num_cu, (GridDev*)E->grids.p + p->gbase, (int)p->grids.size(), p->gbase,
                                    (ProblemDev*)E->probs.p, p->cbase, p->cbase + p->ncells, (double*)E->kappa.p,
                                    (double*)E->acc.p, (Counters*)E->ctr.p);
  if (!eok(E, e, "prep") || !eok(E, launch_reset_stats(s, (SgStats*)E->stats.p, p->tbase, p->ntrees), "reset"))
    return MORAY_EDEVICE;
  p->splits_seen.assign(p->ntrees, 0);
  p->launches = 0;
  p->peak = 0;
  return MORAY_OK;
}

// Finalize the retiring problems and fill in their results.
moray_status retire(Engine* E, std::vector<ServeProblem*>& done) {
  moray_ctx* c = E->c;
  hipStream_t s = c->stream;
  if (done.empty()) return MORAY_OK;
  std::vector<FinalBlock> fb;
  std::vector<int> first(done.size() + 1, 0);
  const long long per = (long long)kFinalBlock * kFinalCellsPerThread;
  for (size_t i = 0; i < done.size(); ++i) {
    first[i] = (int)fb.size();
    ServeProblem* p = done[i];
    for (size_t q = 0; q < p->grids.size(); ++q) {
      const GridDev& G = E->hgrids[p->gbase + q];
      const long long nc = (long long)G.nx * G.ny * G.nz;
      for (long long f = 0; f < nc; f += per) fb.push_back({p->gbase + (int)q, (int)std::min(per, nc - f), f});
    }
  }
  first[done.size()] = (int)fb.size();
  const size_t nb = fb.size();
  const size_t need = nb * (sizeof(FinalBlock) + 8);
  if (need > E->hfin_bytes) {
    free_pinned(E->hfin);
    E->hfin_bytes = 0;
    if (hipHostMalloc(&E->hfin, need, hipHostMallocDefault) != hipSuccess)
      return efail(E, MORAY_ENOMEM, "pinned host allocation failed");
    E->hfin_bytes = need;
  }
  FinalBlock* hfb = (FinalBlock*)E->hfin;
  double* hpart = (double*)((char*)E->hfin + nb * sizeof(FinalBlock));
  std::copy(fb.begin(), fb.end(), hfb);
  moray_status st;
  if ((st = eensure(E, E->fblocks, std::max<size_t>(1, nb) * sizeof(FinalBlock), "finalize blocks")) ||
      (st = eensure(E, E->partial, std::max<size_t>(1, nb) * 8, "partial sums")))
    return st;
  if (nb && (!eok(E, hipMemcpyAsync(E->fblocks.p, hfb, nb * sizeof(FinalBlock), hipMemcpyHostToDevice, s), "upload") ||
             !eok(E, launch_finalize(s, (int)nb, (GridDev*)E->grids.p, (ProblemDev*)E->probs.p,
                                        (FinalBlock*)E->fblocks.p, (double*)E->acc.p, (double*)E->eexc.p,
                                        (double*)E->partial.p, (Counters*)E->ctr.p),
                    "finalize") ||
             !eok(E, hipMemcpyAsync(hpart, E->partial.p, nb * 8, hipMemcpyDeviceToHost, s), "copy")))
    return MORAY_EDEVICE;
  for (ServeProblem* p : done) {
    if (!(p->flags & MORAY_OUT_ON_DEVICE)) {
      const double* ob = (const double*)p->outs.p;
      if (!eok(E, hipMemcpyAsync(p->out->k_ph, ob, p->ncells * 8, hipMemcpyDeviceToHost, s), "copy results") ||
          !eok(E, hipMemcpyAsync(p->out->heating, ob + p->ncells, p->ncells * 8, hipMemcpyDeviceToHost, s),
                  "copy results"))
        return MORAY_EDEVICE;
    }
  }
  if (!eok(E, hipStreamSynchronize(s), "synchronize")) return MORAY_EDEVICE;
  const double t = now_s();
  for (size_t i = 0; i < done.size(); ++i) {
    ServeProblem* p = done[i];
    moray_result& R = *p->out;
    const moray_problem& P = p->prob;
    R.emitted = R.absorbed = R.escaped = R.truncated = 0.0;
    R.segments = R.rays_seeded = R.splits = R.rays_escaped = R.rays_truncated = 0;
    R.thin_segments = 0;
    for (int b = first[i]; b < first[i + 1]; ++b) R.absorbed += hpart[b];
    int k = 0;
    for (int si = 0; si < P.n_sources; ++si) {
      for (int g = 0; g < p->ngroups; ++g, ++k) {
        const SgStats& S = E->hstats[p->tbase + k];
        R.emitted += p->frac[g] * P.sources[si].ndot;
        R.escaped += S.esc_P;
        R.truncated += S.trunc_P;
        R.segments += S.segs;
        R.splits += S.splits;
        R.rays_escaped += S.n_esc;
        R.rays_truncated += S.n_trunc;
        R.rays_seeded += (unsigned long long)std::ldexp(12.0, 2 * P.params.level_init);
        if (R.escaped_sg) R.escaped_sg[si * p->ngroups + g] = S.esc_P;
      }
    }
    R.peak_level_rays = p->peak;
    R.trace_ms = 0.0;
    R.trace_launches = p->launches;
    R.t_admit = p->t_admit;
    R.t_done = t;
    R.from_graph = 0;
  }
  for (ServeProblem* p : done) {
    E->load -= p->bound;
    unplace(E, p);
    finish_ticket(E, p, MORAY_OK, "");
    delete p;
  }
  if (E->running.empty()) {
    E->load = 0.0;
    E->load_frac = kLoadFrac;
  }
  return MORAY_OK;
}

// Give back a set of problems to the front of the pending queue (restart).
void requeue(Engine* E, std::vector<ServeProblem*>& ps) {
  std::lock_guard<std::mutex> lk(E->mu);
  for (auto it = ps.rbegin(); it != ps.rend(); ++it) {
    E->load -= (*it)->bound;
    unplace(E, *it);
    E->pending.push_front(*it);
  }
  if (E->load < 0.0) E->load = 0.0;
}

void fail_all(Engine* E, moray_status st, const std::string& msg) {
  std::vector<ServeProblem*> all = E->running;
  E->running.clear();
  {
    std::lock_guard<std::mutex> lk(E->mu);
    E->fatal = st;
    E->fatal_msg = msg;
    for (ServeProblem* p : E->pending) all.push_back(p);
    E->pending.clear();
  }
  for (ServeProblem* p : all) {
    unplace(E, p);
    finish_ticket(E, p, st, msg);
    delete p;
  }
}

// Status a problem must leave with at this boundary (MORAY_OK: none), from its
// ticket's cancel flag and deadline. Under E->mu.
moray_status leave_status(Engine* E, const ServeProblem* p, double t) {
  auto it = E->tickets.find(p->ticket);
  if (it == E->tickets.end()) return MORAY_OK;
  if (it->second.cancel) return MORAY_ECANCELED;
  if (t >= it->second.deadline) return MORAY_ETIMEOUT;
  return MORAY_OK;
}

const char* leave_message(moray_status st) {
  return st == MORAY_ECANCELED ? "the solve was cancelled" : "the solve passed its deadline";
}

// At a generation boundary: pending problems of cancelled or expired tickets
// are dropped; running ones have their rays removed from the queue that the
// next launch reads (row `row`), and their memory returns to the pools.
// Returns false on a device error (the engine then fails everything).
bool drop_leavers(Engine* E, int row) {
  const double t = now_s();
  std::vector<std::pair<ServeProblem*, moray_status>> gone, stop_running;
  {
    std::lock_guard<std::mutex> lk(E->mu);
    for (auto it = E->pending.begin(); it != E->pending.end();) {
      const moray_status st = leave_status(E, *it, t);
      if (st != MORAY_OK) {
        gone.push_back({*it, st});
        it = E->pending.erase(it);
      } else {
        ++it;
      }
    }
    for (ServeProblem* p : E->running) {
      const moray_status st = leave_status(E, p, t);
      if (st != MORAY_OK) stop_running.push_back({p, st});
    }
  }
  for (auto& [p, st] : gone) {
    finish_ticket(E, p, st, leave_message(st));
    delete p;
  }
  if (stop_running.empty()) return true;
  moray_ctx* c = E->c;
  for (size_t b = 0; b < stop_running.size(); b += kDropRanges) {
    int lo[kDropRanges], hi[kDropRanges], n = 0;
    for (size_t k = b; k < stop_running.size() && n < kDropRanges; ++k, ++n) {
      lo[n] = stop_running[k].first->tbase;
      hi[n] = stop_running[k].first->tbase + stop_running[k].first->ntrees;
    }
    if (!eok(E, launch_drop_trees(c->stream, (uint32_t*)E->qsg[row].p, (Counters*)E->ctr.p, row, E->seg_cap,
                                  E->nseg, lo, hi, n),
             "drop rays"))
      return false;
  }
  if (!eok(E, hipStreamSynchronize(c->stream), "synchronize")) return false;
  for (auto& [p, st] : stop_running) {
    E->running.erase(std::find(E->running.begin(), E->running.end(), p));
    E->load -= p->bound;
    unplace(E, p);
    finish_ticket(E, p, st, leave_message(st));
    delete p;
  }
  if (E->running.empty()) {
    E->load = 0.0;
    E->load_frac = kLoadFrac;
  }
  return true;
}

// One trip of the launch loop. Returns false when the engine must stop.
bool trip(Engine* E) {
  moray_ctx* c = E->c;
  hipStream_t s = c->stream;
  std::vector<ServeProblem*> admitted;
  {
    std::unique_lock<std::mutex> lk(E->mu);
    E->cv_work.wait(lk, [&] { return E->stop || !E->pending.empty() || !E->running.empty(); });
    if (E->stop && E->pending.empty() && E->running.empty()) return false;
  }
  // the next launch reads the queue the last one wrote (row E->gen & 1)
  if (!drop_leavers(E, E->gen & 1)) {
    fail_all(E, MORAY_EDEVICE, E->err);
    return true;
  }
  {
    std::unique_lock<std::mutex> lk(E->mu);
    while (!E->pending.empty()) {
      ServeProblem* p = E->pending.front();
      if (!admitted.empty() && p->l0 != admitted[0]->l0) break;
      if (!place(E, p)) {
        if (E->running.empty() && admitted.empty()) {
          // it cannot fit even alone
          E->pending.pop_front();
          lk.unlock();
          finish_ticket(E, p, MORAY_ENOMEM, "request does not fit the serving pools");
          delete p;
          lk.lock();
          continue;
        }
        break;
      }
      E->pending.pop_front();
      admitted.push_back(p);
      E->load += p->bound;
    }
  }
  // one contiguous block of tree slots for everything admitted now
  int tblock = 0, ttotal = 0;
  while (!admitted.empty()) {
    ttotal = 0;
    for (ServeProblem* p : admitted) ttotal += p->ntrees;
    const long long b = E->tslots.alloc(ttotal);
    if (b >= 0) {
      tblock = (int)b;
      break;
    }
    ServeProblem* last = admitted.back();
    admitted.pop_back();
    if (admitted.empty() && E->running.empty()) {
      E->load -= last->bound;
      unplace(E, last);
      finish_ticket(E, last, MORAY_ENOMEM, "request has more (source, group) trees than the serving tables hold");
      delete last;
      break;
    }
    std::vector<ServeProblem*> back{last};
    requeue(E, back);
  }
  const double t_admit = now_s();
  {
    int t = tblock;
    for (ServeProblem* p : admitted) {
      p->tbase = t;
      t += p->ntrees;
      p->gen0 = E->gen;
      p->t_admit = t_admit;
      const moray_status st = write_tables(E, p);
      if (st != MORAY_OK) {
        fail_all(E, st, E->err);
        for (ServeProblem* q : admitted) {
          unplace(E, q);
          finish_ticket(E, q, st, E->err);
          delete q;
        }
        return true;
      }
    }
  }
  if (!admitted.empty()) {
    // field checks of the new problems: one bad request must not void the launch
    if (!eok(E, hipMemcpyAsync(E->hctr, E->ctr.p, sizeof(Counters), hipMemcpyDeviceToHost, s), "copy") ||
        !eok(E, hipStreamSynchronize(s), "synchronize")) {
      fail_all(E, MORAY_EDEVICE, E->err);
      return true;
    }
    if (E->hctr->err & kErrBadInput) {
      std::vector<ServeProblem*> good;
      for (ServeProblem* p : admitted) {
        const unsigned zero = 0;
        // clear the flag, re-run this problem's checks alone
        if (!eok(E, hipMemcpyAsync(&((Counters*)E->ctr.p)->err, &zero, sizeof zero, hipMemcpyHostToDevice, s), "copy") ||
            !eok(E, hipStreamSynchronize(s), "synchronize") || write_tables(E, p) != MORAY_OK ||
            !eok(E, hipMemcpyAsync(E->hctr, E->ctr.p, sizeof(Counters), hipMemcpyDeviceToHost, s), "copy") ||
            !eok(E, hipStreamSynchronize(s), "synchronize")) {
          fail_all(E, MORAY_EDEVICE, E->err);
          return true;
        }
        if (E->hctr->err & kErrBadInput) {
          E->load -= p->bound;
          unplace(E, p);
          finish_ticket(E, p, MORAY_EINVAL, "a density or neutral fraction is negative, non-finite or x_HI > 1");
          delete p;
        } else {
          good.push_back(p);
        }
      }
      const unsigned zero = 0;
      if (!eok(E, hipMemcpyAsync(&((Counters*)E->ctr.p)->err, &zero, sizeof zero, hipMemcpyHostToDevice, s), "copy") ||
          !eok(E, hipStreamSynchronize(s), "synchronize")) {
        fail_all(E, MORAY_EDEVICE, E->err);
        return true;
      }
      // the surviving problems keep their tree slots; the seed range must stay contiguous
      admitted = good;
      if (!admitted.empty()) {
        std::vector<ServeProblem*> later(admitted.begin() + 1, admitted.end());
        admitted.resize(1);
        requeue(E, later);
      }
    }
  }
  for (ServeProblem* p : admitted) E->running.push_back(p);
  if (E->running.empty()) return true;

  // ---- one launch generation ----
  const int g = E->gen;
  const int cin = g & 1, cout = (g + 1) & 1;
  unsigned max_steps = 64;
  int tlo = E->tree_cap, thi = 0;
  bool cover = false;               // some running problem scales its deposits by the covering factor
  for (ServeProblem* p : E->running) {
    max_steps = std::max(max_steps, p->max_steps);
    cover = cover || p->prob.params.covering != 0;
    if (p->ntrees) {
      tlo = std::min(tlo, p->tbase);
      thi = std::max(thi, p->tbase + p->ntrees);
    }
    ++p->launches;
  }
  const int seed_lo = admitted.empty() ? 0 : admitted.front()->tbase;
  int seed_hi = seed_lo;
  for (ServeProblem* p : admitted) seed_hi = std::max(seed_hi, p->tbase + p->ntrees);
  const int seed_level = admitted.empty() ? 0 : admitted.front()->l0;
  const int blocks = std::max(1, c->num_cu * c->blocks_per_cu);
  const RayQueue qin{(uint64_t*)E->qpix[cin].p, (uint32_t*)E->qsg[cin].p, (double*)E->qr[cin].p, (double*)E->qP[cin].p};
  const RayQueue qout{(uint64_t*)E->qpix[cout].p, (uint32_t*)E->qsg[cout].p, (double*)E->qr[cout].p,
                      (double*)E->qP[cout].p};
  hipError_t e = launch_reset_generation(s, (Counters*)E->ctr.p, cin, cout);
  if (e == hipSuccess) {
    if (E->fp32) {
      TraceArgs<float> A{};
      A.grids = (GridDev*)E->grids.p; A.probs = (ProblemDev*)E->probs.p; A.sgs = (SgDev*)E->sgs.p;
      A.kappa = (float*)E->kappa.p; A.acc = (double*)E->acc.p; A.in = qin; A.out = qout;
      A.seg_cap = E->seg_cap; A.nseg = E->nseg; A.ctr = (Counters*)E->ctr.p; A.stats = (SgStats*)E->stats.p;
      A.gen = g; A.cin = cin; A.cout = cout; A.seed_level = seed_level;
      A.seed_sg_begin = seed_lo; A.seed_sg_end = seed_hi;
      A.chunk = c->chunk; A.refill = c->refill; A.max_steps = max_steps; A.reserve = E->reserve;
      e = launch_trace_level<float>(s, blocks, A, c->cache, cover, false);
    } else {
      TraceArgs<double> A{};
      A.grids = (GridDev*)E->grids.p; A.probs = (ProblemDev*)E->probs.p; A.sgs = (SgDev*)E->sgs.p;
      A.kappa = (double*)E->kappa.p; A.acc = (double*)E->acc.p; A.in = qin; A.out = qout;
      A.seg_cap = E->seg_cap; A.nseg = E->nseg; A.ctr = (Counters*)E->ctr.p; A.stats = (SgStats*)E->stats.p;
      A.gen = g; A.cin = cin; A.cout = cout; A.seed_level = seed_level;
      A.seed_sg_begin = seed_lo; A.seed_sg_end = seed_hi;
      A.chunk = c->chunk; A.refill = c->refill; A.max_steps = max_steps; A.reserve = E->reserve;
      e = launch_trace_level<double>(s, blocks, A, c->cache, cover, false);
    }
  }
  if (!eok(E, e, "trace") ||
      !eok(E, hipMemcpyAsync(E->hctr, E->ctr.p, sizeof(Counters), hipMemcpyDeviceToHost, s), "copy") ||
      (thi > tlo && !eok(E, hipMemcpyAsync(E->hstats + tlo, (SgStats*)E->stats.p + tlo,
                                              (size_t)(thi - tlo) * sizeof(SgStats), hipMemcpyDeviceToHost, s),
                            "copy")) ||
      !eok(E, hipStreamSynchronize(s), "synchronize")) {
    fail_all(E, MORAY_EDEVICE, E->err);
    return false;
  }
  E->gen = g + 1;
  if (E->hctr->err & kErrInternal) {
    fail_all(E, MORAY_EINTERNAL, "a ray exceeded its step bound");
    return false;
  }
  const bool injected = c->overflow_serve_once && E->running.size() > 1;
  if (injected) c->overflow_serve_once = false;
  if ((E->hctr->err & kErrOverflow) || injected) {
    // children were lost: every running problem starts again, with a smaller
    // queue share; one that overflowed alone, or again and again, cannot be served
    std::vector<ServeProblem*> again;
    const bool alone = E->running.size() == 1;
    for (ServeProblem* p : E->running) {
      if (alone || ++p->restarts > 4) {
        E->load -= p->bound;
        unplace(E, p);
        finish_ticket(E, p, MORAY_EQUEUE, "ray queue overflowed; raise queue_capacity or the HBM budget");
        delete p;
      } else {
        again.push_back(p);
      }
    }
    E->running.clear();
    E->load_frac = std::max(0.02, E->load_frac * 0.5);
    if (!eok(E, launch_reset_generation(s, (Counters*)E->ctr.p, cout, cout), "reset")) {
      fail_all(E, MORAY_EDEVICE, E->err);
      return false;
    }
    requeue(E, again);
    return true;
  }
  // a clean generation gives back a quarter of what an overflow took
  E->load_frac = std::min(kLoadFrac, E->load_frac * 1.25);
  unsigned long long pop = 0;
  for (int k = 0; k < E->nseg; ++k) pop += std::min<unsigned long long>(E->hctr->count[cout][k], E->seg_cap);
  std::vector<ServeProblem*> done, still;
  for (ServeProblem* p : E->running) {
    bool live = false;
    for (int k = 0; k < p->ntrees; ++k) {
      const unsigned long long sp = E->hstats[p->tbase + k].splits;
      if (sp != p->splits_seen[k]) live = true;
      p->splits_seen[k] = sp;
    }
    p->peak = std::max(p->peak, pop);
    (live ? still : done).push_back(p);
  }
  E->running = still;
  const moray_status st = retire(E, done);
  if (st != MORAY_OK) {
    for (ServeProblem* p : done) {
      unplace(E, p);
      finish_ticket(E, p, st, E->err);
      delete p;
    }
    fail_all(E, st, E->err);
    return false;
  }
  return true;
}

void engine_main(Engine* E) {
  (void)hipSetDevice(E->c->device);
  while (trip(E)) {
  }
}

ServeProblem* make_problem(const moray_problem& P, unsigned flags, moray_result* out) {
  ServeProblem* p = new ServeProblem();
  p->flags = flags;
  p->out = out;
  p->grids.assign(P.grids, P.grids + P.n_grids);
  if (P.n_sources > 0) p->sources.assign(P.sources, P.sources + P.n_sources);
  const moray_spectrum& Sp = *P.spectrum;
  p->ngroups = Sp.n_groups;
  p->energy.assign(Sp.energy_ev, Sp.energy_ev + Sp.n_groups);
  p->sigma.assign(Sp.sigma_cm2, Sp.sigma_cm2 + Sp.n_groups);
  p->frac.assign(Sp.photon_frac, Sp.photon_frac + Sp.n_groups);
  p->spec = Sp;
  p->spec.energy_ev = p->energy.data();
  p->spec.sigma_cm2 = p->sigma.data();
  p->spec.photon_frac = p->frac.data();
  p->prob = P;
  p->prob.grids = p->grids.data();
  p->prob.sources = p->sources.empty() ? nullptr : p->sources.data();
  p->prob.spectrum = &p->spec;
  p->l0 = P.params.level_init;
  p->ntrees = P.n_sources * Sp.n_groups;
  long long steps = 16;
  for (const moray_grid& G : p->grids) {
    p->ncells += (long long)G.nx * G.ny * G.nz;
    steps += 2LL * (G.nx + G.ny + G.nz);
  }
  p->max_steps = (unsigned)std::min<long long>(steps * 2, 1u << 30);
  p->nacc = p->ncells * p->ngroups;
  p->bound = serve_rays_estimate(p->prob);
  return p;
}

}  // namespace

bool engine_busy(moray_ctx* c) {
  Engine* E = c->engine;
  if (!E) return false;
  std::lock_guard<std::mutex> lk(E->mu);
  return E->in_flight > 0;
}

void engine_stop(moray_ctx* c) {
  Engine* E = c->engine;
  if (!E) return;
  {
    std::lock_guard<std::mutex> lk(E->mu);
    E->stop = true;
  }
  E->cv_work.notify_all();
  if (E->th.joinable()) E->th.join();
  (void)hipSetDevice(c->device);
  engine_release_device(E);
  delete E;
  c->engine = nullptr;
}

}  // namespace moray

extern "C" {

moray_status moray_trace_async(moray_ctx* c, const moray_problem* probs, int n_probs, unsigned flags,
                               moray_result* outs, moray_ticket* ticket) {
  if (!c) return MORAY_EINVAL;
  if (!probs || n_probs < 1 || !outs || !ticket) return fail(c, MORAY_EINVAL, "need problems, results and a ticket");
  if (flags & ~(MORAY_FIELDS_ON_DEVICE | MORAY_OUT_ON_DEVICE)) return fail(c, MORAY_EINVAL, "unknown flags");
  for (int i = 0; i < n_probs; ++i) {
    const moray_status s = validate(c, probs[i], i);
    if (s != MORAY_OK) return s;
    if (!outs[i].k_ph || !outs[i].heating) return fail(c, MORAY_EINVAL, "result buffers are NULL");
    if (outs[i].accel) return fail(c, MORAY_EINVAL, "radiation pressure is computed by moray_trace only");
    if (probs[i].params.tau_thin > 0.0)
      return fail(c, MORAY_EINVAL, "the optically-thin approximation is computed by moray_trace only");
    if (probs[i].spectrum->n_groups > kServeMaxGroups) return fail(c, MORAY_EINVAL, "more than 64 groups");
  }
  if (!c->engine) {
    if (!hip_ok(c, hipSetDevice(c->device), "hipSetDevice")) return MORAY_EDEVICE;
    Engine* E = new Engine();
    E->c = c;
    const moray_status st = engine_setup(c, E);
    if (st != MORAY_OK) {
      engine_release_device(E);
      delete E;
      return st;
    }
    c->engine = E;
    E->th = std::thread(engine_main, E);
  }
  Engine* E = c->engine;
  std::vector<ServeProblem*> ps;
  for (int i = 0; i < n_probs; ++i) ps.push_back(make_problem(probs[i], flags, &outs[i]));
  {
    std::lock_guard<std::mutex> lk(E->mu);
    if (E->fatal != MORAY_OK) {
      for (ServeProblem* p : ps) delete p;
      return fail(c, E->fatal, E->fatal_msg);
    }
    const unsigned long long t = E->next_ticket++;
    Ticket& tk = E->tickets[t];
    tk.remaining = n_probs;
    for (ServeProblem* p : ps) {
      p->ticket = t;
      E->pending.push_back(p);
    }
    E->in_flight += n_probs;
    *ticket = t;
  }
  E->cv_work.notify_all();
  return MORAY_OK;
}

moray_status moray_set_deadline(moray_ctx* c, moray_ticket ticket, double seconds) {
  if (!c) return MORAY_EINVAL;
  if (!(seconds >= 0.0)) return fail(c, MORAY_EINVAL, "the deadline must be a time >= 0 from now");
  Engine* E = c->engine;
  if (!E) return fail(c, MORAY_EINVAL, "unknown ticket");
  {
    std::lock_guard<std::mutex> lk(E->mu);
    auto it = E->tickets.find(ticket);
    if (it == E->tickets.end()) return fail(c, MORAY_EINVAL, "unknown ticket");
    it->second.deadline = now_s() + seconds;
  }
  E->cv_work.notify_all();
  return MORAY_OK;
}

moray_status moray_cancel(moray_ctx* c, moray_ticket ticket) {
  if (!c) return MORAY_EINVAL;
  Engine* E = c->engine;
  if (!E) return fail(c, MORAY_EINVAL, "unknown ticket");
  {
    std::lock_guard<std::mutex> lk(E->mu);
    auto it = E->tickets.find(ticket);
    if (it == E->tickets.end()) return fail(c, MORAY_EINVAL, "unknown ticket");
    it->second.cancel = true;
  }
  E->cv_work.notify_all();
  return MORAY_OK;
}

moray_status moray_query(moray_ctx* c, moray_ticket ticket, int wait_ms) {
  if (!c) return MORAY_EINVAL;
  Engine* E = c->engine;
  if (!E) return fail(c, MORAY_EINVAL, "unknown ticket");
  std::unique_lock<std::mutex> lk(E->mu);
  auto it = E->tickets.find(ticket);
  if (it == E->tickets.end()) return fail(c, MORAY_EINVAL, "unknown ticket");
  auto done = [&] { return it->second.remaining <= 0; };
  if (wait_ms < 0) E->cv_done.wait(lk, done);
  else if (wait_ms > 0) E->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), done);
  if (!done()) return MORAY_EBUSY;
  const moray_status st = it->second.status;
  const std::string msg = it->second.err;
  E->tickets.erase(it);
  if (st != MORAY_OK) c->err = msg;
  return st;
}

}  // extern "C"
