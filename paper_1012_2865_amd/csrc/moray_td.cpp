// Time-dependent rays (section 2.1: a ray halts once it has travelled c dt_P
// and is kept for the next step, section 3.1 step 3j), as a ray pool that
// lives on the device between calls (moray_td_create / moray_td_step /
// moray_td_free).
//
// Every step's sources emit one batch of seed rays (when asked to); a batch
// is a set of (source, group) trees whose rays halt, in a step where the
// batch has completed a steps, at the radius (a + 1) c dt_P. The trees of the
// live batches sit in a ring of `slots` batches: once (a + 1) c dt_P exceeds
// the box diagonal every ray of a batch has left, so a slot is reused after
// `slots` steps. A step is the one-shot launch sequence with two changes:
// before each level's launch, the rays of that level halted in the previous
// step join the level's queue (prefill_level_kernel), and the trace kernel's
// halting variant writes the rays it halts to the other pool.
#include "moray_internal.h"

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <vector>

using namespace moray;

struct moray_td {
  std::vector<int> shape;               // per grid: nx, ny, nz, offset (children)
  int n_src = 0, n_grp = 0, level_init = 0;
  long long n_cells = 0;
  double c_dt = 0.0;
  int slots = 0;
  long long step = 0;
  std::vector<long long> emit_step;     // per slot: the step its batch was emitted, -1 if none
  std::vector<double> P0;               // per slot, source and group: seed photon rate
  size_t cap = 0;                       // pool records; also slots of each level queue
  int nseg = 1;
  unsigned long long seg_cap = 0;
  int cur = 0;                          // pool holding the rays in flight
  unsigned long long n_in = 0;
  unsigned long long lev_in[kLevels] = {};
  bool broken = false;                  // a failed step leaves the pool undefined
  DevBuf pix[2], sg[2], r[2], P[2], lev[2];
  DevBuf qpix[2], qsg[2], qr[2], qP[2];
  DevBuf grids, probs, sgs, stats, ctr, kappa, acc, eexc, fblocks, partial;
  DevBuf keys[2], order[2], sort_temp;  // the halt list sorted by (level, tree, pixel)
  size_t sort_bytes = 0;
  std::vector<FinalBlock> fb;
  void* h_stage = nullptr;
};

static std::vector<int> grid_shape(const moray_problem& P) {
  std::vector<int> v;
  for (int q = 0; q < P.n_grids; ++q) {
    const moray_grid& G = P.grids[q];
    v.insert(v.end(), {G.nx, G.ny, G.nz, q > 0 ? G.offset[0] : 0, q > 0 ? G.offset[1] : 0, q > 0 ? G.offset[2] : 0});
  }
  return v;
}

static bool same_shape(const moray_td* t, const moray_problem& P) {
  return grid_shape(P) == t->shape && P.n_sources == t->n_src && P.spectrum->n_groups == t->n_grp &&
         P.params.level_init == t->level_init;
}

static void td_release(moray_ctx* c, moray_td* t) {
  DevBuf* all[] = {&t->grids, &t->probs, &t->sgs, &t->stats, &t->ctr, &t->kappa, &t->acc, &t->eexc, &t->fblocks,
                   &t->partial};
  for (DevBuf* b : all) release(c, *b);
  release(c, t->sort_temp);
  for (int i = 0; i < 2; ++i) {
    release(c, t->keys[i]);
    release(c, t->order[i]);
    release(c, t->pix[i]); release(c, t->sg[i]); release(c, t->r[i]); release(c, t->P[i]); release(c, t->lev[i]);
    release(c, t->qpix[i]); release(c, t->qsg[i]); release(c, t->qr[i]); release(c, t->qP[i]);
  }
  if (t->h_stage) (void)hipHostFree(t->h_stage);
  t->h_stage = nullptr;
}

moray_status moray_td_create(moray_ctx* c, const moray_problem* prob, double c_dt, size_t pool_rays,
                             moray_td** out) {
  if (!c) return MORAY_EINVAL;
  if (!prob || !out) return fail(c, MORAY_EINVAL, "NULL problem or handle");
  *out = nullptr;
  if (!(c_dt > 0.0) || !std::isfinite(c_dt)) return fail(c, MORAY_EINVAL, "c_dt must be positive and finite");
  if (pool_rays < 1024 || pool_rays > ((size_t)1 << 34)) return fail(c, MORAY_EINVAL, "pool_rays out of range");
  moray_status st = validate(c, *prob, 0);
  if (st != MORAY_OK) return st;
  if (prob->params.covering) return fail(c, MORAY_EINVAL, "time-dependent rays do not take the covering factor");
  if (prob->params.tau_thin > 0.0)
    return fail(c, MORAY_EINVAL, "time-dependent rays do not take the optically-thin approximation");
  if (engine_busy(c)) return fail(c, MORAY_EBUSY, "the context is serving asynchronous solves");
  const moray_grid& G = prob->grids[0];
  const double diag = std::sqrt((double)G.nx * G.nx + (double)G.ny * G.ny + (double)G.nz * G.nz);
  const double need_slots = std::ceil(diag / c_dt) + 2.0;
  const long long per = (long long)prob->n_sources * prob->spectrum->n_groups;
  if (need_slots * (double)per >= 2.0e9) return fail(c, MORAY_EINVAL, "c_dt too small for this many trees");
  long long n_cells = 0;
  for (int q = 0; q < prob->n_grids; ++q)
    n_cells += (long long)prob->grids[q].nx * prob->grids[q].ny * prob->grids[q].nz;
  if ((double)n_cells * prob->spectrum->n_groups >= (double)kNoSlot)
    return fail(c, MORAY_EINVAL, "the grids need fewer than 2^32 - 1 accumulators (cells x groups)");
  if (!hip_ok(c, hipSetDevice(c->device), "hipSetDevice")) return MORAY_EDEVICE;

  moray_td* t = new moray_td();
  t->shape = grid_shape(*prob);
  t->n_cells = n_cells;
  t->n_src = prob->n_sources;
  t->n_grp = prob->spectrum->n_groups;
  t->level_init = prob->params.level_init;
  t->c_dt = c_dt;
  t->slots = (int)need_slots;
  t->emit_step.assign(t->slots, -1);
  t->P0.assign((size_t)t->slots * per, 0.0);
  t->cap = pool_rays;
  t->nseg = queue_segments(pool_rays);
  t->seg_cap = pool_rays / (size_t)t->nseg;
  const int n_sg = (int)(t->slots * per);
  const size_t rsz = c->precision == MORAY_FP32_ACC64 ? sizeof(float) : sizeof(double);
  {
    const long long per_fb = (long long)kFinalBlock * kFinalCellsPerThread;
    for (int q = 0; q < prob->n_grids; ++q) {
      const long long nc = (long long)prob->grids[q].nx * prob->grids[q].ny * prob->grids[q].nz;
      for (long long f = 0; f < nc; f += per_fb) t->fb.push_back({q, (int)std::min(per_fb, nc - f), f});
    }
  }
  const size_t stage = sizeof(Counters) + (size_t)n_sg * sizeof(SgStats) + t->fb.size() * 8;
  for (int i = 0; i < 2 && st == MORAY_OK; ++i) {
    if ((st = ensure(c, t->pix[i], pool_rays * 8, "ray pool")) || (st = ensure(c, t->sg[i], pool_rays * 4, "ray pool")) ||
        (st = ensure(c, t->r[i], pool_rays * 8, "ray pool")) || (st = ensure(c, t->P[i], pool_rays * 8, "ray pool")) ||
        (st = ensure(c, t->lev[i], pool_rays * 4, "ray pool")) ||
        (st = ensure(c, t->qpix[i], pool_rays * 8, "ray queue")) ||
        (st = ensure(c, t->qsg[i], pool_rays * 4, "ray queue")) || (st = ensure(c, t->qr[i], pool_rays * 8, "ray queue")) ||
        (st = ensure(c, t->qP[i], pool_rays * 8, "ray queue")))
      break;
  }
  if (st == MORAY_OK) {
    (void)((st = ensure(c, t->grids, (size_t)prob->n_grids * sizeof(GridDev), "grid table")) ||
           (st = ensure(c, t->probs, sizeof(ProblemDev), "problem table")) ||
           (st = ensure(c, t->sgs, (size_t)n_sg * sizeof(SgDev), "source table")) ||
           (st = ensure(c, t->stats, (size_t)n_sg * sizeof(SgStats), "statistics")) ||
           (st = ensure(c, t->ctr, sizeof(Counters), "counters")) ||
           (st = ensure(c, t->kappa, (size_t)n_cells * rsz, "absorber columns")) ||
           (st = ensure(c, t->acc, (size_t)n_cells * t->n_grp * 8, "accumulators")) ||
           (st = ensure(c, t->eexc, (size_t)t->n_grp * 8, "group energies")) ||
           (st = ensure(c, t->fblocks, t->fb.size() * sizeof(FinalBlock), "finalize blocks")) ||
           (st = ensure(c, t->partial, t->fb.size() * 8, "partial sums")));
  }
  if (st == MORAY_OK && pool_rays < ((size_t)1 << 32)) {
    // sorting needs 32-bit record indices; larger pools are resumed unsorted
    if (!hip_ok(c, td_sort_temp_bytes(pool_rays, &t->sort_bytes), "sort")) st = MORAY_EDEVICE;
    for (int i = 0; i < 2 && st == MORAY_OK; ++i)
      if ((st = ensure(c, t->keys[i], pool_rays * 8, "sort keys")) ||
          (st = ensure(c, t->order[i], pool_rays * 4, "sort order")))
        break;
    if (st == MORAY_OK) st = ensure(c, t->sort_temp, std::max<size_t>(t->sort_bytes, 256), "sort scratch");
  }
  if (st == MORAY_OK && hipHostMalloc(&t->h_stage, stage, hipHostMallocDefault) != hipSuccess) {
    t->h_stage = nullptr;
    st = fail(c, MORAY_ENOMEM, "pinned staging allocation failed");
  }
  if (st == MORAY_OK &&
      !hip_ok(c, hipMemcpyAsync(t->fblocks.p, t->fb.data(), t->fb.size() * sizeof(FinalBlock), hipMemcpyHostToDevice,
                                c->stream), "upload"))
    st = MORAY_EDEVICE;
  if (st == MORAY_OK && !hip_ok(c, hipStreamSynchronize(c->stream), "synchronize")) st = MORAY_EDEVICE;
  if (st != MORAY_OK) {
    td_release(c, t);
    delete t;
    return st;
  }
  *out = t;
  c->err = "no error";
  return MORAY_OK;
}

void moray_td_free(moray_ctx* c, moray_td* t) {
  if (!c || !t) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  td_release(c, t);
  delete t;
}

template <typename R>
static hipError_t launch_level(moray_ctx* c, moray_td* t, int l, int seed_lo, int seed_hi, unsigned max_steps,
                               unsigned long long reserve) {
  const int b = 1 - t->cur;       // the pool the halted rays go to
  TraceArgs<R> A{};
  A.grids = (GridDev*)t->grids.p;
  A.probs = (ProblemDev*)t->probs.p;
  A.sgs = (SgDev*)t->sgs.p;
  A.kappa = (R*)t->kappa.p;
  A.acc = (double*)t->acc.p;
  A.in = RayQueue{(uint64_t*)t->qpix[l & 1].p, (uint32_t*)t->qsg[l & 1].p, (double*)t->qr[l & 1].p,
                  (double*)t->qP[l & 1].p};
  A.out = RayQueue{(uint64_t*)t->qpix[(l + 1) & 1].p, (uint32_t*)t->qsg[(l + 1) & 1].p,
                   (double*)t->qr[(l + 1) & 1].p, (double*)t->qP[(l + 1) & 1].p};
  A.seg_cap = t->seg_cap;
  A.nseg = t->nseg;
  A.ctr = (Counters*)t->ctr.p;
  A.stats = (SgStats*)t->stats.p;
  A.gen = l;
  A.cin = l;
  A.cout = l + 1;
  A.seed_level = l;
  A.seed_sg_begin = seed_lo;
  A.seed_sg_end = seed_hi;
  A.chunk = c->chunk;
  A.refill = c->refill;
  A.max_steps = max_steps;
  A.reserve = reserve;
  A.halt = RayQueue{(uint64_t*)t->pix[b].p, (uint32_t*)t->sg[b].p, (double*)t->r[b].p, (double*)t->P[b].p};
  A.halt_lev = (int*)t->lev[b].p;
  A.halt_cap = t->cap;
  A.tree_fold = (uint32_t)(t->n_src * t->n_grp);
  return launch_trace_level_halt<R>(c->stream, std::max(1, c->num_cu * c->blocks_per_cu), A, c->cache);
}

// Doubles the pools, the level queues and the sort buffers of a state whose
// step overflowed, keeping the rays in flight before the step (pool t->cur,
// which a step only reads). Fails with MORAY_EQUEUE, the state unchanged,
// when the doubled buffers do not fit the context's HBM budget.
static moray_status td_grow(moray_ctx* c, moray_td* t, unsigned long long demand) {
  // at least double; enough for what the failed step asked for, with room for segment imbalance
  size_t ncap = t->cap * 2;
  while ((double)ncap < 1.5 * (double)demand && ncap <= ((size_t)1 << 34)) ncap *= 2;
  if (ncap > ((size_t)1 << 34)) return fail(c, MORAY_EQUEUE, "the ray pool cannot grow beyond 2^34 rays");
  const size_t pool_b = 8 + 4 + 8 + 8 + 4, queue_b = 8 + 4 + 8 + 8, sort_b = 8 + 4;
  size_t sort_tmp = 0;
  if (ncap < ((size_t)1 << 32) && !hip_ok(c, td_sort_temp_bytes(ncap, &sort_tmp), "sort")) return MORAY_EDEVICE;
  const size_t nbytes = ncap * (2 * pool_b + 2 * queue_b + (ncap < ((size_t)1 << 32) ? 2 * sort_b : 0)) +
                        (ncap < ((size_t)1 << 32) ? std::max<size_t>(sort_tmp, 256) : 0);
  const int a = t->cur;
  size_t old = t->sort_temp.bytes + t->pix[1 - a].bytes + t->sg[1 - a].bytes + t->r[1 - a].bytes +
               t->P[1 - a].bytes + t->lev[1 - a].bytes;
  for (int i = 0; i < 2; ++i)
    old += t->qpix[i].bytes + t->qsg[i].bytes + t->qr[i].bytes + t->qP[i].bytes + t->keys[i].bytes + t->order[i].bytes;
  if (c->allocated - old + nbytes + 4096 > c->budget)
    return fail(c, MORAY_EQUEUE, "the ray pool or a level queue overflowed and cannot double within the HBM budget");
  // everything but the rays in flight can go first
  release(c, t->sort_temp);
  for (int i = 0; i < 2; ++i) {
    release(c, t->keys[i]);
    release(c, t->order[i]);
    release(c, t->qpix[i]); release(c, t->qsg[i]); release(c, t->qr[i]); release(c, t->qP[i]);
  }
  release(c, t->pix[1 - a]); release(c, t->sg[1 - a]); release(c, t->r[1 - a]); release(c, t->P[1 - a]);
  release(c, t->lev[1 - a]);
  DevBuf np[5];
  moray_status st;
  if ((st = ensure(c, np[0], ncap * 8, "ray pool")) || (st = ensure(c, np[1], ncap * 4, "ray pool")) ||
      (st = ensure(c, np[2], ncap * 8, "ray pool")) || (st = ensure(c, np[3], ncap * 8, "ray pool")) ||
      (st = ensure(c, np[4], ncap * 4, "ray pool"))) {
    for (DevBuf& b : np) release(c, b);
    t->broken = true;
    return fail(c, MORAY_EQUEUE, "the ray pool overflowed and its doubled buffers could not be allocated");
  }
  hipStream_t s = c->stream;
  const unsigned long long n = t->n_in;
  if (n && (!hip_ok(c, hipMemcpyAsync(np[0].p, t->pix[a].p, n * 8, hipMemcpyDeviceToDevice, s), "copy") ||
            !hip_ok(c, hipMemcpyAsync(np[1].p, t->sg[a].p, n * 4, hipMemcpyDeviceToDevice, s), "copy") ||
            !hip_ok(c, hipMemcpyAsync(np[2].p, t->r[a].p, n * 8, hipMemcpyDeviceToDevice, s), "copy") ||
            !hip_ok(c, hipMemcpyAsync(np[3].p, t->P[a].p, n * 8, hipMemcpyDeviceToDevice, s), "copy") ||
            !hip_ok(c, hipMemcpyAsync(np[4].p, t->lev[a].p, n * 4, hipMemcpyDeviceToDevice, s), "copy"))) {
    t->broken = true;
    return MORAY_EDEVICE;
  }
  if (!hip_ok(c, hipStreamSynchronize(s), "synchronize")) {
    t->broken = true;
    return MORAY_EDEVICE;
  }
  release(c, t->pix[a]); release(c, t->sg[a]); release(c, t->r[a]); release(c, t->P[a]); release(c, t->lev[a]);
  t->pix[a] = np[0]; t->sg[a] = np[1]; t->r[a] = np[2]; t->P[a] = np[3]; t->lev[a] = np[4];
  const int b = 1 - a;
  for (int i = 0; i < 2; ++i) {
    if ((i == b && ((st = ensure(c, t->pix[b], ncap * 8, "ray pool")) || (st = ensure(c, t->sg[b], ncap * 4, "ray pool")) ||
                    (st = ensure(c, t->r[b], ncap * 8, "ray pool")) || (st = ensure(c, t->P[b], ncap * 8, "ray pool")) ||
                    (st = ensure(c, t->lev[b], ncap * 4, "ray pool")))) ||
        (st = ensure(c, t->qpix[i], ncap * 8, "ray queue")) || (st = ensure(c, t->qsg[i], ncap * 4, "ray queue")) ||
        (st = ensure(c, t->qr[i], ncap * 8, "ray queue")) || (st = ensure(c, t->qP[i], ncap * 8, "ray queue"))) {
      t->broken = true;
      return fail(c, MORAY_EQUEUE, "the ray pool overflowed and its doubled buffers could not be allocated");
    }
  }
  t->sort_bytes = 0;
  if (ncap < ((size_t)1 << 32)) {
    t->sort_bytes = sort_tmp;
    for (int i = 0; i < 2; ++i)
      if ((st = ensure(c, t->keys[i], ncap * 8, "sort keys")) || (st = ensure(c, t->order[i], ncap * 4, "sort order"))) {
        t->broken = true;
        return st;
      }
    if ((st = ensure(c, t->sort_temp, std::max<size_t>(sort_tmp, 256), "sort scratch"))) {
      t->broken = true;
      return st;
    }
  }
  t->cap = ncap;
  t->nseg = queue_segments(ncap);
  t->seg_cap = ncap / (size_t)t->nseg;
  return MORAY_OK;
}

moray_status moray_td_step(moray_ctx* c, moray_td* t, const moray_problem* prob, unsigned flags, int emit,
                           moray_result* out, double* held) {
  if (!c) return MORAY_EINVAL;
  if (!t || !prob || !out) return fail(c, MORAY_EINVAL, "NULL state, problem or result");
  if (t->broken) return fail(c, MORAY_EINVAL, "an earlier step of this state failed");
  if (flags != (MORAY_FIELDS_ON_DEVICE | MORAY_OUT_ON_DEVICE))
    return fail(c, MORAY_EINVAL, "time-dependent steps take device fields and device results");
  if (!out->k_ph || !out->heating) return fail(c, MORAY_EINVAL, "result buffers are NULL");
  if (out->accel) return fail(c, MORAY_EINVAL, "time-dependent steps do not compute radiation pressure");
  moray_status st = validate(c, *prob, 0);
  if (st != MORAY_OK) return st;
  if (!same_shape(t, *prob)) return fail(c, MORAY_EINVAL, "the problem's shape differs from the state's");
  if (prob->params.covering) return fail(c, MORAY_EINVAL, "time-dependent rays do not take the covering factor");
  if (prob->params.tau_thin > 0.0)
    return fail(c, MORAY_EINVAL, "time-dependent rays do not take the optically-thin approximation");
  if (engine_busy(c)) return fail(c, MORAY_EBUSY, "the context is serving asynchronous solves");
  if (!hip_ok(c, hipSetDevice(c->device), "hipSetDevice")) return MORAY_EDEVICE;
  const moray_problem& P = *prob;
  const moray_grid& G = P.grids[0];
  const moray_spectrum& Sp = *P.spectrum;
  const long long n_cells = t->n_cells;
  const int per = t->n_src * t->n_grp;
  const int n_sg = t->slots * per;
  const int cur_slot = (int)(t->step % t->slots);
  const double npix0 = std::ldexp(12.0, 2 * P.params.level_init);
  // what this step changes in the state before it has run (restored when it fails)
  const long long saved_emit = t->emit_step[cur_slot];
  const std::vector<double> saved_P0(t->P0.begin() + (size_t)cur_slot * per, t->P0.begin() + (size_t)(cur_slot + 1) * per);
  auto restore = [&]() {
    t->emit_step[cur_slot] = saved_emit;
    std::copy(saved_P0.begin(), saved_P0.end(), t->P0.begin() + (size_t)cur_slot * per);
  };
  if (emit) {
    t->emit_step[cur_slot] = t->step;
    for (int s = 0; s < t->n_src; ++s)
      for (int g = 0; g < t->n_grp; ++g)
        t->P0[(size_t)cur_slot * per + s * t->n_grp + g] = Sp.photon_frac[g] * P.sources[s].ndot / npix0;
  } else {
    t->emit_step[cur_slot] = -1;          // an older batch here has left the box
  }

  // An overflow leaves the rays in flight before the step untouched: the
  // buffers double and the step runs again.
  for (int attempt = 0;; ++attempt) {
  // tables: the root grid, then its children (cells numbered in grid order)
  std::vector<GridDev> gds(P.n_grids);
  long long steps_bound = 16;
  {
    long long off = 0;
    for (int q = 0; q < P.n_grids; ++q) {
      const moray_grid& Gq = P.grids[q];
      GridDev& gd = gds[q];
      gd.nx = Gq.nx; gd.ny = Gq.ny; gd.nz = Gq.nz;
      gd.is_child = q > 0;
      gd.ox = q > 0 ? Gq.offset[0] : 0;
      gd.oy = q > 0 ? Gq.offset[1] : 0;
      gd.oz = q > 0 ? Gq.offset[2] : 0;
      gd.problem = 0;
      gd.cell_off = off;
      gd.dx_cm = Gq.dx_cm;
      gd.n_h = Gq.n_h;
      gd.x_hi = Gq.x_hi;
      gd.out_kph = out->k_ph + off;
      gd.out_heat = out->heating + off;
      off += (long long)Gq.nx * Gq.ny * Gq.nz;
      steps_bound += 2LL * (Gq.nx + Gq.ny + Gq.nz);
    }
  }
  ProblemDev pd{};
  pd.root_grid = 0;
  pd.n_groups = t->n_grp;
  pd.cell_off = 0;
  pd.n_cells = n_cells;
  pd.acc_off = 0;
  pd.eexc_off = 0;
  std::vector<double> eexc(t->n_grp);
  for (int g = 0; g < t->n_grp; ++g) eexc[g] = (Sp.energy_ev[g] - Sp.e_ion_ev) * kEvErgConst;
  std::vector<SgDev> sgs(n_sg);
  for (int b = 0; b < t->slots; ++b)
    for (int s = 0; s < t->n_src; ++s)
      for (int g = 0; g < t->n_grp; ++g) {
        SgDev& d = sgs[(size_t)b * per + s * t->n_grp + g];
        const moray_source& S = P.sources[s];
        d.sx = S.x; d.sy = S.y; d.sz = S.z;
        d.P0 = t->P0[(size_t)b * per + s * t->n_grp + g];
        d.pmin0 = P.params.p_min_frac * d.P0;
        d.sigma64 = Sp.sigma_cm2[g];
        d.sigma32 = (float)Sp.sigma_cm2[g];
        d.four_pi_phi_c = 4.0 * kPiConst * P.params.phi_c;
        d.split_t2_base = P.params.phi_c > 0.0 ? (float)(12.0 / (4.0 * kPiConst * P.params.phi_c)) : FLT_MAX;
        d.acc_slot = (long long)g * n_cells;
        d.problem = 0;
        d.root_grid = 0;
        d.rnx = G.nx; d.rny = G.ny; d.rnz = G.nz;
        d.rcell_off = 0;
        d.level_init = P.params.level_init;
        d.gen0 = P.params.level_init;
        d.level_max = P.params.phi_c > 0.0 ? P.params.level_max : P.params.level_init;
        const long long age = t->emit_step[b] >= 0 ? t->step - t->emit_step[b] : -1;
        d.r_halt = age >= 0 ? (double)(age + 1) * t->c_dt : 0.0;
      }
  hipStream_t s = c->stream;
  auto up = [&](DevBuf& b, const void* src, size_t bytes) {
    return hip_ok(c, hipMemcpyAsync(b.p, src, bytes, hipMemcpyHostToDevice, s), "upload");
  };
  if (!up(t->grids, gds.data(), gds.size() * sizeof(GridDev)) || !up(t->probs, &pd, sizeof pd) || !up(t->sgs, sgs.data(), sgs.size() * sizeof(SgDev)) ||
      !up(t->eexc, eexc.data(), eexc.size() * 8))
    return MORAY_EDEVICE;

  // levels: the seeds' and those of the rays in flight, up to the deepest a ray can reach
  const int l_hi = reach_level(P);
  int l_lo = emit ? P.params.level_init : kLevels;
  for (int l = 0; l < kLevels; ++l)
    if (t->lev_in[l]) { l_lo = std::min(l_lo, l); break; }
  unsigned max_steps = (unsigned)std::min<long long>(2 * steps_bound, 1LL << 30);
  const double waves = (double)std::max(1, c->num_cu * c->blocks_per_cu) * (kTraceBlock / kWave);
  unsigned long long reserve =
      (unsigned long long)std::min<double>((double)kReserveMax, (double)t->cap / (8.0 * waves));
  reserve = std::max<unsigned long long>(4, reserve & ~3ull);
  Counters* ctr = (Counters*)t->ctr.p;
  const bool fp32 = c->precision == MORAY_FP32_ACC64;
  const int a = t->cur;
  const RayQueue pool_in{(uint64_t*)t->pix[a].p, (uint32_t*)t->sg[a].p, (double*)t->r[a].p, (double*)t->P[a].p};
  auto queue = [&](int l) {
    return RayQueue{(uint64_t*)t->qpix[l & 1].p, (uint32_t*)t->qsg[l & 1].p, (double*)t->qr[l & 1].p,
                    (double*)t->qP[l & 1].p};
  };
  hipError_t e = launch_reset(s, ctr, (SgStats*)t->stats.p, n_sg);
  if (e == hipSuccess)
    e = fp32 ? launch_prep<float>(s, c->num_cu, (GridDev*)t->grids.p, P.n_grids, 0, (ProblemDev*)t->probs.p, 0, n_cells,
                                  (float*)t->kappa.p, (double*)t->acc.p, ctr)
             : launch_prep<double>(s, c->num_cu, (GridDev*)t->grids.p, P.n_grids, 0, (ProblemDev*)t->probs.p, 0, n_cells,
                                   (double*)t->kappa.p, (double*)t->acc.p, ctr);
  if (!hip_ok(c, e, "prep")) return MORAY_EDEVICE;
  int launches = 0;
  // the rays in flight sorted by (level, tree, pixel) when the key fits 64 bits
  int tree_bits = 1;
  while (tree_bits < 31 && ((long long)1 << tree_bits) < n_sg) ++tree_bits;
  const int pix_bits = 2 * l_hi + 4;
  const bool sorted = t->n_in > 0 && t->keys[0].p && 5 + tree_bits + pix_bits <= 64;
  unsigned long long first[kLevels] = {};
  if (sorted) {
    unsigned long long o = 0;
    for (int l = 0; l < kLevels; ++l) { first[l] = o; o += t->lev_in[l]; }
    if (!hip_ok(c, launch_td_sort(s, c->num_cu, pool_in, (const int*)t->lev[a].p, t->n_in, tree_bits, pix_bits,
                                  (unsigned long long*)t->keys[0].p, (unsigned long long*)t->keys[1].p,
                                  (uint32_t*)t->order[0].p, (uint32_t*)t->order[1].p, t->sort_temp.p, t->sort_bytes),
                "sort"))
      return MORAY_EDEVICE;
  }
  auto prefill = [&](int l) {
    if (sorted)
      return launch_prefill_sorted(s, c->num_cu, pool_in, (const uint32_t*)t->order[1].p, first[l], t->lev_in[l],
                                   queue(l), t->seg_cap, t->nseg, ctr, l);
    return launch_prefill_level(s, c->num_cu, pool_in, (const int*)t->lev[a].p, t->n_in, l, queue(l), t->seg_cap,
                                t->nseg, ctr, l);
  };
  if (l_lo <= l_hi) {
    if (t->lev_in[l_lo] && !hip_ok(c, prefill(l_lo), "prefill")) return MORAY_EDEVICE;
    for (int l = l_lo; l <= l_hi; ++l) {
      if (l + 1 <= l_hi && l + 1 < kLevels && t->lev_in[l + 1] && !hip_ok(c, prefill(l + 1), "prefill"))
        return MORAY_EDEVICE;
      const bool seeds = emit && l == P.params.level_init;
      const int lo = seeds ? cur_slot * per : 0, hi = seeds ? (cur_slot + 1) * per : 0;
      e = fp32 ? launch_level<float>(c, t, l, lo, hi, max_steps, reserve)
               : launch_level<double>(c, t, l, lo, hi, max_steps, reserve);
      if (!hip_ok(c, e, "trace")) return MORAY_EDEVICE;
      ++launches;
    }
  }
  if (!hip_ok(c, launch_finalize(s, (int)t->fb.size(), (GridDev*)t->grids.p, (ProblemDev*)t->probs.p,
                                 (FinalBlock*)t->fblocks.p, (double*)t->acc.p, (double*)t->eexc.p,
                                 (double*)t->partial.p, ctr), "finalize"))
    return MORAY_EDEVICE;
  char* hs = (char*)t->h_stage;
  Counters* hctr = (Counters*)hs;
  SgStats* hst = (SgStats*)(hs + sizeof(Counters));
  double* hpart = (double*)(hs + sizeof(Counters) + (size_t)n_sg * sizeof(SgStats));
  if (!hip_ok(c, hipMemcpyAsync(hctr, ctr, sizeof(Counters), hipMemcpyDeviceToHost, s), "copy") ||
      !hip_ok(c, hipMemcpyAsync(hst, t->stats.p, (size_t)n_sg * sizeof(SgStats), hipMemcpyDeviceToHost, s), "copy") ||
      !hip_ok(c, hipMemcpyAsync(hpart, t->partial.p, t->fb.size() * 8, hipMemcpyDeviceToHost, s), "copy") ||
      !hip_ok(c, hipStreamSynchronize(s), "synchronize"))
    return MORAY_EDEVICE;
  if (hctr->err & kErrBadInput) {
    restore();
    return fail(c, MORAY_EINVAL, "a density or neutral fraction is negative, non-finite or x_HI > 1");
  }
  if (hctr->err & kErrInternal) {
    t->broken = true;
    return fail(c, MORAY_EINTERNAL, "a ray exceeded its step bound");
  }
  if (hctr->err & kErrOverflow) {
    // what the step asked for: the halt list's records and the largest level queue's slots
    unsigned long long demand = hctr->halt_count;
    for (int l = 0; l < kLevels; ++l) {
      unsigned long long n = 0;
      for (int sgi = 0; sgi < t->nseg; ++sgi) n += hctr->count[l][sgi];
      demand = std::max(demand, n);
    }
    const moray_status gs = attempt < 8 ? td_grow(c, t, demand)
                                        : fail(c, MORAY_EQUEUE, "the ray pool or a level queue overflowed eight times");
    if (gs == MORAY_OK) continue;
    if (!t->broken) restore();
    return gs;
  }
  // results of the step
  moray_result& Rr = *out;
  Rr.emitted = Rr.absorbed = Rr.escaped = Rr.truncated = 0.0;
  Rr.segments = Rr.rays_seeded = Rr.splits = Rr.rays_escaped = Rr.rays_truncated = 0;
  Rr.thin_segments = 0;
  if (emit)
    for (int si = 0; si < t->n_src; ++si)
      for (int g = 0; g < t->n_grp; ++g) Rr.emitted += Sp.photon_frac[g] * P.sources[si].ndot;
  for (size_t b = 0; b < t->fb.size(); ++b) Rr.absorbed += hpart[b];
  // the photons the halted rays hold, summed over the halt list
  double h = 0.0;
  // the halt list's records (empty ones, which waves reserved and did not
  // fill, hold no photons); records beyond the pool were never written
  const unsigned long long n_held = std::min<unsigned long long>(hctr->halt_count, t->cap);
  if (n_held) {
    const int nb = (int)std::min<size_t>(t->fb.size(), 1024);
    if (!hip_ok(c, launch_sum_blocks(s, nb, (const double*)t->P[1 - t->cur].p, n_held, (double*)t->partial.p),
                "sum") ||
        !hip_ok(c, hipMemcpyAsync(hpart, t->partial.p, (size_t)nb * 8, hipMemcpyDeviceToHost, s), "copy") ||
        !hip_ok(c, hipStreamSynchronize(s), "synchronize"))
      return MORAY_EDEVICE;
    for (int b = 0; b < nb; ++b) h += hpart[b];
  }
  if (Rr.escaped_sg)
    for (int k = 0; k < per; ++k) Rr.escaped_sg[k] = 0.0;
  for (int k = 0; k < n_sg; ++k) {
    const SgStats& S = hst[k];
    if (Rr.escaped_sg) Rr.escaped_sg[k % per] += S.esc_P;
    Rr.escaped += S.esc_P;
    Rr.truncated += S.trunc_P;
    Rr.segments += S.segs;
    Rr.splits += S.splits;
    Rr.rays_escaped += S.n_esc;
    Rr.rays_truncated += S.n_trunc;
  }
  Rr.rays_seeded = emit ? (unsigned long long)per * (unsigned long long)npix0 : 0ull;
  unsigned long long peak = 0;
  for (int l = 0; l < kLevels; ++l) {
    unsigned long long n = 0;
    for (int sgi = 0; sgi < t->nseg; ++sgi) n += std::min<unsigned long long>(hctr->count[l][sgi], t->seg_cap);
    peak = std::max(peak, n);
  }
  Rr.peak_level_rays = peak;
  Rr.trace_ms = 0.0;
  Rr.trace_launches = launches;
  Rr.t_admit = Rr.t_done = 0.0;
  Rr.from_graph = 0;
  // the halted rays are the next step's rays in flight
  t->n_in = n_held;
  std::memcpy(t->lev_in, hctr->halt_levels, sizeof t->lev_in);
  t->cur = 1 - t->cur;
  t->step++;
  if (held) *held = h;
  c->err = "no error";
  return MORAY_OK;
  }  // attempts
}
