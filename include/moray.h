/*
 * moray.h -- C ABI of the MI355X adaptive ray tracer.
 *
 * The library computes one radiative-transfer pass of photon-conserving
 * adaptive ray tracing from point sources (Wise & Abel, Enzo+Moray):
 *   - rays start on the centres of the HEALPix nested pixels of level
 *     `level_init` around every source, one ray set per energy group, the
 *     group's photon rate shared equally (section 2.1);
 *   - each ray marches cell by cell (Eq. trace) and deposits
 *     dP = P (1 - exp(-tau)), tau = sigma n_H x_HI dr (Eqs. dtau, flux), into
 *     the cell's photo-ionisation rate k_ph and photo-heating rate
 *     (Eqs. kph, gamma: k_ph = sum dP / (n_H x_HI V_cell),
 *     heating = sum dP (E - E_ion) / (n_H x_HI V_cell));
 *   - a ray whose solid angle at its cell exit exceeds 1/phi_c of a cell face
 *     (12 * 4^l < 4 pi phi_c t_exit^2 in local cell units, Eq. split and
 *     step 3e of section 3.1) is replaced by its four nested children
 *     4p..4p+3, which keep its radius and take a quarter of its photons each;
 *   - a ray ends when P < p_min_frac * P0 (P0: its unattenuated share) or when
 *     it leaves the root grid (isolated boundaries, section 2.1);
 *   - a ray entering a root cell covered by a 2x-refined child grid continues
 *     in the child (section 3.1 step 3c) and returns to the root on leaving it.
 * The pass is single-shot (infinite speed of light), so P is a photon rate
 * and the timestep of Eq. kph cancels: k_ph is in 1/s, heating in erg/s, per
 * absorber.
 *
 * Conventions: fields are float32, x fastest (cell i + nx*(j + ny*k)).
 * Source positions are in cells of the root grid, measured from its lower
 * corner. Outputs are float64, concatenated over a problem's grids in grid
 * order; root cells covered by a child grid report 0.
 *
 * Every function returns a moray_status (0 = MORAY_OK); no exception crosses
 * the ABI. On any error moray_last_error() describes it. A context is used by
 * one host thread at a time.
 */
#ifndef MORAY_H
#define MORAY_H
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MORAY_OK = 0,
  MORAY_EINVAL = -1,     /* invalid argument or input value; outputs untouched */
  MORAY_ENOMEM = -2,     /* device memory or the context's HBM budget exhausted */
  MORAY_EDEVICE = -3,    /* no usable GPU, or a HIP runtime call failed */
  MORAY_EQUEUE = -4,     /* ray queue overflowed even after automatic retries */
  MORAY_EBUSY = -5,      /* an asynchronous solve has not finished yet */
  MORAY_ETIMEOUT = -6,   /* an asynchronous solve passed its deadline (moray_set_deadline) */
  MORAY_EINTERNAL = -7,  /* a device-side consistency check failed */
  MORAY_ECANCELED = -8   /* an asynchronous solve was cancelled (moray_cancel) */
} moray_status;

typedef enum {
  MORAY_FP64 = 0,        /* geometry, optical depth and accumulation in float64 */
  MORAY_FP32_ACC64 = 1   /* geometry and optical depth in float32; photon counts,
                            accumulators and split decisions near their threshold
                            in float64 */
} moray_precision;

/* flags of moray_trace */
#define MORAY_FIELDS_ON_DEVICE 1u   /* n_h / x_hi pointers are device memory */
#define MORAY_OUT_ON_DEVICE 2u      /* k_ph / heating pointers are device memory */

typedef struct moray_ctx moray_ctx;

typedef struct {
  int device;                 /* HIP device ordinal */
  int precision;              /* moray_precision */
  size_t hbm_budget_bytes;    /* cap on the context's device memory; 0 = half of the free memory */
  size_t queue_capacity;      /* rays per level buffer; 0 = sized from each problem's worst case */
  int waves_per_cu;           /* persistent trace waves per compute unit; 0 = default */
  int refill_lanes;           /* a wave refetches rays once this many of its 64 lanes are idle; 0 = default (64:
                                 once the whole wave is idle, so new rays start together) */
  int chunk_rays;             /* rays a wave claims from the level queue per atomic; 0 = default (256);
                                 the largest claim: on a level with fewer rays than one claim for
                                 every wave of the launch, waves halve it, down to 64 */
  void* hip_stream;           /* hipStream_t for every launch; NULL = the null stream */
  int profile;                /* nonzero: time every trace-kernel launch with HIP events */
  int deposit_cache;          /* >= 0: combine deposits in a per-wave LDS table (default);
                                 < 0: one float64 atomic per segment */
  int reserve_rays;           /* next-level queue slots a wave reserves per atomic; 0 = from the queue size */
} moray_init_params;

typedef struct {
  double x, y, z;             /* position in root-grid cells, inside [0, n) per axis */
  double ndot;                /* ionising photon rate, photons/s, > 0 */
} moray_source;

typedef struct {
  int n_groups;               /* >= 1 monochromatic groups (section 3.2) */
  const double* energy_ev;    /* [n_groups] photon energy, >= e_ion_ev */
  const double* sigma_cm2;    /* [n_groups] absorption cross-section, >= 0 */
  const double* photon_frac;  /* [n_groups] share of each source's photons, >= 0, sum 1 +- 1e-12 */
  double e_ion_ev;            /* ionisation energy of the absorber (13.6 for HI) */
} moray_spectrum;             /* host memory */

typedef struct {
  int nx, ny, nz;             /* cells */
  double dx_cm;               /* cell width; a child's is exactly half the root's */
  int parent;                 /* -1 for the root (grid 0), 0 for a child of the root */
  int offset[3];              /* child: lower corner in root cells; its nx/2 x ny/2 x nz/2
                                 root cells must lie inside the root and not overlap another child */
  const float* n_h;           /* [nx*ny*nz] hydrogen density, cm^-3, finite, >= 0 */
  const float* x_hi;          /* [nx*ny*nz] neutral fraction, in [0, 1] */
} moray_grid;

typedef struct {
  double phi_c;               /* rays per cell face below which a ray splits; 0 = never split */
  int level_init;             /* HEALPix level of the seed rays, 0 <= level_init <= level_max */
  int level_max;              /* rays at this level never split, <= 29 */
  double p_min_frac;          /* a ray ends once P < p_min_frac * P0, in [0, 1) */
  int covering;               /* nonzero: scale each segment's contribution to k_ph and heating (not
                                 its attenuation) by the covering factor of section 2.3 (Eqs.
                                 midpoint, fc); the results are then not photon-conserving, and
                                 `absorbed` reports the scaled sum */
  double tau_thin;            /* > 0: the optically-thin approximation of section 2.4 (Eq. optthin,
                                 the per-source marker field); 0 (or a zero-initialised struct):
                                 off. Finite and >= 0. A ray whose optical depth from its source
                                 is still below tau_thin where it leaves a cell is thin there: it
                                 removes no photons, is split against min(1, phi_c) rays per cell
                                 face instead of phi_c, and gives the cell, once per (source,
                                 group), the rate sigma P / (Omega_ray r_cell^2) of its flux moved
                                 to the cell centre (Omega_ray = 4 pi / N_pix(l), r_cell in cm), and
                                 heating that rate times (E - E_ion); in a cell that holds the
                                 source (inside or on its boundary) it adds its general deposit
                                 P (1 - e^-tau) to the rate instead. A ray that is not thin in a
                                 cell deposits and attenuates as usual and stays thick. The thin
                                 rates are in k_ph and heating (also where n_H x_HI = 0) but not in
                                 `absorbed` or the other totals, which count removed photons only.
                                 Not with radiation pressure (`accel`) in the same batch, the
                                 serving engine or time-dependent rays (MORAY_EINVAL). */
} moray_trace_params;

typedef struct {
  const moray_grid* grids;    /* [n_grids], grid 0 is the root */
  int n_grids;
  const moray_source* sources;/* [n_sources], host memory */
  int n_sources;
  const moray_spectrum* spectrum;
  moray_trace_params params;
} moray_problem;

typedef struct {
  double* k_ph;               /* [total cells] caller-owned output, 1/s per absorber */
  double* heating;            /* [total cells] caller-owned output, erg/s per absorber */
  double* escaped_sg;         /* optional host [n_sources*n_groups] escaped photons/s, or NULL */
  double* accel;              /* optional [3 * total cells] caller-owned output (host or device like
                                 k_ph), or NULL: the radiation-pressure acceleration of the gas
                                 (section 2.5.4, Eq. radpres), cm/s^2, component-major over the
                                 problem's concatenated cells, accel[k * total_cells + cell] for
                                 k = x, y, z. Every absorbed photon rate dP hands the momentum rate
                                 dP E_ph / c along its ray to its cell (the covering factor does not
                                 scale it); a = that sum / (m_H n_H V) with m_H = 1.6735575e-24 g,
                                 0 where n_H = 0. Asking for it runs a variant of the trace kernel
                                 with three more sums per segment. moray_trace only: the serving
                                 engine rejects it. */
  /* filled by the library: */
  double emitted;             /* sum over sources and groups of the photon rate */
  double absorbed;            /* sum over cells of the absorbed photon rate */
  double escaped;             /* photon rate leaving the root grid */
  double truncated;           /* photon rate left in rays ended by p_min_frac */
  unsigned long long segments;        /* (ray, cell) crossings with dr > 0 that deposited */
  unsigned long long rays_seeded, splits, rays_escaped, rays_truncated;
  unsigned long long peak_level_rays; /* largest level population of this solve's ray queue */
  double trace_ms;            /* summed trace-kernel device time of the call (profile only) */
  int trace_launches;         /* trace-kernel launches the problem took part in */
  double t_admit, t_done;     /* asynchronous solves: CLOCK_MONOTONIC seconds when the problem
                                 was admitted to the device and when its results were complete */
  int from_graph;             /* 1 when the call replayed the launch sequence captured for the
                                 same descriptors (device fields and results, see moray_trace) */
  unsigned long long thin_segments;   /* of `segments`, those of rays that were optically thin in
                                         their cell (params.tau_thin > 0; else 0) */
} moray_result;

typedef unsigned long long moray_ticket;

/* Create a context on params->device. Returns MORAY_EDEVICE when no GPU is
 * visible or the device cannot be used, MORAY_EINVAL for bad parameters.
 * *ctx is NULL on failure. */
moray_status moray_init(moray_ctx** ctx, const moray_init_params* params);

/* Trace n_probs independent problems in one batched pass (n_probs >= 1), all
 * of them through the same launch sequence. Inputs are read-only and must stay
 * valid until the call returns; outputs are written only on success (on
 * MORAY_EINVAL they are untouched, on device-side errors their content is
 * undefined). Blocks until the results are complete. A batch holds fewer than
 * 2^31 - 1 cells and fewer than 2^32 - 1 accumulators (cells x groups summed
 * over its problems, plus 3 per cell of the problems that ask for the
 * radiation-pressure acceleration); larger batches return MORAY_EINVAL.
 * With both MORAY_FIELDS_ON_DEVICE and MORAY_OUT_ON_DEVICE (and profiling
 * off), a call whose descriptors, field and result pointers and settings
 * equal the previous call's captures its launch sequence in a HIP graph, and
 * later such calls replay it; field values may change in place between
 * calls. Any other call drops the captured sequence. */
moray_status moray_trace(moray_ctx* ctx, const moray_problem* probs, int n_probs, unsigned flags,
                         moray_result* outs);

/* moray_trace for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same solve, with every scratch buffer (absorber columns, accumulators,
 * ray queues, tables, counters, host-field upload and host-result staging)
 * carved from one fixed array of 256 MiB that the library holds in device
 * memory on each GPU it runs on, for the life of the process. The call makes
 * no hipMalloc, hipFree or other device allocation, captures no graph and
 * does not time its launches (profile is ignored). A batch whose scratch
 * does not fit the array fails with MORAY_ENOMEM and a message that says so
 * (the ray queues take what the other buffers leave; a queue too small for
 * the batch is handled as in moray_trace, by tracing its trees in chunks,
 * and fails with MORAY_EQUEUE only when one tree does not fit); so does a
 * batch whose per-tree statistics and finalize partial sums exceed the
 * context's 1 MiB pinned read-back staging. Every call on one GPU uses that
 * GPU's one array and leaves its contents behind (each call zeroes what it
 * needs zeroed): calls that overlap on one GPU, from any contexts or
 * threads, race and must not be made. Arguments, flags, results and errors
 * otherwise as moray_trace; the context's own buffers are not touched. */
moray_status moray_trace_noalloc(moray_ctx* ctx, const moray_problem* probs, int n_probs, unsigned flags,
                                 moray_result* outs);

/* Launch settings chosen by moray_autotune. */
typedef struct {
  int chunk_rays;             /* rays a wave claims from a level queue per atomic */
  int refill_lanes;           /* idle lanes of 64 that make a wave refetch rays */
  int reserve_rays;           /* next-level queue slots a wave reserves per atomic (split-queue depth) */
  int waves_per_cu;           /* persistent trace waves per compute unit */
  double first_ms;            /* fastest solve of the batch with the settings the context had */
  double best_ms;             /* fastest solve with the chosen settings */
  int trials;                 /* settings timed */
} moray_tune_result;

/* Autotuner (not part of the paper's method): time the batch under candidate
 * launch settings, one coordinate-descent pass over chunk size, refill
 * threshold, reservation block and waves per compute unit (each setting the
 * fastest of three solves), and keep the fastest in the context for later
 * moray_trace calls. Fields as in moray_trace (flags); results go to scratch
 * device memory. max_trials bounds the settings timed (0 = all candidates).
 * out may be NULL. Errors as in moray_trace; on error the context keeps the
 * settings it had. */
moray_status moray_autotune(moray_ctx* ctx, const moray_problem* probs, int n_probs, unsigned flags,
                            int max_trials, moray_tune_result* out);

/* Persistent autotune cache (not part of the paper's method): moray_autotune
 * whose outcome is kept in the text file `path` (host path, NUL-terminated).
 * The key is the library version, the device's architecture name and compute
 * units, the context's precision and deposit-table setting, and a hash of the
 * batch's shape (grid sizes and nesting, source and group counts, the trace
 * parameters; not the field values, source positions or photon rates). On a
 * hit (the last valid line with this key) the context takes the recorded
 * settings without timing anything, `out` receives them with the recorded
 * timings, and *from_cache is set to 1. On a miss the file is opened for
 * appending first (MORAY_EINVAL, nothing changed, when it cannot be), the
 * batch is tuned as by moray_autotune, and one line is appended; if that
 * line cannot be written the context keeps the new settings and the call
 * returns MORAY_EINVAL. Lines that do not parse or whose settings are out of
 * range for the device are ignored. Concurrent processes may share a file:
 * each appends whole lines. from_cache may be NULL. Other errors as in
 * moray_autotune. */
moray_status moray_autotune_cached(moray_ctx* ctx, const char* path, const moray_problem* probs, int n_probs,
                                   unsigned flags, int max_trials, moray_tune_result* out, int* from_cache);

/* Settings of moray_equilibrate. */
typedef struct {
  double alpha_b;             /* case-B recombination coefficient, cm^3/s (2.59e-13 at 1e4 K), > 0 */
  double damping;             /* weight of the new root in each update, in (0, 1] */
  double tol;                 /* stop once the largest change of x in an update is below tol, > 0 */
  int max_iter;               /* at most this many updates, >= 1 */
} moray_equilibrium_params;

/* Photo-ionisation equilibrium around the trace (section 2.2, Eq. dndt, the
 * update that follows the ray tracing in section 3.1), hydrogen only: no
 * collisional term, n_e = n_p = (1 - x) n_H and dn/dt = 0, so in every cell
 *     alpha_b n_H (1 - x)^2 = k_ph x   for the neutral fraction x.
 * Damped fixed-point iteration: from the problem's x_hi, trace, solve that
 * quadratic per cell (its root in [0, 1], computed as
 * 2a / ((2a + k) + sqrt(k^2 + 4ak)) with a = alpha_b n_H, and x = 1 where
 * n_H = 0), set x <- (1 - damping) x + damping x_root, and repeat until the
 * largest change of x is below tol or max_iter updates are done; then trace
 * once more with the final x into `out` (host or device results by flags, as
 * in moray_trace; escaped_sg is filled when given).
 * The problem must have device-resident fields (flags must include
 * MORAY_FIELDS_ON_DEVICE); every grid is updated, except the root cells a
 * child grid covers, which keep their x (their field lives in the child), and
 * the largest change is taken over all grids. Its x_hi arrays are updated in
 * place: they hold the float32 neutral fraction of every iterate and, on
 * return, of the last one; the iteration itself keeps x in float64, which
 * x_out (device memory, [total cells] in grid order, or NULL) receives.
 * *iterations (or NULL) receives the number of updates made. Returns
 * MORAY_EINVAL for bad parameters or host fields (nothing is changed then),
 * and the errors of moray_trace (x_hi then holds the last iterate). */
moray_status moray_equilibrate(moray_ctx* ctx, const moray_problem* prob, unsigned flags,
                               const moray_equilibrium_params* params, double* x_out, moray_result* out,
                               int* iterations);

/* Settings of moray_evolve. */
typedef struct {
  double alpha_b;             /* case-B recombination coefficient, cm^3/s (2.59e-13 at 1e4 K), > 0 */
  double eps_ion;             /* largest fractional change of the neutral density per step (Eq. dtelec), > 0 */
  double tau_front;           /* a cell limits the step when its own optical depth sigma_bar n_H x dx
                                 exceeds this (0.5), >= 0 */
  double dt_max;              /* step of the cells outside the front and bound of every step, s, > 0 */
  double t_end;               /* time to evolve for, s, > 0 */
  int max_steps;              /* at most this many steps, >= 1 */
} moray_evolve_params;

/* Time-stepped photo-ionisation (the radiative-transfer timestep of section
 * 3.4.1 around the cycle of section 3.1, with the hydrogen-only rate equation
 * of section 2.2, Eq. dndt, as its chemistry step: no collisional term,
 * n_e = n_p = (1 - x) n_H for the neutral fraction x). From the problem's x_hi
 * and t = 0, each step
 *   1. traces with the current x (k_ph per cell, as moray_trace);
 *   2. takes per cell dt_cell = eps_ion / (k_ph + n_e alpha_b) (Eq. dtelec)
 *      where the cell's own optical depth sigma_bar n_H x dx exceeds tau_front
 *      (sigma_bar = sum_g photon_frac_g sigma_g), dt_max elsewhere, and at
 *      most dt_max; smooths that field over 3^3 cells with the binomial
 *      weights (1/4, 1/2, 1/4) per axis, normalised over the neighbours inside
 *      the grid; dt = its minimum, at most twice the previous step (Eq.
 *      dtchange, from the second step on), dt_max and t_end - t;
 *   3. advances every cell by the exact solution over dt of
 *      dx/dt = alpha_b n_H (1 - x)^2 - k_ph x with k_ph held (cells with
 *      n_H = 0 keep x), and t += dt;
 * until t reaches t_end or max_steps steps are done; then traces once more
 * with the final x into `out` (host or device results by flags, as in
 * moray_trace; escaped_sg is filled when given).
 * The problem must have device-resident fields (flags must include
 * MORAY_FIELDS_ON_DEVICE). With child grids, each grid's limits are smoothed
 * within that grid, the step is the smallest over the grids, and the root
 * cells a child covers keep their x and take dt_max as their limit. The x_hi
 * arrays are updated in place and hold the float32 neutral fraction of every
 * step; the evolution keeps x in float64, which x_out (device memory, [total
 * cells] in grid order, or NULL) receives. *steps, *t_reached and dt_steps
 * (host memory, [max_steps]) receive, when not NULL, the steps taken, the
 * time reached and each step's dt. Returns MORAY_EINVAL for bad parameters or
 * host fields (nothing is changed then), and the errors of moray_trace (x_hi
 * then holds the last step's x). */
moray_status moray_evolve(moray_ctx* ctx, const moray_problem* prob, unsigned flags,
                          const moray_evolve_params* params, double* x_out, moray_result* out, int* steps,
                          double* t_reached, double* dt_steps);

/* Time-dependent rays (section 2.1: a ray halts once it has travelled c dt_P
 * and continues from there in the next step, which keeps the time derivative
 * of the transfer equation; section 3.1 step 3j). A moray_td holds, on the
 * device, the rays in flight between steps of one problem (a root grid and
 * its children).
 *
 * moray_td_create: state for problems shaped like prob (its grid sizes and
 * offsets, source and group counts and level_init; its fields may change from
 * step to step).
 * c_dt is c dt_P in root cells (c dt_P / dx_cm), > 0; pool_rays (1024 to
 * 2^34) bounds the rays in flight, with up to 63 empty records per wave of
 * each level launch (waves reserve the records of halted rays 64 at a time),
 * and each level's queue (both grow when a step needs more, see moray_td_step); the state holds
 * about 144 bytes of device memory per pool ray (two pools of 32 B, two
 * level queues of 28 B and the 24 B of sort buffers that order the rays in
 * flight, the latter only below 2^32 rays). The covering factor is
 * not taken. Returns MORAY_EINVAL for bad arguments, MORAY_ENOMEM when the
 * buffers do not fit the context's HBM budget.
 *
 * moray_td_step: one step. The rays in flight continue; when emit is nonzero
 * the sources emit new seed rays with their current ndot (a source that emits
 * in some steps only is a pulsed source). A ray that has completed a steps
 * since its emission halts at the radius (a + 1) c_dt from its source: its
 * segment in that cell ends there and deposits accordingly, and it keeps its
 * remaining photons for the next step. Splits, truncation and escape are
 * those of moray_trace, so when the fields and sources stay fixed, a step
 * made after every ray has had time to leave deposits what moray_trace does.
 * flags must be MORAY_FIELDS_ON_DEVICE | MORAY_OUT_ON_DEVICE; out receives
 * this step's k_ph, heating and totals (emitted counts this step's emission;
 * emitted + the previous step's held = absorbed + escaped + truncated + held)
 * and *held (or NULL) the photon rate of the rays in flight after the step.
 * accel must be NULL. When the pool or a level queue overflows, the step
 * keeps the rays in flight from before it, grows the pools and queues (at
 * least doubling them, within the context's HBM budget) and runs again;
 * MORAY_EQUEUE when they cannot grow, with the state as before the step (it
 * may be retried, e.g. after other buffers were freed). Not thread-safe per
 * state.
 *
 * moray_td_free: release the state (before its context). */
typedef struct moray_td moray_td;
moray_status moray_td_create(moray_ctx* ctx, const moray_problem* prob, double c_dt, size_t pool_rays,
                             moray_td** td);
moray_status moray_td_step(moray_ctx* ctx, moray_td* td, const moray_problem* prob, unsigned flags, int emit,
                           moray_result* out, double* held);
void moray_td_free(moray_ctx* ctx, moray_td* td);

/* Serving: queue n_probs problems (n_probs >= 1) for asynchronous tracing and
 * return at once with a ticket. Not part of the paper's method: this is the
 * request loop around it. A host thread of the context runs launch
 * generations of the trace kernel; each generation advances every admitted
 * problem's rays by one HEALPix level, and problems queued meanwhile are
 * admitted between generations, in arrival order, as their cells, absorber
 * columns, accumulators, table slots and ray-queue share fit the context's HBM
 * budget. Their rays then share the launches with the problems already
 * running, and a problem leaves as soon as it has no rays left (its k_ph,
 * heating and totals are written then). A problem's results are the same as
 * from moray_trace up to the order of floating-point additions into each cell.
 * Inputs (field arrays, descriptors) and outputs (the moray_result structs and
 * their buffers) must stay valid until moray_query reports the ticket done.
 * Returns MORAY_EINVAL for invalid problems (nothing is queued), MORAY_ENOMEM
 * when the serving pools cannot be created inside the budget; a problem that
 * cannot fit even alone, or whose fields hold invalid values, completes with
 * that error on its ticket. While a context has queued or running solves,
 * moray_trace on it returns MORAY_EBUSY. */
moray_status moray_trace_async(moray_ctx* ctx, const moray_problem* probs, int n_probs, unsigned flags,
                               moray_result* outs, moray_ticket* ticket);

/* Wait up to wait_ms milliseconds (0: do not wait, < 0: until done) for a
 * ticket. Returns MORAY_EBUSY if it is not done yet, otherwise the ticket's
 * status (MORAY_OK when every problem's results are written), after which the
 * ticket is forgotten; MORAY_EINVAL for an unknown ticket. */
moray_status moray_query(moray_ctx* ctx, moray_ticket ticket, int wait_ms);

/* Serving failure handling (not part of the paper's method). Both act at the
 * serving engine's next launch-generation boundary, so every kernel in
 * flight finishes normally; the problems of the ticket that have not
 * finished by then leave the engine (pending ones are dropped, running ones
 * have their rays removed from the ray queue and their memory returned to
 * the pools), and moray_query then reports the ticket's status. Problems of
 * the ticket that finished before keep their results; the outputs of the
 * others are undefined. Other tickets are not affected.
 *
 * moray_set_deadline: the ticket fails with MORAY_ETIMEOUT unless all of its
 * problems are done `seconds` from now (CLOCK_MONOTONIC; seconds >= 0).
 * moray_cancel: the ticket fails with MORAY_ECANCELED.
 * Both return MORAY_EINVAL for an unknown ticket (or a negative time), and
 * MORAY_OK otherwise, also when the ticket is already done (its status is
 * then the one it finished with). */
moray_status moray_set_deadline(moray_ctx* ctx, moray_ticket ticket, double seconds);
moray_status moray_cancel(moray_ctx* ctx, moray_ticket ticket);

/* Release every device and host resource of the context (NULL is allowed).
 * Queued and running asynchronous solves are finished first. */
void moray_free(moray_ctx* ctx);

/* Description of the last error on this context (never NULL). */
const char* moray_last_error(const moray_ctx* ctx);

/* Library version as "major.minor.patch". */
const char* moray_version(void);

#ifdef __cplusplus
}
#endif
#endif
