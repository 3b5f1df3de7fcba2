// Internal layout shared by the host runtime and the HIP kernels of the
// adaptive ray tracer. Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace moray {

constexpr int kMaxLevel = 29;
constexpr int kLevels = kMaxLevel + 2;
constexpr int kWave = 64;
constexpr int kTraceBlock = 256;
constexpr int kFinalBlock = 256;
constexpr int kFinalCellsPerThread = 4;
constexpr unsigned long long kReserveMax = 256;   // next-level queue slots a wave reserves per atomic
// Time-dependent rays: a wave reserves the halt list's records in blocks of
// kHaltBlock; the records of its last block that it does not fill are empty,
// with the level kHaltHole (above every HEALPix level, so they sort last).
// The list's one counter takes an atomic per block from every wave of the
// device: blocks of 256 rather than 64 records took a steady step of the
// 128^3 workload (c dt_P = 32 cells) from 12.8 to 12.05 ms, at the price of
// up to 255 empty records per wave and launch in the list and its sort.
constexpr int kHaltBlock = 256;
constexpr int kHaltHole = 31;
static_assert(kLevels <= kHaltHole, "empty halt records need a level above every real one");
constexpr uint32_t kNoTree = 0xffffffffu;      // tree index of an empty queue slot
constexpr int kDropRanges = 16;                // tree ranges one queue filter pass removes (serving)
constexpr int kSkip = 0, kStarted = 1, kEscaped = 2;
constexpr int kCacheLog2 = 9;                  // per-wave LDS deposit cache: 512 entries
constexpr int kCacheEntries = 1 << kCacheLog2;
constexpr uint32_t kNoSlot = 0xffffffffu;      // empty cache entry
constexpr double kHydrogenMassG = 1.6735575e-24;   // mass of a hydrogen atom, g
constexpr double kLightCms = 2.99792458e10;        // speed of light, cm/s
constexpr int kEvictCap = 128;                 // per-wave buffer of evicted sums (drained at > 64)
constexpr int kTallyLog2 = 7;                  // per-block LDS table of per-tree statistics: 128 entries
constexpr int kTallySlots = 1 << kTallyLog2;
constexpr int kTallyProbes = 16;               // entries a tree tries before it adds to global counters
constexpr int kStageFlush = 16;                // split parents staged before their children are written
constexpr int kStageCap = kStageFlush + kWave; // one iteration adds at most 64 parents

// One uniform grid patch of one problem, in the batch-wide cell numbering.
struct GridDev {
  int nx, ny, nz;
  int ox, oy, oz;          // lower corner in root cells (children), 0 for roots
  int is_child;            // 0: root (unit scale), 1: 2x-refined child of the root
  int problem;
  long long cell_off;      // first cell of this grid in the batch-wide numbering
  double dx_cm;            // local cell width
  const float* n_h;        // device copies (or caller device memory) of the inputs
  const float* x_hi;
  double* out_kph;         // where finalize writes this grid's k_ph and heating
  double* out_heat;
  double* out_acc;         // radiation-pressure acceleration: component k of local cell i at
                           // out_acc[k * (problem's cells) + i]; NULL when not asked for
};

struct ProblemDev {
  int root_grid;           // index of the root grid in the grid table
  int n_groups;
  long long cell_off;      // first cell of the problem
  long long n_cells;       // cells of all its grids
  long long acc_off;       // first accumulator slot: group g of cell c is acc_off + g*n_cells + (c - cell_off)
  int eexc_off;            // first of its n_groups (E - E_ion) values in erg
  int pad;
  int acc_stride = 1;      // 1: one float64 sum per (group, cell), group g of cell c at
                           //   acc_off + g*n_cells + (c - cell_off);
                           // 2 (optically-thin approximation): a 16-byte record per (group, cell) at
                           //   acc_off + 2*(g*n_cells + (c - cell_off)): absorbed rate, then the
                           //   deposits of thin rays in cells that hold their source (nothing removed);
                           // 4 (radiation pressure asked for): a 32-byte record per (group, cell) at
                           //   acc_off + 4*(g*n_cells + (c - cell_off)): absorbed rate, then the three
                           //   components of the absorbed momentum rate
  // optically-thin approximation: the mark of the problem's (source, group) tree t (tree table
  // index sg_first + t) on cell c is the byte mark[mark_off + t*n_cells + (c - cell_off)], t < mark_trees
  int mark_trees = 0;      // 0: the problem does not use the approximation
  int sg_first = 0;        // its first tree in the tree table (its trees are consecutive)
  long long mark_off = 0;
};

// One (source, group) ray tree, with the shape of its problem's root grid so
// a ray can start without another table lookup.
struct SgDev {
  double sx, sy, sz;       // source position, root cells
  double P0;               // photon rate of one seed ray
  double pmin0;            // p_min_frac * P0 (quartered per level below the seeds)
  long long acc_slot;      // accumulator of cell c (batch numbering) is acc[acc_slot + c]
  float sigma32;
  float split_t2_base;     // 12 / (4 pi phi_c), float; FLT_MAX when the problem never splits
  int level_init;
  int level_max;
  int gen0;                // launch generation of the tree's seed rays: a ray of generation g is at
                           // HEALPix level level_init + (g - gen0)
  int root_grid;           // grid-table index of the problem's root grid
  int rnx, rny, rnz;       // its shape
  long long rcell_off;     // its first cell
  double sigma64;          // cross-section, cm^2
  double four_pi_phi_c;    // 4 pi phi_c of its problem
  int problem;
  int covering;            // scale deposits into the accumulators by the covering factor
  uint32_t acc_stride = 1; // its problem's acc_stride: the deposit into cell c (batch numbering) goes to
                           //   acc[acc_slot + acc_stride * c], the momentum (stride 4) to the next three
  double mom_scale;        // E_ph / c of the group (erg s/cm), 0 without radiation pressure
  double r_halt = __builtin_huge_val();   // time-dependent rays: radius (root cells) where the
                                          // tree's rays halt in this step
  // optically-thin approximation (tau_thin > 0)
  double tau_thin = 0.0;   // a ray is thin in a cell while its optical depth on leaving it is below this
  double four_pi_phi_thin; // 4 pi min(1, phi_c): the split threshold of thin rays
  float split_t2_thin;     // 12 / (4 pi min(1, phi_c)), float; FLT_MAX when the problem never splits
  long long mark_base;     // its mark on cell c (batch numbering) is the byte mark[mark_base + c]
  double thin_coef;        // sigma Ndot_g / (4 pi dx_root^2): the thin rate at r root cells is thin_coef / r^2
};

struct SgStats {
  double esc_P;            // escaped photon rate
  double trunc_P;          // photon rate left in truncated rays
  unsigned long long segs, splits, n_esc, n_trunc;
  unsigned long long thin_segs;   // of segs, those of optically thin rays
};

// A level queue is split into up to kSegMax segments of seg_cap slots, each
// with its own write and claim counters, so the same-address atomics that
// reserve and claim rays spread over many addresses (a float64 or integer
// atomic on one address serialises at the memory side).
constexpr int kSegMax = 64;

struct Counters {
  unsigned long long count[kLevels][kSegMax];   // slots written to each segment of each level queue
  unsigned long long head[kLevels][kSegMax];    // slots claimed from each segment
  unsigned long long lost_rays;                 // children dropped on overflow
  double lost_P;
  unsigned int err;                             // bit flags, see kErr*
  unsigned int pad;
  unsigned long long halt_count;                // time-dependent rays halted in this step
  unsigned long long halt_levels[kLevels];      // of them, per HEALPix level
};

constexpr unsigned kErrOverflow = 1u;
constexpr unsigned kErrBadInput = 2u;
constexpr unsigned kErrInternal = 8u;

// Level queue, structure of arrays. The radius is float64 in both precision
// modes so a child starts exactly where its parent's exit distance put it.
struct RayQueue {
  uint64_t* pix;
  uint32_t* sg;
  double* r;
  double* P;
};

template <typename R>
struct TraceArgs {
  const GridDev* grids;
  const ProblemDev* probs;
  const SgDev* sgs;
  const R* kappa;          // n_H x_HI dx_root per leaf cell; -(child+1) on covered root cells
  double* acc;             // absorbed photons/s per (problem, group, leaf cell)
  uint32_t rec_base;       // deposit keys >= rec_base start 4-sum radiation-pressure records (32-byte aligned)
  RayQueue in, out;                    // nseg segments of seg_cap slots each
  unsigned long long seg_cap;
  int nseg;                            // segments per level queue: a power of two
  Counters* ctr;
  SgStats* stats;
  int gen;                             // launch generation (the HEALPix level in a one-shot solve)
  int cin, cout;                       // counter rows of the input and output queues
  int seed_level;                      // HEALPix level of the seed rays of this launch
  int seed_sg_begin, seed_sg_end;      // trees seeded in this launch
  int chunk;                           // rays claimed per atomic
  int refill;                          // idle lanes that trigger a refill
  unsigned max_steps;                  // hard cap on cells per ray (never reached)
  unsigned long long reserve;          // next-level slots a wave reserves at once (multiple of 4)
  // time-dependent rays: where rays halted in this step go (halt_cap records; level in halt_lev)
  RayQueue halt;
  int* halt_lev;
  unsigned long long halt_cap;
  uint32_t tree_fold;                  // statistics of tree k are kept under k % tree_fold (the trees
                                       // of one batch), so the block tables hold one batch's trees
  uint8_t* mark;                       // optically-thin marks (see ProblemDev), or NULL
  const double* kappa64;               // float kernels with the optically-thin approximation: the
                                       // columns in float64 (same layout as kappa), else NULL
};

// One finalize block: cells [first, first + count) of one grid.
struct FinalBlock {
  int grid;
  int count;
  long long first;
};

}  // namespace moray
