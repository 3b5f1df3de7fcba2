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

// One uniform grid patch of one problem, in the batch-wide cell numbering.
struct GridDev {
  int nx, ny, nz;
  int ox, oy, oz;          // lower corner in root cells (children), 0 for roots
  int is_child;            // 0: root (unit scale), 1: 2x-refined child of the root
  int problem;
  long long cell_off;      // first cell of this grid in the batch-wide arrays
  double dx_cm;            // local cell width
  double inv_vol;          // 1 / dx^3
  const float* n_h;        // device copies (or caller device memory) of the inputs
  const float* x_hi;
  double* out_kph;         // where finalize writes this grid's k_ph and heating
  double* out_heat;
};

struct ProblemDev {
  int root_grid;           // index of the root grid in the grid table
  int level_max;
  double four_pi_phi_c;    // 4 pi phi_c, the canonical split constant
  float split_t2_base;     // 12 / (4 pi phi_c) as float (local-cell units^2 at level 0), inf if phi_c = 0
};

// One (source, group) ray tree.
struct SgDev {
  double sx, sy, sz;       // source position, root cells
  double P0;               // photon rate of one seed ray
  double pmin0;            // p_min_frac * P0 (halved twice per level below the seeds)
  double eexc_erg;         // (E - E_ion) in erg
  double sigma64;          // cross-section, cm^2
  float sigma32;
  float src_err;           // |s - float(s)| max over axes (0 for sources on the 2^-12 lattice)
  int problem;
  int level_init;
};

struct SgStats {
  double esc_P;            // escaped photon rate
  double trunc_P;          // photon rate left in truncated rays
  unsigned long long segs, splits, n_esc, n_trunc;
};

struct Counters {
  unsigned long long count[kLevels];   // rays written to each level queue
  unsigned long long head[kLevels];    // rays claimed from each level queue
  unsigned long long lost_rays;        // children dropped on overflow
  double lost_P;
  unsigned int err;                    // bit flags, see kErr*
  unsigned int pad;
};

constexpr unsigned kErrOverflow = 1u;
constexpr unsigned kErrBadInput = 2u;
constexpr unsigned kErrNonFinite = 4u;
constexpr unsigned kErrInternal = 8u;

template <typename R>
struct RayQueue {
  uint64_t* pix;
  uint32_t* sg;
  R* r;
  double* P;
};

template <typename R>
struct TraceArgs {
  const GridDev* grids;
  const ProblemDev* probs;
  const SgDev* sgs;
  const R* kappa;          // n_H x_HI dx_root per leaf cell; -(child+1) on covered root cells
  double* acc_abs;         // absorbed photons/s per leaf cell (batch-wide)
  double* acc_heat;        // absorbed energy erg/s per leaf cell
  RayQueue<R> in, out;
  unsigned long long capacity;
  Counters* ctr;
  SgStats* stats;
  int level;
  int seed_sg_begin, seed_sg_end;      // trees seeded at this level
  int chunk;                           // rays claimed per atomic
  int refill;                          // idle lanes that trigger a refill
  unsigned max_steps;                  // hard cap on cells per ray (never reached)
};

}  // namespace moray
