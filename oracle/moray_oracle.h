/*
 * moray_oracle.h -- plain FP64 CPU reference of the single-pass adaptive ray
 * trace (Wise & Abel, Enzo+Moray: section 2.1 adaptive ray tracing, section
 * 2.2 radiation field, section 3.1 steps 1-3).
 *
 * TEST INFRASTRUCTURE ONLY. This library exists to check the GPU library
 * against. Only the test-suite, the smoke check and the benchmark's CPU
 * baseline may call it; the product path never links or loads it. It shares
 * no code, header, table or helper with the GPU library.
 *
 * Units: positions and radii in cells of the root grid; dx in cm; densities
 * in cm^-3; photon rates in photons/s; energies in eV on input, erg on output.
 * Fields are float32, x fastest (index i + nx*(j + ny*k)).
 */
#ifndef MORAY_ORACLE_H
#define MORAY_ORACLE_H
#include <stddef.h>
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int nx, ny, nz;          /* cells */
  double dx_cm;            /* cell width */
  const float* n_h;        /* hydrogen density */
  const float* x_hi;       /* neutral fraction */
  int parent;              /* -1 root, 0 child of the root (refinement 2) */
  int offset[3];           /* lower corner in root cells (children only) */
} orc_grid;

typedef struct { double x, y, z, ndot; } orc_source;   /* root cells; photons/s */

typedef struct {
  int n_groups;
  const double* energy_ev;
  const double* sigma_cm2;
  const double* frac;      /* photon-number fraction of each group */
  double e_ion_ev;
} orc_spectrum;

typedef struct {
  double phi_c;            /* split when fewer than phi_c rays cross a cell face */
  int level_init;          /* HEALPix level of the seed rays */
  int level_max;           /* rays at this level are never split */
  double p_min_frac;       /* a ray ends once P < p_min_frac * P0 */
  int covering;            /* nonzero: scale each segment's contribution to the absorbed
                              and energy rates (not its attenuation) by the covering
                              factor f_c of section 2.3 (Eqs. midpoint, fc) */
  double tau_thin;         /* > 0: the optically-thin approximation of section 2.4 (Eq.
                              optthin) for rays whose optical depth from the source is
                              below tau_thin when they leave a cell; 0: off. Single pass
                              only (orc_trace_td and accel reject it). */
} orc_params;

typedef struct {
  double emitted, absorbed, escaped, truncated;       /* photons/s, compensated sums */
  uint64_t segments, rays_seeded, splits, rays_escaped, rays_truncated;
  /* optically-thin approximation (tau_thin > 0; zero otherwise): segments of
     rays that were thin in their cell, the (cell, source, group) rates set
     from Eq. optthin, and the smallest |tau_exit - tau_thin| / tau_thin of
     any thin-or-thick decision (INFINITY when none was taken) */
  uint64_t thin_segments, thin_marked;
  double thin_margin;
} orc_totals;

/* Trace every (source, group, seed pixel) ray tree of one problem.
 * Outputs (caller-allocated, concatenated over grids in grid order, every one
 * overwritten): absorbed [photons/s per cell], energy [erg/s per cell], k_ph
 * [1/s per absorber], heating [erg/s per absorber] (with tau_thin > 0 these
 * include the optically-thin rates, which `absorbed` and `energy` do not: see
 * the notes in moray_oracle.c); escaped_sg
 * [n_src*n_groups] escaped photons/s per (source, group) (may be NULL).
 * n_threads > 1 splits (source, group) items cyclically over OpenMP threads,
 * each with private accumulators summed in thread order.
 * Returns 0, or -1 on invalid input (nothing written). */
int orc_trace(const orc_grid* grids, int n_grids, const orc_source* src, int n_src,
              const orc_spectrum* spec, const orc_params* par, int n_threads,
              double* absorbed, double* energy, double* k_ph, double* heating,
              double* escaped_sg, orc_totals* tot);

/* orc_trace, and when accel is not NULL also the radiation-pressure
 * acceleration of the gas (section 2.5.4, Eq. radpres): every absorbed
 * photon rate dP hands the momentum rate dP E_ph / c along its ray to its
 * cell, and accel = (that sum) / (m_H n_H V), m_H = 1.6735575e-24 g, in
 * cm/s^2 (0 where n_H = 0). accel holds 3 planes (x, y, z) of the
 * concatenated cells: accel[k * total_cells + cell]. */
int orc_trace_accel(const orc_grid* grids, int n_grids, const orc_source* src, int n_src,
                    const orc_spectrum* spec, const orc_params* par, int n_threads,
                    double* absorbed, double* energy, double* k_ph, double* heating,
                    double* escaped_sg, double* accel, orc_totals* tot);

/* A ray in flight between the steps of a time-dependent trace. */
typedef struct {
  int src, grp;            /* its source and group */
  int level;               /* HEALPix level */
  int age;                 /* steps completed since its emission */
  uint64_t pix;            /* nested pixel */
  double r, P, P0;         /* radius (root cells), photon rate, unattenuated share */
} orc_tray;

/* One step of a trace with time-dependent rays (section 2.1: a ray is
 * halted once it has travelled c dt_P and continues from there in the next
 * step; section 3.1 step 3j). The rays in[0..n_in) continue, one step older;
 * when emit is set the sources emit new seed rays (their totals count as
 * this step's `emitted`). A ray that has completed a steps since its emission
 * halts at the radius (a + 1) c_dt (root cells, c_dt = c dt_P / dx_root):
 * its segment in that cell ends there and deposits accordingly, and the ray,
 * with its remaining photons, goes to out (at most out_cap; *n_out receives
 * the count, and when it exceeds out_cap the call returns -2). *held
 * receives the photon rate of the halted rays. Splitting, truncation and
 * escape are those of the single pass, so once every ray of a static problem
 * has had time to leave, a step's k_ph equals the single pass's.
 * One thread; outputs as in orc_trace. Returns 0, -1 on invalid input, -2
 * when out is too small. */
int orc_trace_td(const orc_grid* grids, int n_grids, const orc_source* src, int n_src,
                 const orc_spectrum* spec, const orc_params* par, double c_dt, int emit,
                 const orc_tray* in, size_t n_in, orc_tray* out, size_t out_cap, size_t* n_out,
                 double* held, double* absorbed, double* energy, double* k_ph, double* heating,
                 orc_totals* tot);

/* HEALPix nested-scheme pixel centre as a unit vector (z = polar axis,
 * phi = 0 along +x). */
void orc_pix2vec_nest(int level, uint64_t pix, double v[3]);

/* Constants the oracle uses (for the unit pins). */
double orc_const_ev_erg(void);

#ifdef __cplusplus
}
#endif
#endif
