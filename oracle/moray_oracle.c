/*
 * moray_oracle.c -- plain, slow FP64 CPU reference of the single-pass
 * adaptive ray trace of Wise & Abel (Enzo+Moray).
 *
 * TEST INFRASTRUCTURE ONLY: it exists to check the GPU library against and is
 * called only by the test-suite, the smoke check and the benchmark's CPU
 * baseline. Nothing here is shared with the GPU library.
 *
 * What it computes, in the paper's order (section 3.1, steps 1-3):
 *   Step 1  For every source and energy group, 12*4^l0 rays on the HEALPix
 *           nested pixel centres of level l0, each with an equal share of the
 *           group's photon rate (section 2.1).
 *   Step 2  All radiation fields start at zero.
 *   Step 3  Every ray is marched cell by cell. In each cell:
 *     3b/3d the exit distance t_exit = min over axes of (next boundary plane
 *           - source coordinate) / direction component (Eq. trace);
 *     3e    if the ray's solid angle at t_exit exceeds phi_c rays per cell
 *           face, i.e. 12*4^l < 4*pi*phi_c*t_exit^2 in cell units (Eq. split),
 *           the ray is replaced by its four nested children 4p..4p+3, which
 *           keep the radius, take a quarter of the photon rate each and are
 *           traced next (child 0 first);
 *     3f    otherwise the segment dr = t_exit - r absorbs
 *           dP = P (1 - exp(-tau)) with tau = sigma n_H x_HI dr (Eqs. dtau,
 *           flux); dP is added to the cell's absorbed-photon rate and
 *           dP (E - E_ion) to its heating rate (Eqs. kph, gamma);
 *     3h    P -= dP, r = t_exit;
 *     3i    the ray ends once P < p_min_frac * P0 (its unattenuated share);
 *     3k    a ray leaving the root grid escapes (isolated boundaries); a ray
 *           entering a root cell covered by a child grid continues in the
 *           child at the crossing point (step 3c), and returns to the root
 *           when it leaves the child.
 *   Finally k_ph = absorbed / (n_H x_HI V_cell) and heating likewise; the
 *   time step dt_P cancels because P is a rate (single pass, infinite c).
 *
 * Readings of points the paper leaves open (each also listed in the design
 * notes): the split is tested at the exit radius (step 3e); a split is strict
 * (<); children may split again at once; a point on a cell plane belongs to
 * the upper cell when the direction component is >= 0, else the lower one;
 * exit-axis ties go to the lowest axis; dr = max(0, t_exit - r) and r never
 * decreases; the residual of a ray cut off by p_min_frac is tallied as
 * "truncated" so that absorbed + escaped + truncated = emitted.
 *
 * Optically-thin approximation (section 2.4, Eq. optthin; params.tau_thin >
 * 0). Every ray carries its optical depth tau from the source. In each cell
 * the ray is thin when tau + tau_cell < tau_thin (tau once it leaves the
 * cell; strict <). A thin ray
 *   - is split against phi_thin = min(1, phi_c) rays per cell face instead
 *     of phi_c: one ray per cell suffices where the gas is thin;
 *   - removes no photons, so its P stays its unattenuated share P0;
 *   - sets the cell's rate once per (source, group): the first thin ray of
 *     that item to leave the cell adds k = sigma P / (Omega_ray r_cell^2) to
 *     k_ph and k (E - E_ion) to the heating, where Omega_ray = 4 pi / N_pix(l)
 *     is the ray's solid angle and r_cell the distance (cm) from the source
 *     to the cell centre, and marks the cell for that item (a byte per cell
 *     here, one bit per item of a 32-bit field in the paper); a ray that only
 *     grazes the cell, along a segment shorter than 2^-40 of its exit radius
 *     (through an edge or a corner), does not count as crossing it;
 *   - in a cell that holds the source (inside or on its boundary, where
 *     r_cell can vanish), adds the general deposit P (1 - e^-tau_cell) to the
 *     cell's rate instead, still removing no photons, and marks nothing. (A
 *     child ray starts at its parent's radius along its own direction, so it
 *     can enter such a cell at r > 0.)
 * A ray that is not thin in its cell deposits and attenuates as above and is
 * never thin again (tau only grows). The thin rates enter k_ph and heating
 * but not `absorbed`, `energy` or the totals, as no photons are removed for
 * them; k_ph and heating of a cell without absorbers keep the thin rate.
 * Readings: the printed Eq. optthin divides by a linear angle and multiplies
 * by r_cell / r_ray, which does not give a rate; the text says the factor
 * moves the ray's flux from its exit point to the cell centre, and the flux of
 * a ray of solid angle Omega at radius r is P / (Omega r^2), so the rate at
 * the centre is sigma P / (Omega r_cell^2) (dt_P cancels, P being a rate).
 * Because a thin ray has lost no photons, P / Omega is the same for every thin
 * ray of one item, so the rate does not depend on which ray reaches the cell
 * first. The source's own cell and phi_thin are readings of points the paper
 * leaves open.
 */
#include "moray_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define EV_ERG 1.602176634e-12
#define C_CMS 2.99792458e10          /* speed of light, cm/s (exact) */
#define M_H_G 1.6735575e-24          /* mass of a hydrogen atom, g */
#define PI_D 3.14159265358979323846
#define MAX_LEVEL 29
#define STACK_MAX 512

double orc_const_ev_erg(void) { return EV_ERG; }

/* ---- Neumaier-compensated sum ------------------------------------------ */
typedef struct { double s, c; } csum;
static void cs_add(csum* a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
  else a->c += (x - t) + a->s;
  a->s = t;
}
static double cs_get(const csum* a) { return a->s + a->c; }

/* ---- HEALPix nested pixel centre (Gorski et al. 2005) ------------------- */
/* The pixel index is split into base face f and in-face coordinates (ix, iy)
 * (even bits -> ix, odd bits -> iy). The ring index is j = jr(f)*Ns - ix - iy - 1.
 * In the polar caps z = 1 - nr^2/(3 Ns^2), in the equatorial belt
 * z = 2(2Ns - j)/(3Ns); the azimuth is phi = (pi/2)(jp - (s+1)/2)/nr.
 * z and sin(theta) are formed from exact integers, and cos/sin(phi) are taken
 * of the angle reduced to the first octant, so multiples of pi/4 come out
 * exact and the pixel set keeps its mirror symmetries bit for bit. */
void orc_pix2vec_nest(int level, uint64_t pix, double v[3]) {
  static const int jrll[12] = {2, 2, 2, 2, 3, 3, 3, 3, 4, 4, 4, 4};
  static const int jpll[12] = {1, 3, 5, 7, 0, 2, 4, 6, 1, 3, 5, 7};
  const int64_t ns = (int64_t)1 << level;
  const uint64_t npface = (uint64_t)ns * (uint64_t)ns;
  const int face = (int)(pix / npface);
  const uint64_t ipf = pix % npface;
  int64_t ix = 0, iy = 0;
  for (int b = 0; b < level; ++b) {
    ix |= (int64_t)((ipf >> (2 * b)) & 1u) << b;
    iy |= (int64_t)((ipf >> (2 * b + 1)) & 1u) << b;
  }
  const int64_t jr = (int64_t)jrll[face] * ns - ix - iy - 1;
  int64_t nr;
  int kshift;
  double z, sth;
  if (jr < ns || jr > 3 * ns) {
    nr = (jr < ns) ? jr : 4 * ns - jr;
    const double den = 3.0 * (double)ns * (double)ns;
    z = (double)(3 * ns * ns - nr * nr) / den;
    sth = (double)nr * sqrt((double)(6 * ns * ns - nr * nr)) / den;
    if (jr > 3 * ns) z = -z;
    kshift = 0;
  } else {
    nr = ns;
    const int64_t m = 2 * (2 * ns - jr);
    z = (double)m / (3.0 * (double)ns);
    sth = sqrt((double)(9 * ns * ns - m * m)) / (3.0 * (double)ns);
    kshift = (int)((jr - ns) & 1);
  }
  int64_t jp = ((int64_t)jpll[face] * nr + ix - iy + 1 + kshift) / 2;
  if (jp > 4 * nr) jp -= 4 * nr;
  if (jp < 1) jp += 4 * nr;
  const int64_t num = 2 * jp - kshift - 1, den = 2 * nr;   /* phi / (pi/2) = num/den */
  const int64_t q = num / den, rem = num % den;
  double c, s;
  if (2 * rem == den) {
    c = s = sqrt(0.5);
  } else {
    const int64_t m = (2 * rem < den) ? rem : den - rem;
    const double beta = ((double)m / (double)den) * (PI_D / 2.0);
    const double cb = cos(beta), sb = sin(beta);
    if (2 * rem < den) { c = cb; s = sb; } else { c = sb; s = cb; }
  }
  double cx, cy;
  switch (q & 3) {
    case 0: cx = c; cy = s; break;
    case 1: cx = -s; cy = c; break;
    case 2: cx = -c; cy = -s; break;
    default: cx = s; cy = -c; break;
  }
  v[0] = sth * cx;
  v[1] = sth * cy;
  v[2] = z;
}

/* ---- grid hierarchy ------------------------------------------------------ */
typedef struct {
  const orc_grid* g;
  int n_grids;
  int* cover;          /* root cell -> index of the child grid over it, or -1 */
  size_t* cell_off;    /* first cell of grid q in the concatenated outputs */
  size_t n_cells;
} hier;

/* Cell containing coordinate x for a ray with direction component n: points on
 * a plane go to the upper cell when n >= 0 and to the lower cell otherwise. */
static long cell_rule(double x, double n) { return n >= 0.0 ? (long)floor(x) : (long)ceil(x) - 1; }
static long floor_half(long c) { return c >= 0 ? c / 2 : -((-c + 1) / 2); }

static int in_grid(const orc_grid* G, const long c[3]) {
  return c[0] >= 0 && c[1] >= 0 && c[2] >= 0 && c[0] < G->nx && c[1] < G->ny && c[2] < G->nz;
}

/* Enter child grid ch from root cell rc at radius r; along the crossing axis
 * the fine cell follows from the face crossed, along the others from the
 * position, kept inside the two fine cells under rc. */
static void enter_child(const hier* H, int ch, const long rc[3], int ax, int dir, const double s[3],
                        const double n[3], double r, long c[3]) {
  const orc_grid* G = &H->g[ch];
  for (int a = 0; a < 3; ++a) {
    const long lo = 2 * (rc[a] - G->offset[a]);
    if (a == ax) {
      c[a] = lo + (dir < 0 ? 1 : 0);
    } else {
      const double x = s[a] + r * n[a];
      long cl = cell_rule(2.0 * (x - (double)G->offset[a]), n[a]);
      if (cl < lo) cl = lo;
      if (cl > lo + 1) cl = lo + 1;
      c[a] = cl;
    }
  }
}

/* Locate the leaf cell holding the point s + r n. Returns -1 outside the root. */
static int locate(const hier* H, const double s[3], const double n[3], double r, int* q, long c[3]) {
  const orc_grid* R = &H->g[0];
  long rc[3];
  double x[3];
  for (int a = 0; a < 3; ++a) {
    x[a] = s[a] + r * n[a];
    rc[a] = cell_rule(x[a], n[a]);
  }
  if (!in_grid(R, rc)) return -1;
  const int ch = H->cover[rc[0] + (long)R->nx * (rc[1] + (long)R->ny * rc[2])];
  if (ch < 0) {
    *q = 0;
    c[0] = rc[0]; c[1] = rc[1]; c[2] = rc[2];
    return 0;
  }
  const orc_grid* G = &H->g[ch];
  for (int a = 0; a < 3; ++a) c[a] = cell_rule(2.0 * (x[a] - (double)G->offset[a]), n[a]);
  *q = ch;
  return 0;
}

typedef struct {
  double* absorbed;
  double* energy;
  double* mom;         /* NULL, or 3 planes of n_cells: momentum rate absorbed per cell (dyn) */
  uint64_t segments, splits, seeded, n_escaped, n_truncated;
  /* optically-thin approximation (NULL when off): rates per absorber set from
     Eq. optthin, deposits of thin rays in their source's cell (photons/s and
     erg/s, nothing removed), and the current item's marks, a byte per cell */
  double *k_thin, *h_thin, *thin_dep, *thin_energy;
  unsigned char* mark;
  uint64_t thin_segments, thin_marked;
  double thin_margin;
} acc;

typedef struct {
  const hier* H;
  const orc_source* src;
  const orc_spectrum* spec;
  const orc_params* par;
  double four_pi_phi_c;
  double four_pi_phi_thin;   /* 4 pi min(1, phi_c): the split threshold of thin rays */
} job;

/* a ray: HEALPix level and pixel, radius, photon rate, its unattenuated
   share P0, the radius where it halts in this step (infinite in a single
   pass), the steps since its emission, its optical depth from the source and
   whether it is still optically thin */
typedef struct { int level; uint64_t pix; double r, P, P0, rh; int age; double tau; int thin; } oray;

/* rays halted in this step (time-dependent rays) */
typedef struct {
  orc_tray* ray;
  size_t cap, n;
  int overflow;
  csum held;             /* their photon rate */
} halted;

/* Covering factor of a segment (section 2.3, Eqs. midpoint and fc), in
 * units of the local cell: the segment's midpoint lies D_c,i from the cell
 * centre along each axis, D_edge = 1/2 - max_i D_c,i from the closest face;
 * the pixel, taken as a square, is L_pix = R_0 theta_pix wide with R_0 the
 * radius where the segment starts and theta_pix = sqrt(4 pi / N_pix);
 * f_c = (1/2 + D_edge / L_pix)^2, and 1 once the pixel lies within the
 * face (f_c >= 1, which includes R_0 = 0). sl: source in local cells; r, dr:
 * entry radius and chord in root cells; h: local cells per root cell. */
static double covering_factor(const double sl[3], const double n[3], const long c[3], double r, double dr,
                              double h, int level) {
  const double rmid = (r + 0.5 * dr) * h;
  double dmax = 0.0;
  for (int a = 0; a < 3; ++a) {
    const double d = fabs(sl[a] + rmid * n[a] - ((double)c[a] + 0.5));
    if (d > dmax) dmax = d;
  }
  const double d_edge = 0.5 - dmax;
  const double theta = sqrt(4.0 * PI_D / ldexp(12.0, 2 * level));
  const double lpix = r * h * theta;
  if (!(lpix > 0.0)) return 1.0;
  const double f = 0.5 + d_edge / lpix;
  return f * f >= 1.0 ? 1.0 : f * f;
}

/* Trace one ray of item (si, gi) and all its descendants, depth first.
   A ray whose segment would end beyond its halting radius rh deposits up to
   rh and is recorded in *hl (time-dependent rays, section 2.1 and section
   3.1 step 3j) instead of going on. */
static void march(const job* J, int si, int gi, oray first, acc* A, csum* esc, csum* trunc, halted* hl) {
  const hier* H = J->H;
  const orc_source* S = &J->src[si];
  const double s[3] = {S->x, S->y, S->z};
  const double sigma = J->spec->sigma_cm2[gi];
  const double eexc = (J->spec->energy_ev[gi] - J->spec->e_ion_ev) * EV_ERG;
  const int lmax = J->par->level_max;

  oray stack[STACK_MAX];
  {
    int sp = 0;
    stack[sp++] = first;
    while (sp > 0) {
      oray R = stack[--sp];
    new_ray:;
      double n[3];
      orc_pix2vec_nest(R.level, R.pix, n);
      int q;
      long c[3];
      if (locate(H, s, n, R.r, &q, c) < 0) {   /* starts outside the root grid */
        cs_add(esc, R.P);
        A->n_escaped++;
        continue;
      }
      for (;;) {
        const orc_grid* G = &H->g[q];
        const double h = (q == 0) ? 1.0 : 2.0;
        double sl[3];
        for (int a = 0; a < 3; ++a) sl[a] = (q == 0) ? s[a] : h * (s[a] - (double)G->offset[a]);
        /* exit distance (root-cell units) and exit axis */
        double t_exit = INFINITY;
        int ax = -1;
        for (int a = 0; a < 3; ++a) {
          if (n[a] == 0.0) continue;
          const long b = (n[a] > 0.0) ? c[a] + 1 : c[a];
          const double ta = (((double)b - sl[a]) / n[a]) / h;
          if (ta < t_exit) { t_exit = ta; ax = a; }
        }
        const size_t cell = (size_t)c[0] + (size_t)G->nx * ((size_t)c[1] + (size_t)G->ny * (size_t)c[2]);
        const double nabs = (double)G->n_h[cell] * (double)G->x_hi[cell];
        /* optically-thin approximation: is the ray still thin once it leaves
           this cell? (the decision also picks its split threshold) */
        int thin = 0;
        if (R.thin) {
          const double dr0 = t_exit - R.r;
          const double tau_exit = R.tau + (dr0 > 0.0 ? sigma * nabs * ((dr0 * h) * G->dx_cm) : 0.0);
          thin = tau_exit < J->par->tau_thin;
          const double margin = fabs(tau_exit - J->par->tau_thin) / J->par->tau_thin;
          if (margin < A->thin_margin) A->thin_margin = margin;
        }
        /* split test at the exit radius, in units of the local cell */
        if (R.level < lmax) {
          const double u = t_exit * h;
          if (ldexp(12.0, 2 * R.level) < (thin ? J->four_pi_phi_thin : J->four_pi_phi_c) * (u * u)) {
            A->splits++;
            for (int k = 3; k >= 1; --k)
              stack[sp++] = (oray){R.level + 1, 4 * R.pix + (uint64_t)k, R.r, 0.25 * R.P, 0.25 * R.P0, R.rh, R.age,
                                   R.tau, R.thin};
            R = (oray){R.level + 1, 4 * R.pix, R.r, 0.25 * R.P, 0.25 * R.P0, R.rh, R.age, R.tau, R.thin};
            goto new_ray;
          }
        }
        /* a ray that reaches its halting radius inside this cell stops there */
        const int halt = t_exit > R.rh;
        const double t_end = halt ? R.rh : t_exit;
        const double dr = t_end - R.r;
        if (dr > 0.0 && thin) {
          /* a thin ray removes no photons (section 2.4) */
          const double tau = sigma * nabs * ((dr * h) * G->dx_cm);
          const size_t o = H->cell_off[q] + cell;
          int holds = 1;
          for (int a = 0; a < 3; ++a) holds = holds && (double)c[a] <= sl[a] && sl[a] <= (double)c[a] + 1.0;
          if (holds) {
            /* a cell that holds the source (on its boundary too): the
               general deposit, kept apart */
            const double dP = R.P * (-expm1(-tau));
            const double fc = J->par->covering ? covering_factor(sl, n, c, R.r, dr, h, R.level) : 1.0;
            A->thin_dep[o] += dP * fc;
            A->thin_energy[o] += dP * fc * eexc;
          } else if (!A->mark[o] && dr > ldexp(t_exit, -40)) {
            /* Eq. optthin: the ray's flux P / (Omega_ray r^2) taken at the
               cell centre, once per cell for this (source, group) */
            double r2 = 0.0;
            for (int a = 0; a < 3; ++a) {
              const double centre = (q == 0) ? (double)c[a] + 0.5 : (double)G->offset[a] + 0.5 * ((double)c[a] + 0.5);
              const double d = (centre - s[a]) * H->g[0].dx_cm;
              r2 += d * d;
            }
            const double omega = 4.0 * PI_D / ldexp(12.0, 2 * R.level);
            const double k = sigma * R.P / (omega * r2);
            A->mark[o] = 1;
            A->thin_marked++;
            A->k_thin[o] += k;
            A->h_thin[o] += k * eexc;
          }
          R.tau += tau;
          A->thin_segments++;
          A->segments++;
          R.r = t_end;
        } else if (dr > 0.0) {
          R.thin = 0;
          const double tau = sigma * nabs * ((dr * h) * G->dx_cm);
          const double dP = R.P * (-expm1(-tau));
          const double fc = J->par->covering ? covering_factor(sl, n, c, R.r, dr, h, R.level) : 1.0;
          A->absorbed[H->cell_off[q] + cell] += dP * fc;
          A->energy[H->cell_off[q] + cell] += dP * fc * eexc;
          if (A->mom) {
            /* radiation pressure (section 2.5.4, Eq. radpres): the absorbed
               photons' momentum dP E_ph / c along the ray; the covering
               factor scales only k_ph and heating, not the absorption */
            const double m = dP * (J->spec->energy_ev[gi] * EV_ERG) / C_CMS;
            const size_t o = H->cell_off[q] + cell;
            A->mom[o] += m * n[0];
            A->mom[H->n_cells + o] += m * n[1];
            A->mom[2 * H->n_cells + o] += m * n[2];
          }
          R.P -= dP;
          A->segments++;
          R.r = t_end;
        }
        if (halt) {
          if (hl->n < hl->cap)
            hl->ray[hl->n] = (orc_tray){si, gi, R.level, R.age, R.pix, R.r, R.P, R.P0};
          else
            hl->overflow = 1;
          hl->n++;
          cs_add(&hl->held, R.P);
          break;
        }
        const int dir = (n[ax] > 0.0) ? 1 : -1;
        c[ax] += dir;
        if (R.P < J->par->p_min_frac * R.P0) {
          cs_add(trunc, R.P);
          A->n_truncated++;
          break;
        }
        if (q == 0) {
          if (!in_grid(G, c)) {
            cs_add(esc, R.P);
            A->n_escaped++;
            break;
          }
          const int ch = H->cover[c[0] + (long)G->nx * (c[1] + (long)G->ny * c[2])];
          if (ch >= 0) {
            long rc[3] = {c[0], c[1], c[2]};
            enter_child(H, ch, rc, ax, dir, s, n, R.r, c);
            q = ch;
          }
        } else if (!in_grid(G, c)) {
          long rc[3];
          for (int a = 0; a < 3; ++a) rc[a] = (long)G->offset[a] + floor_half(c[a]);
          const orc_grid* Rg = &H->g[0];
          if (!in_grid(Rg, rc)) {
            cs_add(esc, R.P);
            A->n_escaped++;
            break;
          }
          const int ch = H->cover[rc[0] + (long)Rg->nx * (rc[1] + (long)Rg->ny * rc[2])];
          if (ch >= 0) {
            enter_child(H, ch, rc, ax, dir, s, n, R.r, c);
            q = ch;
          } else {
            q = 0;
            c[0] = rc[0]; c[1] = rc[1]; c[2] = rc[2];
          }
        }
      }
    }
  }
}


/* Trace all seed rays of one (source, group) item (single pass). */
static void trace_item(const job* J, int si, int gi, acc* A, csum* esc, csum* trunc) {
  const orc_source* S = &J->src[si];
  const int l0 = J->par->level_init;
  const uint64_t npix0 = (uint64_t)12 << (2 * l0);
  const double P0 = J->spec->frac[gi] * S->ndot / (double)npix0;
  const int thin = J->par->tau_thin > 0.0;
  if (thin) memset(A->mark, 0, J->H->n_cells);     /* marks are per (source, group) */
  halted none = {NULL, 0, 0, 0, {0.0, 0.0}};
  for (uint64_t p0 = 0; p0 < npix0; ++p0) {
    A->seeded++;
    march(J, si, gi, (oray){l0, p0, 0.0, P0, P0, INFINITY, 0, 0.0, thin}, A, esc, trunc, &none);
  }
}

static int finite_nonneg(double x) { return isfinite(x) && x >= 0.0; }

static int validate(const orc_grid* g, int ng, const orc_source* src, int ns, const orc_spectrum* sp,
                    const orc_params* p) {
  if (!g || ng < 1 || !sp || !p || ns < 0 || (ns > 0 && !src)) return -1;
  if (g[0].parent != -1) return -1;
  for (int q = 0; q < ng; ++q) {
    const orc_grid* G = &g[q];
    if (G->nx < 1 || G->ny < 1 || G->nz < 1 || !(G->dx_cm > 0.0) || !isfinite(G->dx_cm)) return -1;
    if (!G->n_h || !G->x_hi) return -1;
    const size_t nc = (size_t)G->nx * G->ny * G->nz;
    for (size_t i = 0; i < nc; ++i) {
      if (!finite_nonneg(G->n_h[i]) || !finite_nonneg(G->x_hi[i]) || G->x_hi[i] > 1.0f) return -1;
    }
    if (q > 0) {
      if (G->parent != 0 || (G->nx & 1) || (G->ny & 1) || (G->nz & 1)) return -1;
      if (G->dx_cm != 0.5 * g[0].dx_cm) return -1;
      if (G->offset[0] < 0 || G->offset[1] < 0 || G->offset[2] < 0) return -1;
      if (G->offset[0] + G->nx / 2 > g[0].nx || G->offset[1] + G->ny / 2 > g[0].ny ||
          G->offset[2] + G->nz / 2 > g[0].nz)
        return -1;
    }
  }
  for (int i = 0; i < ns; ++i) {
    const orc_source* S = &src[i];
    if (!(S->x >= 0.0 && S->x < g[0].nx && S->y >= 0.0 && S->y < g[0].ny && S->z >= 0.0 && S->z < g[0].nz))
      return -1;
    if (!(S->ndot > 0.0) || !isfinite(S->ndot)) return -1;
  }
  if (sp->n_groups < 1 || !sp->energy_ev || !sp->sigma_cm2 || !sp->frac) return -1;
  double fsum = 0.0;
  for (int k = 0; k < sp->n_groups; ++k) {
    if (!finite_nonneg(sp->sigma_cm2[k]) || !finite_nonneg(sp->frac[k])) return -1;
    if (!(sp->energy_ev[k] >= sp->e_ion_ev) || !isfinite(sp->energy_ev[k])) return -1;
    fsum += sp->frac[k];
  }
  if (fabs(fsum - 1.0) > 1e-12) return -1;
  if (!finite_nonneg(p->phi_c) || p->level_init < 0 || p->level_init > p->level_max ||
      p->level_max > MAX_LEVEL || !(p->p_min_frac >= 0.0 && p->p_min_frac < 1.0) || !finite_nonneg(p->tau_thin))
    return -1;
  return 0;
}

int orc_trace(const orc_grid* grids, int n_grids, const orc_source* src, int n_src, const orc_spectrum* spec,
              const orc_params* par, int n_threads, double* absorbed, double* energy, double* k_ph,
              double* heating, double* escaped_sg, orc_totals* tot) {
  return orc_trace_accel(grids, n_grids, src, n_src, spec, par, n_threads, absorbed, energy, k_ph, heating,
                         escaped_sg, NULL, tot);
}

/* One trace of a problem. Single pass: in == NULL, emit = 1, cdt infinite.
   Time-dependent step (one thread): the rays in[0..n_in) continue one step
   older, the sources emit new seed rays when emit is set, every ray halts at
   (age + 1) * cdt root cells from its source, and the halted rays go to
   out[0..out_cap) (their count to *n_out, their photon rate to *held). */
static int run_trace(const orc_grid* grids, int n_grids, const orc_source* src, int n_src,
                     const orc_spectrum* spec, const orc_params* par, int n_threads, double* absorbed,
                     double* energy, double* k_ph, double* heating, double* escaped_sg, double* accel,
                     orc_totals* tot, const orc_tray* in, size_t n_in, int emit, double cdt, orc_tray* out,
                     size_t out_cap, size_t* n_out, double* held) {
  if (validate(grids, n_grids, src, n_src, spec, par) != 0) return -1;
  if (!absorbed || !energy || !k_ph || !heating || !tot) return -1;
  const int td = in != NULL || out != NULL;
  if (td && (!(cdt > 0.0) || (n_in > 0 && !in) || !n_out || !held)) return -1;
  const int thin = par->tau_thin > 0.0;
  if (thin && (td || accel)) return -1;   /* the thin approximation is a single-pass option */
  for (size_t i = 0; i < n_in; ++i)
    if (in[i].src < 0 || in[i].src >= n_src || in[i].grp < 0 || in[i].grp >= spec->n_groups || in[i].level < 0 ||
        in[i].level > par->level_max || in[i].age < 0)
      return -1;
  hier H;
  H.g = grids;
  H.n_grids = n_grids;
  H.cell_off = (size_t*)malloc(sizeof(size_t) * (size_t)(n_grids + 1));
  H.cell_off[0] = 0;
  for (int q = 0; q < n_grids; ++q)
    H.cell_off[q + 1] = H.cell_off[q] + (size_t)grids[q].nx * grids[q].ny * grids[q].nz;
  H.n_cells = H.cell_off[n_grids];
  const orc_grid* R = &grids[0];
  const size_t nroot = (size_t)R->nx * R->ny * R->nz;
  H.cover = (int*)malloc(sizeof(int) * nroot);
  for (size_t i = 0; i < nroot; ++i) H.cover[i] = -1;
  for (int q = 1; q < n_grids; ++q) {
    const orc_grid* G = &grids[q];
    for (int k = 0; k < G->nz / 2; ++k)
      for (int j = 0; j < G->ny / 2; ++j)
        for (int i = 0; i < G->nx / 2; ++i) {
          const size_t rc = (size_t)(G->offset[0] + i) +
                            (size_t)R->nx * ((size_t)(G->offset[1] + j) + (size_t)R->ny * (size_t)(G->offset[2] + k));
          if (H.cover[rc] >= 0) { free(H.cover); free(H.cell_off); return -1; }   /* overlapping children */
          H.cover[rc] = q;
        }
  }

  job J = {&H, src, spec, par, 4.0 * PI_D * par->phi_c, 4.0 * PI_D * (par->phi_c < 1.0 ? par->phi_c : 1.0)};
  const int n_items = n_src * spec->n_groups;
  int T = n_threads < 1 || td ? 1 : n_threads;
  if (T > n_items && n_items > 0) T = n_items;
  acc* A = (acc*)calloc((size_t)T, sizeof(acc));
  for (int t = 0; t < T; ++t) {
    A[t].absorbed = (double*)calloc(H.n_cells, sizeof(double));
    A[t].energy = (double*)calloc(H.n_cells, sizeof(double));
    A[t].mom = accel ? (double*)calloc(3 * H.n_cells, sizeof(double)) : NULL;
    A[t].thin_margin = INFINITY;
    if (thin) {
      A[t].k_thin = (double*)calloc(H.n_cells, sizeof(double));
      A[t].h_thin = (double*)calloc(H.n_cells, sizeof(double));
      A[t].thin_dep = (double*)calloc(H.n_cells, sizeof(double));
      A[t].thin_energy = (double*)calloc(H.n_cells, sizeof(double));
      A[t].mark = (unsigned char*)calloc(H.n_cells, 1);
    }
  }
  csum* esc = (csum*)calloc((size_t)(n_items > 0 ? n_items : 1), sizeof(csum));
  csum* trn = (csum*)calloc((size_t)(n_items > 0 ? n_items : 1), sizeof(csum));

  halted hl = {out, out_cap, 0, 0, {0.0, 0.0}};
  if (!td) {
#ifdef _OPENMP
#pragma omp parallel num_threads(T)
    {
      const int t = omp_get_thread_num();
#else
    for (int t = 0; t < T; ++t) {
#endif
      for (int it = t; it < n_items; it += T)
        trace_item(&J, it / spec->n_groups, it % spec->n_groups, &A[t], &esc[it], &trn[it]);
    }
  } else {
    /* the rays in flight first, in their order, then the new seeds */
    for (size_t i = 0; i < n_in; ++i) {
      const orc_tray* T0 = &in[i];
      const int age = T0->age + 1;
      march(&J, T0->src, T0->grp, (oray){T0->level, T0->pix, T0->r, T0->P, T0->P0, (double)(age + 1) * cdt, age, 0.0, 0},
            &A[0], &esc[T0->src * spec->n_groups + T0->grp], &trn[T0->src * spec->n_groups + T0->grp], &hl);
    }
    if (emit) {
      const int l0 = par->level_init;
      const uint64_t npix0 = (uint64_t)12 << (2 * l0);
      for (int it = 0; it < n_items; ++it) {
        const int si = it / spec->n_groups, gi = it % spec->n_groups;
        const double P0 = spec->frac[gi] * src[si].ndot / (double)npix0;
        for (uint64_t p0 = 0; p0 < npix0; ++p0) {
          A[0].seeded++;
          march(&J, si, gi, (oray){l0, p0, 0.0, P0, P0, cdt, 0, 0.0, 0}, &A[0], &esc[it], &trn[it], &hl);
        }
      }
    }
    *n_out = hl.n;
    *held = cs_get(&hl.held);
  }

  memset(tot, 0, sizeof(*tot));
  csum cem = {0, 0}, cab = {0, 0}, ces = {0, 0}, ctr = {0, 0};
  if (emit)
    for (int i = 0; i < n_src; ++i)
      for (int k = 0; k < spec->n_groups; ++k) cs_add(&cem, spec->frac[k] * src[i].ndot);
  for (int it = 0; it < n_items; ++it) {
    cs_add(&ces, cs_get(&esc[it]));
    cs_add(&ctr, cs_get(&trn[it]));
    if (escaped_sg) escaped_sg[it] = cs_get(&esc[it]);
  }
  for (size_t i = 0; i < H.n_cells; ++i) {
    double a = 0.0, e = 0.0;
    for (int t = 0; t < T; ++t) { a += A[t].absorbed[i]; e += A[t].energy[i]; }
    absorbed[i] = a;
    energy[i] = e;
    cs_add(&cab, a);
  }
  tot->thin_margin = INFINITY;
  for (int t = 0; t < T; ++t) {
    tot->segments += A[t].segments;
    tot->splits += A[t].splits;
    tot->rays_seeded += A[t].seeded;
    tot->rays_escaped += A[t].n_escaped;
    tot->rays_truncated += A[t].n_truncated;
    tot->thin_segments += A[t].thin_segments;
    tot->thin_marked += A[t].thin_marked;
    if (A[t].thin_margin < tot->thin_margin) tot->thin_margin = A[t].thin_margin;
  }
  tot->emitted = cs_get(&cem);
  tot->absorbed = cs_get(&cab);
  tot->escaped = cs_get(&ces);
  tot->truncated = cs_get(&ctr);

  /* k_ph and heating per absorber (Eqs. kph, gamma with dt_P cancelled) */
  for (int q = 0; q < n_grids; ++q) {
    const orc_grid* G = &grids[q];
    const double vol = G->dx_cm * G->dx_cm * G->dx_cm;
    const size_t nc = (size_t)G->nx * G->ny * G->nz;
    for (size_t i = 0; i < nc; ++i) {
      const double nabs = (double)G->n_h[i] * (double)G->x_hi[i];
      const size_t o = H.cell_off[q] + i;
      double a = absorbed[o], e = energy[o], kt = 0.0, ht = 0.0;
      if (thin)
        for (int t = 0; t < T; ++t) {
          a += A[t].thin_dep[o];
          e += A[t].thin_energy[o];
          kt += A[t].k_thin[o];
          ht += A[t].h_thin[o];
        }
      if (nabs > 0.0) {
        k_ph[o] = a / (nabs * vol) + kt;
        heating[o] = e / (nabs * vol) + ht;
      } else {
        k_ph[o] = kt;
        heating[o] = ht;
      }
    }
  }
  for (int t = 0; t < T; ++t) {
    free(A[t].absorbed);
    free(A[t].energy);
    free(A[t].k_thin);
    free(A[t].h_thin);
    free(A[t].thin_dep);
    free(A[t].thin_energy);
    free(A[t].mark);
  }
  /* radiation-pressure acceleration a = dp / (rho V) with rho = m_H n_H
     (section 2.5.4; dt_P cancels as P is a rate) */
  if (accel) {
    for (int q = 0; q < n_grids; ++q) {
      const orc_grid* G = &grids[q];
      const double vol = G->dx_cm * G->dx_cm * G->dx_cm;
      const size_t nc = (size_t)G->nx * G->ny * G->nz;
      for (size_t i = 0; i < nc; ++i) {
        const size_t o = H.cell_off[q] + i;
        const double rho = M_H_G * (double)G->n_h[i];
        for (int k = 0; k < 3; ++k) {
          double m = 0.0;
          for (int t = 0; t < T; ++t) m += A[t].mom[k * H.n_cells + o];
          accel[k * H.n_cells + o] = rho > 0.0 ? m / (rho * vol) : 0.0;
        }
      }
    }
    for (int t = 0; t < T; ++t) free(A[t].mom);
  }
  free(A);
  free(esc);
  free(trn);
  free(H.cover);
  free(H.cell_off);
  return hl.overflow ? -2 : 0;
}

int orc_trace_accel(const orc_grid* grids, int n_grids, const orc_source* src, int n_src, const orc_spectrum* spec,
                    const orc_params* par, int n_threads, double* absorbed, double* energy, double* k_ph,
                    double* heating, double* escaped_sg, double* accel, orc_totals* tot) {
  return run_trace(grids, n_grids, src, n_src, spec, par, n_threads, absorbed, energy, k_ph, heating, escaped_sg,
                   accel, tot, NULL, 0, 1, INFINITY, NULL, 0, NULL, NULL);
}

int orc_trace_td(const orc_grid* grids, int n_grids, const orc_source* src, int n_src, const orc_spectrum* spec,
                 const orc_params* par, double c_dt, int emit, const orc_tray* in, size_t n_in, orc_tray* out,
                 size_t out_cap, size_t* n_out, double* held, double* absorbed, double* energy, double* k_ph,
                 double* heating, orc_totals* tot) {
  if (!out && out_cap > 0) return -1;
  orc_tray dummy;
  return run_trace(grids, n_grids, src, n_src, spec, par, 1, absorbed, energy, k_ph, heating, NULL, NULL, tot, in,
                   n_in, emit, c_dt, out ? out : &dummy, out ? out_cap : 0, n_out, held);
}
