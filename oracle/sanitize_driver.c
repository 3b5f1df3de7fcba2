/*
 * Driver of the oracle's sanitizer build (TEST INFRASTRUCTURE): compiled with
 * -fsanitize=address,undefined together with moray_oracle.c, it runs small
 * problems through every entry point -- a uniform box with a vertex source, a
 * pseudo-random medium with several sources, a 2x-refined child grid holding
 * a source, the covering factor, the optically-thin approximation, the
 * radiation-pressure acceleration, time-dependent steps (including an
 * out-list that is too small) and the
 * rejected inputs -- and checks photon conservation, so that an
 * out-of-bounds access, an overflow or undefined arithmetic anywhere on those
 * paths stops the run with a report. Exit status 0 when every case passed.
 */
#include "moray_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>

static unsigned long long rng_state = 0x9E3779B97F4A7C15ull;
static double urand(void) {     /* xorshift64*, uniform in [0, 1) */
  rng_state ^= rng_state >> 12;
  rng_state ^= rng_state << 25;
  rng_state ^= rng_state >> 27;
  return (double)((rng_state * 2685821657736338717ull) >> 11) * (1.0 / 9007199254740992.0);
}

static int conserved(const char* name, const orc_totals* t, double tol) {
  const double bal = t->absorbed + t->escaped + t->truncated - t->emitted;
  const int ok = fabs(bal) <= tol * t->emitted && t->rays_seeded + 4 * t->splits ==
                                                      t->splits + t->rays_escaped + t->rays_truncated;
  printf("%-28s segments %10llu splits %8llu conservation %+.2e %s\n", name, (unsigned long long)t->segments,
         (unsigned long long)t->splits, bal / t->emitted, ok ? "ok" : "FAILED");
  return ok;
}

int main(void) {
  int ok = 1;
  const double dx = 3.0856775814913673e18 * 15.625;
  const double e[2] = {13.6, 30.0}, sig[2] = {6.3e-18, 6.3e-18 * pow(30.0 / 13.6, -3.0)}, fr[2] = {0.5, 0.5};
  const orc_spectrum sp = {2, e, sig, fr, 13.6};
  orc_params par = {5.1, 1, 14, 1e-8, 0};
  enum { N = 12, NC = 8 };
  float nh[N * N * N], xh[N * N * N], cnh[NC * NC * NC], cxh[NC * NC * NC];
  for (int i = 0; i < N * N * N; ++i) {
    nh[i] = (float)(1e-2 * exp(2.0 * urand() - 1.0));
    xh[i] = (float)(0.5 + 0.5 * urand());
  }
  for (int i = 0; i < NC * NC * NC; ++i) {
    cnh[i] = (float)(3e-2 * urand());
    cxh[i] = (float)(0.5 + 0.5 * urand());
  }
  const size_t cells = N * N * N + NC * NC * NC;
  double* buf = (double*)calloc(7 * cells + 64, sizeof(double));
  double *ab = buf, *en = ab + cells, *kp = en + cells, *he = kp + cells, *acc = he + cells, *esc = acc + 3 * cells;
  orc_totals tot;

  /* uniform box, source on a cell vertex */
  float un[N * N * N], ux[N * N * N];
  for (int i = 0; i < N * N * N; ++i) { un[i] = 2e-3f; ux[i] = 1.0f; }
  orc_grid ug = {N, N, N, dx, un, ux, -1, {0, 0, 0}};
  orc_source vs = {6.0, 6.0, 6.0, 1e49};
  ok &= orc_trace(&ug, 1, &vs, 1, &sp, &par, 1, ab, en, kp, he, esc, &tot) == 0 && conserved("uniform, vertex source", &tot, 1e-12);

  /* pseudo-random medium, general source positions, two threads */
  orc_grid g[2] = {{N, N, N, dx, nh, xh, -1, {0, 0, 0}}, {NC, NC, NC, dx / 2, cnh, cxh, 0, {4, 3, 5}}};
  orc_source src[3] = {{urand() * N, urand() * N, urand() * N, 1e48},
                       {6.123456789, 5.5 + 1e-13, 7.0 - 1e-12, 3e49},
                       {urand() * N, urand() * N, urand() * N, 1e50}};
  ok &= orc_trace(g, 1, src, 3, &sp, &par, 2, ab, en, kp, he, esc, &tot) == 0 && conserved("lognormal-like, 3 sources", &tot, 1e-12);

  /* nested child grid holding a source, and the covering factor */
  src[1].x = 6.25; src[1].y = 5.75; src[1].z = 7.5;
  ok &= orc_trace(g, 2, src, 3, &sp, &par, 1, ab, en, kp, he, esc, &tot) == 0 && conserved("nested, source in child", &tot, 1e-12);
  par.covering = 1;
  ok &= orc_trace(g, 2, src, 3, &sp, &par, 1, ab, en, kp, he, esc, &tot) == 0;
  printf("%-28s segments %10llu\n", "covering factor", (unsigned long long)tot.segments);
  par.covering = 0;

  /* the optically-thin approximation, two threads; it is refused with
     radiation pressure and with time-dependent rays */
  par.tau_thin = 0.1;
  ok &= orc_trace(g, 2, src, 3, &sp, &par, 2, ab, en, kp, he, esc, &tot) == 0 && conserved("optically thin", &tot, 1e-12);
  printf("%-28s thin segments %10llu marked %8llu margin %.2e\n", "optically thin",
         (unsigned long long)tot.thin_segments, (unsigned long long)tot.thin_marked, tot.thin_margin);
  ok &= tot.thin_segments > 0 && tot.thin_marked > 0;
  ok &= orc_trace_accel(g, 2, src, 3, &sp, &par, 1, ab, en, kp, he, esc, acc, &tot) == -1;
  {
    size_t n0 = 0;
    double h0 = 0.0;
    orc_tray one;
    ok &= orc_trace_td(g, 2, src, 3, &sp, &par, 3.0, 1, NULL, 0, &one, 1, &n0, &h0, ab, en, kp, he, &tot) == -1;
  }
  par.tau_thin = 0.0;

  /* radiation pressure */
  ok &= orc_trace_accel(g, 2, src, 3, &sp, &par, 1, ab, en, kp, he, esc, acc, &tot) == 0 &&
        conserved("radiation pressure", &tot, 1e-12);

  /* time-dependent steps, then an out-list too small */
  size_t cap = 1 << 18, n_out = 0, n_in = 0;
  orc_tray* a = (orc_tray*)malloc(cap * sizeof(orc_tray));
  orc_tray* b = (orc_tray*)malloc(cap * sizeof(orc_tray));
  double held = 0.0, held_prev = 0.0;
  for (int step = 0; step < 4; ++step) {
    const int rc = orc_trace_td(g, 2, src, 3, &sp, &par, 3.0, 1, a, n_in, b, cap, &n_out, &held, ab, en, kp, he, &tot);
    const double bal = tot.emitted + held_prev - tot.absorbed - tot.escaped - tot.truncated - held;
    const int good = rc == 0 && fabs(bal) <= 1e-12 * (tot.emitted + held_prev);
    printf("%-28s step %d in flight %zu balance %+.2e %s\n", "time-dependent", step, n_out,
           bal / (tot.emitted + held_prev), good ? "ok" : "FAILED");
    ok &= good;
    orc_tray* t = a; a = b; b = t;
    n_in = n_out;
    held_prev = held;
  }
  ok &= orc_trace_td(g, 2, src, 3, &sp, &par, 3.0, 1, a, n_in, b, 16, &n_out, &held, ab, en, kp, he, &tot) == -2;

  /* rejected inputs write nothing */
  orc_source outside = {(double)N, 1.0, 1.0, 1e49};
  orc_params bad = {5.1, 15, 14, 1e-8, 0};
  ok &= orc_trace(g, 1, &outside, 1, &sp, &par, 1, ab, en, kp, he, esc, &tot) == -1;
  ok &= orc_trace(g, 1, src, 1, &sp, &bad, 1, ab, en, kp, he, esc, &tot) == -1;

  free(a);
  free(b);
  free(buf);
  printf("%s\n", ok ? "ALL OK" : "SOME CASE FAILED");
  return ok ? 0 : 1;
}
