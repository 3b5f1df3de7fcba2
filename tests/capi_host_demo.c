/* A caller of the C ABI with nothing but include/moray.h and libmoray.so:
 * host fields, host results, one batched one-shot solve of two problems.
 * Reads a little binary input (written by the test that builds this), traces
 * in both precisions and prints the totals and two k_ph checksums per problem.
 *
 * input layout (little endian): int32 n_probs; per problem: int32 nx, ny, nz,
 * n_sources, n_groups; float64 dx_cm, e_ion_ev, phi_c, p_min_frac;
 * int32 level_init, level_max; float32 n_h[nx*ny*nz], x_hi[nx*ny*nz];
 * float64 sources[n_sources*4]; float64 energy[n_groups], sigma[n_groups],
 * frac[n_groups]. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "moray.h"

#define MAXP 4

static void* read_all(FILE* f, size_t n) {
  void* p = malloc(n ? n : 1);
  if (fread(p, 1, n, f) != n) {
    fprintf(stderr, "short input\n");
    exit(2);
  }
  return p;
}

int main(int argc, char** argv) {
  if (argc < 2) return 2;
  FILE* f = fopen(argv[1], "rb");
  if (!f) return 2;
  int n = 0;
  if (fread(&n, 4, 1, f) != 1 || n < 1 || n > MAXP) return 2;
  moray_problem probs[MAXP];
  moray_grid grids[MAXP];
  moray_spectrum specs[MAXP];
  moray_result res[MAXP];
  long long cells[MAXP];
  memset(probs, 0, sizeof probs);
  memset(grids, 0, sizeof grids);
  for (int i = 0; i < n; ++i) {
    int hdr[5];
    double par[4];
    int lev[2];
    if (fread(hdr, 4, 5, f) != 5 || fread(par, 8, 4, f) != 4 || fread(lev, 4, 2, f) != 2) return 2;
    cells[i] = (long long)hdr[0] * hdr[1] * hdr[2];
    grids[i].nx = hdr[0]; grids[i].ny = hdr[1]; grids[i].nz = hdr[2];
    grids[i].dx_cm = par[0];
    grids[i].parent = -1;
    grids[i].n_h = (const float*)read_all(f, cells[i] * 4);
    grids[i].x_hi = (const float*)read_all(f, cells[i] * 4);
    moray_source* src = (moray_source*)read_all(f, (size_t)hdr[3] * 32);
    specs[i].n_groups = hdr[4];
    specs[i].energy_ev = (const double*)read_all(f, (size_t)hdr[4] * 8);
    specs[i].sigma_cm2 = (const double*)read_all(f, (size_t)hdr[4] * 8);
    specs[i].photon_frac = (const double*)read_all(f, (size_t)hdr[4] * 8);
    specs[i].e_ion_ev = par[1];
    probs[i].grids = &grids[i];
    probs[i].n_grids = 1;
    probs[i].sources = src;
    probs[i].n_sources = hdr[3];
    probs[i].spectrum = &specs[i];
    probs[i].params.phi_c = par[2];
    probs[i].params.p_min_frac = par[3];
    probs[i].params.level_init = lev[0];
    probs[i].params.level_max = lev[1];
  }
  fclose(f);
  for (int prec = 0; prec < 2; ++prec) {
    moray_init_params ip;
    memset(&ip, 0, sizeof ip);
    ip.precision = prec == 0 ? MORAY_FP64 : MORAY_FP32_ACC64;
    moray_ctx* ctx = NULL;
    moray_status st = moray_init(&ctx, &ip);
    if (st != MORAY_OK) {
      fprintf(stderr, "moray_init: %d %s\n", (int)st, moray_last_error(NULL));
      return 1;
    }
    for (int i = 0; i < n; ++i) {
      memset(&res[i], 0, sizeof res[i]);
      res[i].k_ph = (double*)malloc(cells[i] * 8);
      res[i].heating = (double*)malloc(cells[i] * 8);
    }
    st = moray_trace(ctx, probs, n, 0u, res);
    if (st != MORAY_OK) {
      fprintf(stderr, "moray_trace: %d %s\n", (int)st, moray_last_error(ctx));
      return 1;
    }
    for (int i = 0; i < n; ++i) {
      double s1 = 0.0, s2 = 0.0;
      for (long long c = 0; c < cells[i]; ++c) {
        s1 += res[i].k_ph[c];
        s2 += res[i].heating[c];
      }
      printf("precision %d problem %d segments %llu splits %llu emitted %.17g absorbed %.17g escaped %.17g "
             "truncated %.17g sum_kph %.17g sum_heat %.17g\n",
             ip.precision, i, res[i].segments, res[i].splits, res[i].emitted, res[i].absorbed, res[i].escaped,
             res[i].truncated, s1, s2);
      free(res[i].k_ph);
      free(res[i].heating);
    }
    moray_free(ctx);
  }
  printf("version %s\n", moray_version());
  return 0;
}
