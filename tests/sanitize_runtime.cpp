// Host-code check of the library (test infrastructure) under AddressSanitizer and
// UndefinedBehaviorSanitizer (built for the host only, run without a GPU by
// the test-suite): every entry point with a NULL context or bad arguments,
// context creation without a device, and the problem validation and
// queue-sizing routines on valid and invalid problems of every kind the
// validation knows. Exit status 0 when every check held.
#include "moray_internal.h"

#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

using namespace moray;

static int failures = 0;
#define CHECK(cond)                                                   \
  do {                                                                \
    if (!(cond)) {                                                    \
      std::printf("FAILED line %d: %s\n", __LINE__, #cond);          \
      ++failures;                                                     \
    }                                                                 \
  } while (0)

int main() {
  // entry points without a context
  CHECK(std::string(moray_version()).size() >= 5);
  CHECK(moray_last_error(nullptr) != nullptr);
  moray_ctx* ctx = nullptr;
  CHECK(moray_init(nullptr, nullptr) == MORAY_EINVAL);
  moray_init_params ip{};
  ip.precision = 7;
  CHECK(moray_init(&ctx, &ip) == MORAY_EINVAL && ctx == nullptr);
  ip.precision = MORAY_FP32_ACC64;
  ip.refill_lanes = 65;
  CHECK(moray_init(&ctx, &ip) == MORAY_EINVAL && ctx == nullptr);
  ip.refill_lanes = 0;
  int n_dev = 0;
  if (hipGetDeviceCount(&n_dev) != hipSuccess || n_dev == 0) {
    CHECK(moray_init(&ctx, &ip) == MORAY_EDEVICE && ctx == nullptr);
    CHECK(std::string(moray_last_error(nullptr)).find("GPU") != std::string::npos);
  }
  moray_result res{};
  moray_ticket t = 0;
  CHECK(moray_trace(nullptr, nullptr, 1, 0, &res) == MORAY_EINVAL);
  CHECK(moray_trace_noalloc(nullptr, nullptr, 1, 0, &res) == MORAY_EINVAL);
  CHECK(moray_trace_async(nullptr, nullptr, 1, 0, &res, &t) == MORAY_EINVAL);
  CHECK(moray_query(nullptr, 1, 0) == MORAY_EINVAL);
  CHECK(moray_cancel(nullptr, 1) == MORAY_EINVAL);
  CHECK(moray_set_deadline(nullptr, 1, 1.0) == MORAY_EINVAL);
  CHECK(moray_autotune(nullptr, nullptr, 1, 0, 0, nullptr) == MORAY_EINVAL);
  CHECK(moray_autotune_cached(nullptr, "x", nullptr, 1, 0, 0, nullptr, nullptr) == MORAY_EINVAL);
  CHECK(moray_td_create(nullptr, nullptr, 1.0, 4096, nullptr) == MORAY_EINVAL);
  moray_free(nullptr);

  // validation on a host-only context (no device is touched)
  moray_ctx c;
  std::vector<float> f(16 * 16 * 16, 0.5f), fc(8 * 8 * 8, 0.5f);
  const double e[2] = {13.6, 30.0}, s[2] = {6.3e-18, 6.0e-19}, fr[2] = {0.5, 0.5};
  moray_spectrum sp{2, e, s, fr, 13.6};
  moray_grid g[2];
  g[0] = moray_grid{16, 16, 16, 1e20, -1, {0, 0, 0}, f.data(), f.data()};
  g[1] = moray_grid{8, 8, 8, 5e19, 0, {4, 4, 4}, fc.data(), fc.data()};
  moray_source src[2] = {{3.25, 7.5, 11.0, 1e49}, {6.1, 6.2, 6.3, 1e48}};
  auto fresh = [&]() {
    moray_problem p{};
    p.grids = g;
    p.n_grids = 2;
    p.sources = src;
    p.n_sources = 2;
    p.spectrum = &sp;
    p.params = moray_trace_params{5.1, 1, 14, 1e-8, 0};
    return p;
  };
  moray_problem p = fresh();
  CHECK(validate(&c, p, 0) == MORAY_OK);
  CHECK(reach_level(p) >= 1 && reach_level(p) <= 14);
  CHECK(level_rays_bound(p) > 0.0);
  CHECK(queue_segments(1 << 10) == 1 && queue_segments((size_t)1 << 30) == kSegMax);
  // each invalid variant is rejected with a message
  struct Case {
    const char* what;
    void (*mutate)(moray_problem&, moray_grid*, moray_source*, moray_spectrum*);
  };
  static double e_low[2] = {13.6, 10.0}, fr_bad[2] = {0.5, 0.6}, nanv[2] = {NAN, 0.5};
  const Case cases[] = {
      {"no grids", [](moray_problem& q, moray_grid*, moray_source*, moray_spectrum*) { q.n_grids = 0; }},
      {"null spectrum", [](moray_problem& q, moray_grid*, moray_source*, moray_spectrum*) { q.spectrum = nullptr; }},
      {"root with a parent", [](moray_problem&, moray_grid* G, moray_source*, moray_spectrum*) { G[0].parent = 0; }},
      {"zero dimension", [](moray_problem&, moray_grid* G, moray_source*, moray_spectrum*) { G[0].ny = 0; }},
      {"nan dx", [](moray_problem&, moray_grid* G, moray_source*, moray_spectrum*) { G[0].dx_cm = NAN; }},
      {"odd child", [](moray_problem&, moray_grid* G, moray_source*, moray_spectrum*) { G[1].nx = 7; }},
      {"child dx", [](moray_problem&, moray_grid* G, moray_source*, moray_spectrum*) { G[1].dx_cm = 4e19; }},
      {"child outside", [](moray_problem&, moray_grid* G, moray_source*, moray_spectrum*) { G[1].offset[2] = 13; }},
      {"source outside", [](moray_problem&, moray_grid*, moray_source* S, moray_spectrum*) { S[0].x = 16.0; }},
      {"nan source", [](moray_problem&, moray_grid*, moray_source* S, moray_spectrum*) { S[1].y = NAN; }},
      {"zero rate", [](moray_problem&, moray_grid*, moray_source* S, moray_spectrum*) { S[1].ndot = 0.0; }},
      {"energy below E_ion", [](moray_problem&, moray_grid*, moray_source*, moray_spectrum* X) { X->energy_ev = e_low; }},
      {"fractions", [](moray_problem&, moray_grid*, moray_source*, moray_spectrum* X) { X->photon_frac = fr_bad; }},
      {"nan cross-section", [](moray_problem&, moray_grid*, moray_source*, moray_spectrum* X) { X->sigma_cm2 = nanv; }},
      {"negative phi_c", [](moray_problem& q, moray_grid*, moray_source*, moray_spectrum*) { q.params.phi_c = -1.0; }},
      {"levels", [](moray_problem& q, moray_grid*, moray_source*, moray_spectrum*) { q.params.level_init = 15; }},
      {"level_max", [](moray_problem& q, moray_grid*, moray_source*, moray_spectrum*) { q.params.level_max = 30; }},
      {"p_min", [](moray_problem& q, moray_grid*, moray_source*, moray_spectrum*) { q.params.p_min_frac = 1.0; }},
      {"tau_thin", [](moray_problem& q, moray_grid*, moray_source*, moray_spectrum*) { q.params.tau_thin = NAN; }},
      {"negative tau_thin", [](moray_problem& q, moray_grid*, moray_source*, moray_spectrum*) { q.params.tau_thin = -0.1; }},
  };
  for (const Case& k : cases) {
    moray_grid gg[2] = {g[0], g[1]};
    moray_source ss[2] = {src[0], src[1]};
    moray_spectrum xx = sp;
    moray_problem q = fresh();
    q.grids = gg;
    q.sources = ss;
    q.spectrum = &xx;
    k.mutate(q, gg, ss, &xx);
    const moray_status st = validate(&c, q, 3);
    std::printf("%-22s -> %d (%s)\n", k.what, (int)st, c.err.c_str());
    CHECK(st == MORAY_EINVAL && c.err.find("problem 3") == 0);
  }
  std::printf("%s\n", failures ? "SOME CHECK FAILED" : "ALL OK");
  return failures ? 1 : 0;
}
