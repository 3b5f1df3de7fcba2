// Persistent autotune cache: the launch settings moray_autotune picks for a
// batch, kept in a text file so that a later process with the same device,
// library version, precision and batch shape takes them without timing.
//
// One line per tuned batch, fields separated by single spaces:
//   moray-tune-1 <library version> <device arch> <compute units> <precision>
//   <deposit table on> <batch shape hash, 16 hex digits> <chunk_rays>
//   <refill_lanes> <reserve_rays> <waves_per_cu> <first_ms> <best_ms> <trials>
// The last valid line for a key wins; lines that do not parse, or whose
// settings are out of range for this device, are ignored.
#include <hip/hip_runtime.h>

#include <cerrno>
#include <cinttypes>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>

#include "moray.h"
#include "moray_device.h"
#include "moray_internal.h"

using namespace moray;

namespace {

struct Fnv {
  uint64_t h = 1469598103934665603ull;
  void add(uint64_t v) {
    for (int i = 0; i < 8; ++i) {
      h ^= (v >> (8 * i)) & 0xffu;
      h *= 1099511628211ull;
    }
  }
  void add_double(double d) {
    uint64_t u;
    std::memcpy(&u, &d, sizeof u);
    add(u);
  }
};

// Everything about a batch that shapes its launches: grid shapes and nesting,
// source and group counts, the trace parameters. Field values, source
// positions and photon rates are not part of it.
uint64_t batch_shape(const moray_problem* probs, int n) {
  Fnv f;
  f.add((uint64_t)n);
  for (int i = 0; i < n; ++i) {
    const moray_problem& P = probs[i];
    f.add((uint64_t)P.n_grids);
    for (int q = 0; q < P.n_grids; ++q) {
      const moray_grid& g = P.grids[q];
      f.add((uint64_t)(uint32_t)g.nx);
      f.add((uint64_t)(uint32_t)g.ny);
      f.add((uint64_t)(uint32_t)g.nz);
      f.add((uint64_t)(uint32_t)g.parent);
      for (int a = 0; a < 3; ++a) f.add((uint64_t)(uint32_t)g.offset[a]);
    }
    f.add((uint64_t)P.n_sources);
    f.add((uint64_t)P.spectrum->n_groups);
    f.add((uint64_t)(uint32_t)P.params.level_init);
    f.add((uint64_t)(uint32_t)P.params.level_max);
    f.add_double(P.params.phi_c);
    f.add_double(P.params.p_min_frac);
    f.add((uint64_t)(P.params.covering != 0));
  }
  return f.h;
}

std::string key_of(moray_ctx* c, const moray_problem* probs, int n, std::string* why) {
  hipDeviceProp_t prop;
  const hipError_t e = hipGetDeviceProperties(&prop, c->device);
  if (e != hipSuccess) {
    *why = std::string("hipGetDeviceProperties: ") + hipGetErrorString(e);
    return std::string();
  }
  std::string arch = prop.gcnArchName;
  for (char& ch : arch)
    if (ch == ' ' || ch == '\t' || ch == '\n') ch = '_';
  char sig[17];
  std::snprintf(sig, sizeof sig, "%016" PRIx64, batch_shape(probs, n));
  std::ostringstream k;
  k << "moray-tune-1 " << moray_version() << ' ' << arch << ' ' << prop.multiProcessorCount << ' ' << c->precision
    << ' ' << (c->cache ? 1 : 0) << ' ' << sig;
  return k.str();
}

struct Entry {
  int chunk = 0, refill = 0, reserve = 0, waves = 0, trials = 0;
  double first_ms = 0.0, best_ms = 0.0;
};

// The last line of `path` with this key whose settings are valid here.
bool lookup(const std::string& path, const std::string& key, int bpc_max, Entry* out) {
  std::ifstream in(path);
  if (!in) return false;
  bool found = false;
  std::string line;
  while (std::getline(in, line)) {
    if (line.size() <= key.size() + 1 || line.compare(0, key.size(), key) != 0 || line[key.size()] != ' ') continue;
    std::istringstream rest(line.substr(key.size() + 1));
    Entry e;
    std::string tail;
    if (!(rest >> e.chunk >> e.refill >> e.reserve >> e.waves >> e.first_ms >> e.best_ms >> e.trials) ||
        (rest >> tail))
      continue;
    const int per_block = kTraceBlock / kWave;
    if (e.chunk < 1 || e.chunk > (1 << 20) || e.refill < 1 || e.refill > kWave || e.reserve < 0 ||
        e.reserve > (1 << 20) || e.waves < per_block || e.waves % per_block != 0 || e.waves / per_block > bpc_max)
      continue;
    *out = e;
    found = true;
  }
  return found;
}

}  // namespace

extern "C" moray_status moray_autotune_cached(moray_ctx* c, const char* path, const moray_problem* probs, int n_probs,
                                              unsigned flags, int max_trials, moray_tune_result* out,
                                              int* from_cache) {
  if (!c) return MORAY_EINVAL;
  if (from_cache) *from_cache = 0;
  if (!path || !path[0]) return fail(c, MORAY_EINVAL, "cache path is NULL or empty");
  if (!probs || n_probs < 1) return fail(c, MORAY_EINVAL, "need n_probs >= 1 problems");
  if (flags & ~(MORAY_FIELDS_ON_DEVICE | MORAY_OUT_ON_DEVICE)) return fail(c, MORAY_EINVAL, "unknown flags");
  for (int i = 0; i < n_probs; ++i) {
    const moray_status s = validate(c, probs[i], i);
    if (s != MORAY_OK) return s;
  }
  if (engine_busy(c)) return fail(c, MORAY_EBUSY, "asynchronous solves are still running on this context");
  if (!hip_ok(c, hipSetDevice(c->device), "hipSetDevice")) return MORAY_EDEVICE;
  std::string why;
  const std::string key = key_of(c, probs, n_probs, &why);
  if (key.empty()) return fail(c, MORAY_EDEVICE, why);
  int bpc_max = 1;
  if (!hip_ok(c, trace_occupancy(c->precision, c->cache, &bpc_max), "occupancy query")) return MORAY_EDEVICE;
  Entry e;
  if (lookup(path, key, bpc_max, &e)) {
    c->chunk = e.chunk;
    c->refill = e.refill;
    c->reserve_user = e.reserve;
    c->blocks_per_cu = e.waves / (kTraceBlock / kWave);
    if (out) {
      out->chunk_rays = e.chunk;
      out->refill_lanes = e.refill;
      out->reserve_rays = e.reserve;
      out->waves_per_cu = e.waves;
      out->first_ms = e.first_ms;
      out->best_ms = e.best_ms;
      out->trials = e.trials;
    }
    if (from_cache) *from_cache = 1;
    c->err = "no error";
    return MORAY_OK;
  }
  // a miss: the file must take a line before any timing starts
  FILE* f = std::fopen(path, "a");
  if (!f) return fail(c, MORAY_EINVAL, std::string("cannot open the cache file for appending: ") + std::strerror(errno));
  moray_tune_result r{};
  const moray_status st = moray_autotune(c, probs, n_probs, flags, max_trials, &r);
  if (st != MORAY_OK) {
    std::fclose(f);
    return st;
  }
  if (out) *out = r;
  char line[1024];
  const int len = std::snprintf(line, sizeof line, "%s %d %d %d %d %.6f %.6f %d\n", key.c_str(), r.chunk_rays,
                                r.refill_lanes, r.reserve_rays, r.waves_per_cu, r.first_ms, r.best_ms, r.trials);
  // one write of a whole line, so concurrent appenders do not interleave
  const bool ok = len > 0 && len < (int)sizeof line && std::fwrite(line, 1, (size_t)len, f) == (size_t)len;
  const bool closed = std::fclose(f) == 0;
  if (!ok || !closed)
    return fail(c, MORAY_EINVAL, "tuned (the context keeps the new settings), but the cache file could not be written");
  c->err = "no error";
  return MORAY_OK;
}
