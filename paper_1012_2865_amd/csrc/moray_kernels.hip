// HIP kernels of the adaptive ray tracer (gfx950).
//
// One radiative-transfer pass (section 3.1, steps 1-3 of Wise & Abel) is the
// launch sequence
//   reset -> prep (absorber column per cell, input checks, zeroed accumulators)
//   -> trace_level(l) for l = l0 .. l_reach -> finalize,
// on one stream. A ray splits at most once per level: every launch consumes
// the rays of HEALPix level l (children written by the previous launch plus
// the seed rays of trees that start at level l) and writes the children of
// level l+1 into the other half of a ping-pong queue, so no launch ever waits
// on work produced inside itself.
//
// Inside trace_level the grid is persistent: every wave keeps 64 rays in
// flight, one per lane, marches them cell by cell (Eq. trace), tests the split
// criterion at each cell exit (Eq. split), deposits P (1 - e^-tau) with two
// float64 atomics per segment (Eqs. dtau, flux, kph, gamma), and refills idle
// lanes from a private chunk of the level queue claimed with one atomic.
// Children of splitting lanes are compacted with a wave ballot and written as
// four consecutive structure-of-arrays records per parent.
#include "moray_device.h"

#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdint>

namespace moray {

// ---------------------------------------------------------------------------
// HEALPix nested pixel centre (Gorski et al. 2005), float64.
// Face f, in-face coordinates (ix, iy) from the even/odd bits of the in-face
// index; ring j = jr(f) Ns - ix - iy - 1; polar caps z = 1 - nr^2/(3 Ns^2),
// equatorial belt z = 2(2 Ns - j)/(3 Ns); azimuth (pi/2)(jp - (s+1)/2)/nr.
// z and sin(theta) come from exact integers; the azimuth is reduced to the
// first octant before sin/cos so multiples of pi/4 are exact.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t compact_even_bits(uint64_t x) {
  x &= 0x5555555555555555ull;
  x = (x | (x >> 1)) & 0x3333333333333333ull;
  x = (x | (x >> 2)) & 0x0F0F0F0F0F0F0F0Full;
  x = (x | (x >> 4)) & 0x00FF00FF00FF00FFull;
  x = (x | (x >> 8)) & 0x0000FFFF0000FFFFull;
  x = (x | (x >> 16)) & 0x00000000FFFFFFFFull;
  return x;
}

__device__ void healpix_dir(int level, uint64_t pix, double& vx, double& vy, double& vz) {
  const int64_t ns = (int64_t)1 << level;
  const int face = (int)(pix >> (2 * level));
  const uint64_t ipf = pix & ((1ull << (2 * level)) - 1ull);
  const int64_t ix = (int64_t)compact_even_bits(ipf);
  const int64_t iy = (int64_t)compact_even_bits(ipf >> 1);
  const int row = face >> 2;                              // 0 north, 1 equator, 2 south
  const int64_t jr = (int64_t)(row + 2) * ns - ix - iy - 1;
  const int64_t jpf = 2 * (face & 3) + (row == 1 ? 0 : 1);
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
  int64_t jp = (jpf * nr + ix - iy + 1 + kshift) >> 1;   // the numerator is always even
  if (jp > 4 * nr) jp -= 4 * nr;
  if (jp < 1) jp += 4 * nr;
  const int64_t num = 2 * jp - kshift - 1, den = 2 * nr;
  const int64_t q = num / den, rem = num - q * den;
  double c, s;
  if (2 * rem == den) {
    c = s = sqrt(0.5);
  } else {
    const bool low = 2 * rem < den;
    const int64_t m = low ? rem : den - rem;
    const double beta = ((double)m / (double)den) * (M_PI / 2.0);
    double sb, cb;
    sincos(beta, &sb, &cb);
    c = low ? cb : sb;
    s = low ? sb : cb;
  }
  double cx, cy;
  switch (q & 3) {
    case 0: cx = c; cy = s; break;
    case 1: cx = -s; cy = c; break;
    case 2: cx = -c; cy = -s; break;
    default: cx = s; cy = -c; break;
  }
  vx = sth * cx;
  vy = sth * cy;
  vz = z;
}

// ---------------------------------------------------------------------------
// Precision-specific arithmetic. Float64 geometry mirrors the definition
// exactly (no contraction, true division); float32 geometry multiplies by a
// per-ray reciprocal.
// ---------------------------------------------------------------------------
template <typename R> struct Arith;

template <> struct Arith<double> {
  static __device__ __forceinline__ double mul(double a, double b) { return __dmul_rn(a, b); }
  static __device__ __forceinline__ double add(double a, double b) { return __dadd_rn(a, b); }
  static __device__ __forceinline__ double inv(double) { return 0.0; }
  // exit distance to plane b, root units: ((b - s) / d) * hinv
  static __device__ __forceinline__ double tplane(double b, double s, double d, double, double hinv) {
    return ((b - s) / d) * hinv;
  }
  static __device__ __forceinline__ double neg_expm1(double tau) { return -expm1(-tau); }
  static __device__ __forceinline__ double inf() { return __builtin_huge_val(); }
};

template <> struct Arith<float> {
  static __device__ __forceinline__ float mul(float a, float b) { return __fmul_rn(a, b); }
  static __device__ __forceinline__ float add(float a, float b) { return __fadd_rn(a, b); }
  static __device__ __forceinline__ float inv(float d) { return 1.0f / d; }
  static __device__ __forceinline__ float tplane(float b, float s, float, float id, float hinv) {
    return ((b - s) * id) * hinv;
  }
  static __device__ __forceinline__ double neg_expm1(float tau) { return (double)(-expm1f(-tau)); }
  static __device__ __forceinline__ float inf() { return __builtin_huge_valf(); }
};

__device__ __forceinline__ int cell_rule_d(double x, double d) {
  return d >= 0.0 ? (int)floor(x) : (int)ceil(x) - 1;
}
__device__ __forceinline__ int cell_rule_f(float x, float d) {
  return d >= 0.0f ? (int)floorf(x) : (int)ceilf(x) - 1;
}
template <typename R> __device__ __forceinline__ int cell_rule(R x, R d);
template <> __device__ __forceinline__ int cell_rule<double>(double x, double d) { return cell_rule_d(x, d); }
template <> __device__ __forceinline__ int cell_rule<float>(float x, float d) { return cell_rule_f(x, d); }

template <typename R> __device__ __forceinline__ R rmin(R a, R b) { return b < a ? b : a; }

__device__ __forceinline__ int floor_half(int c) { return c >= 0 ? c / 2 : -((-c + 1) / 2); }

// Per-lane ray state.
template <typename R>
struct Ray {
  uint64_t pix;
  uint32_t sg;
  int level_max;
  double P, pmin, eexc;
  R sigma;
  R r;                    // radius (root cells)
  R split_t2;             // split when (t_exit in local cells)^2 > split_t2 (float path)
  R eps_u;                // float path: bound on the source-position error in local cells / |d|
  double four_pi_phi_c;
  // direction and its reciprocal
  R d0, d1, d2, i0, i1, i2;
  // grid frame
  int q;                  // grid index
  int c0, c1, c2;         // local cell
  int n0, n1, n2;         // grid dims
  int lin;                // batch-wide cell index
  R s0, s1, s2;           // source in local cells
  R hinv, hloc;           // 1/scale, scale (1 root, 2 child)
  R t0, t1, t2;           // distance to the next plane per axis (root cells)
  R kap;                  // absorber column per root-cell length of the current cell
  unsigned segs;
};

template <typename R>
struct Tracer {
  const TraceArgs<R>& a;
  __device__ explicit Tracer(const TraceArgs<R>& args) : a(args) {}

  // Load grid q's frame and the exit distances from local cell (c0, c1, c2).
  __device__ void set_frame(Ray<R>& L, int q) const {
    const GridDev& G = a.grids[q];
    const SgDev& S = a.sgs[L.sg];
    L.q = q;
    L.n0 = G.nx; L.n1 = G.ny; L.n2 = G.nz;
    if (G.is_child) {
      L.hinv = (R)0.5; L.hloc = (R)2;
      L.s0 = (R)(2.0 * (S.sx - (double)G.ox));
      L.s1 = (R)(2.0 * (S.sy - (double)G.oy));
      L.s2 = (R)(2.0 * (S.sz - (double)G.oz));
    } else {
      L.hinv = (R)1; L.hloc = (R)1;
      L.s0 = (R)S.sx; L.s1 = (R)S.sy; L.s2 = (R)S.sz;
    }
    const R inf = Arith<R>::inf();
    L.t0 = L.d0 == (R)0 ? inf : Arith<R>::tplane((R)(L.c0 + (L.d0 > (R)0)), L.s0, L.d0, L.i0, L.hinv);
    L.t1 = L.d1 == (R)0 ? inf : Arith<R>::tplane((R)(L.c1 + (L.d1 > (R)0)), L.s1, L.d1, L.i1, L.hinv);
    L.t2 = L.d2 == (R)0 ? inf : Arith<R>::tplane((R)(L.c2 + (L.d2 > (R)0)), L.s2, L.d2, L.i2, L.hinv);
    L.lin = (int)G.cell_off + L.c0 + G.nx * (L.c1 + G.ny * L.c2);
  }

  // Enter child grid `ch` from root cell (rc0, rc1, rc2) across axis `ax`
  // moving in direction `dir`, at the current radius.
  __device__ void enter_child(Ray<R>& L, int ch, int rc0, int rc1, int rc2, int ax, int dir) const {
    const GridDev& G = a.grids[ch];
    const SgDev& S = a.sgs[L.sg];
    const int rc[3] = {rc0, rc1, rc2};
    const int o[3] = {G.ox, G.oy, G.oz};
    const R sr[3] = {(R)S.sx, (R)S.sy, (R)S.sz};
    const R d[3] = {L.d0, L.d1, L.d2};
    int c[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int lo = 2 * (rc[k] - o[k]);
      if (k == ax) {
        c[k] = lo + (dir < 0 ? 1 : 0);
      } else {
        const R x = Arith<R>::add(sr[k], Arith<R>::mul(L.r, d[k]));
        int cl = cell_rule<R>((R)2 * (x - (R)o[k]), d[k]);
        cl = cl < lo ? lo : (cl > lo + 1 ? lo + 1 : cl);
        c[k] = cl;
      }
    }
    L.c0 = c[0]; L.c1 = c[1]; L.c2 = c[2];
    set_frame(L, ch);
  }

  // After a step along `ax` by `dir`: resolve leaving the current grid and
  // entering a covered root cell. Returns false when the ray left the root.
  __device__ bool settle(Ray<R>& L, int ax, int dir) const {
    const GridDev& G = a.grids[L.q];
    if (!G.is_child) {
      if ((unsigned)L.c0 >= (unsigned)L.n0 || (unsigned)L.c1 >= (unsigned)L.n1 || (unsigned)L.c2 >= (unsigned)L.n2)
        return false;
      const R k = a.kappa[L.lin];
      if (k < (R)0) {
        enter_child(L, (int)(-k) - 1, L.c0, L.c1, L.c2, ax, dir);
        L.kap = a.kappa[L.lin];
      } else {
        L.kap = k;
      }
      return true;
    }
    if ((unsigned)L.c0 < (unsigned)L.n0 && (unsigned)L.c1 < (unsigned)L.n1 && (unsigned)L.c2 < (unsigned)L.n2) {
      L.kap = a.kappa[L.lin];
      return true;
    }
    // leave the child for the root cell beyond its face
    const int rc0 = G.ox + floor_half(L.c0), rc1 = G.oy + floor_half(L.c1), rc2 = G.oz + floor_half(L.c2);
    const int root = a.probs[G.problem].root_grid;
    const GridDev& Rg = a.grids[root];
    if ((unsigned)rc0 >= (unsigned)Rg.nx || (unsigned)rc1 >= (unsigned)Rg.ny || (unsigned)rc2 >= (unsigned)Rg.nz)
      return false;
    const int rlin = (int)Rg.cell_off + rc0 + Rg.nx * (rc1 + Rg.ny * rc2);
    const R k = a.kappa[rlin];
    if (k < (R)0) {
      enter_child(L, (int)(-k) - 1, rc0, rc1, rc2, ax, dir);
      L.kap = a.kappa[L.lin];
    } else {
      L.c0 = rc0; L.c1 = rc1; L.c2 = rc2;
      set_frame(L, root);
      L.kap = k;
    }
    return true;
  }

  // Start ray `idx` of this level: from the queue or synthesised as a seed.
  // Returns false when it starts outside the root grid (escaped at once).
  __device__ bool start(Ray<R>& L, unsigned long long idx, unsigned long long n_children) const {
    const int level = a.level;
    if (idx < n_children) {
      L.pix = a.in.pix[idx];
      L.sg = a.in.sg[idx];
      L.r = a.in.r[idx];
      L.P = a.in.P[idx];
    } else {
      const unsigned long long j = idx - n_children;
      const unsigned long long npix = 12ull << (2 * level);
      L.sg = (uint32_t)(a.seed_sg_begin + j / npix);
      L.pix = j % npix;
      L.r = (R)0;
      L.P = a.sgs[L.sg].P0;
    }
    const SgDev& S = a.sgs[L.sg];
    const ProblemDev& Pb = a.probs[S.problem];
    const int dl = level - S.level_init;
    L.pmin = ldexp(S.pmin0, -2 * dl);
    L.eexc = S.eexc_erg;
    L.level_max = Pb.level_max;
    L.four_pi_phi_c = Pb.four_pi_phi_c;
    L.segs = 0;
    if constexpr (sizeof(R) == 4) {
      L.sigma = S.sigma32;
      L.split_t2 = ldexpf(Pb.split_t2_base, 2 * level);
    } else {
      L.sigma = S.sigma64;
      L.split_t2 = 0.0;
    }
    double v0, v1, v2;
    healpix_dir(level, L.pix, v0, v1, v2);
    L.d0 = (R)v0; L.d1 = (R)v1; L.d2 = (R)v2;
    L.i0 = Arith<R>::inv(L.d0); L.i1 = Arith<R>::inv(L.d1); L.i2 = Arith<R>::inv(L.d2);
    if constexpr (sizeof(R) == 4) {
      const float im = fmaxf(fabsf(L.i0), fmaxf(fabsf(L.i1), fabsf(L.i2)));
      L.eps_u = S.src_err * 2.0f * im;   // child frames double the source error
    } else {
      L.eps_u = 0.0;
    }
    // locate the leaf cell holding s + r d
    const int root = Pb.root_grid;
    const GridDev& Rg = a.grids[root];
    const R x0 = Arith<R>::add((R)S.sx, Arith<R>::mul(L.r, L.d0));
    const R x1 = Arith<R>::add((R)S.sy, Arith<R>::mul(L.r, L.d1));
    const R x2 = Arith<R>::add((R)S.sz, Arith<R>::mul(L.r, L.d2));
    const int rc0 = cell_rule<R>(x0, L.d0), rc1 = cell_rule<R>(x1, L.d1), rc2 = cell_rule<R>(x2, L.d2);
    if ((unsigned)rc0 >= (unsigned)Rg.nx || (unsigned)rc1 >= (unsigned)Rg.ny || (unsigned)rc2 >= (unsigned)Rg.nz)
      return false;
    const int rlin = (int)Rg.cell_off + rc0 + Rg.nx * (rc1 + Rg.ny * rc2);
    const R k = a.kappa[rlin];
    if (k < (R)0) {
      const int ch = (int)(-k) - 1;
      const GridDev& G = a.grids[ch];
      // the fine cell lies under root cell rc (exact in floating point; kept in range regardless)
      const int f0 = 2 * (rc0 - G.ox), f1 = 2 * (rc1 - G.oy), f2 = 2 * (rc2 - G.oz);
      L.c0 = min(max(cell_rule<R>((R)2 * (x0 - (R)G.ox), L.d0), f0), f0 + 1);
      L.c1 = min(max(cell_rule<R>((R)2 * (x1 - (R)G.oy), L.d1), f1), f1 + 1);
      L.c2 = min(max(cell_rule<R>((R)2 * (x2 - (R)G.oz), L.d2), f2), f2 + 1);
      set_frame(L, ch);
      L.kap = a.kappa[L.lin];
    } else {
      L.c0 = rc0; L.c1 = rc1; L.c2 = rc2;
      set_frame(L, root);
      L.kap = k;
    }
    return true;
  }

  // Float64 re-evaluation of the split test for the current cell, in the
  // canonical form 12 * 4^l < (4 pi phi_c) * u^2, u = t_exit in local cells.
  __device__ bool split_exact(const Ray<R>& L) const {
    const SgDev& S = a.sgs[L.sg];
    const GridDev& G = a.grids[L.q];
    double v[3];
    healpix_dir(a.level, L.pix, v[0], v[1], v[2]);
    const double h = G.is_child ? 2.0 : 1.0;
    const double s[3] = {S.sx, S.sy, S.sz};
    const int o[3] = {G.ox, G.oy, G.oz};
    const int c[3] = {L.c0, L.c1, L.c2};
    double te = __builtin_huge_val();
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (v[k] == 0.0) continue;
      const double sl = G.is_child ? h * (s[k] - (double)o[k]) : s[k];
      const double b = (double)(c[k] + (v[k] > 0.0 ? 1 : 0));
      const double t = ((b - sl) / v[k]) / h;
      te = t < te ? t : te;
    }
    const double u = te * h;
    return ldexp(12.0, 2 * a.level) < L.four_pi_phi_c * (u * u);
  }
};

template <typename R>
__device__ __forceinline__ void flush_end(const TraceArgs<R>& a, const Ray<R>& L, int kind) {
  SgStats& st = a.stats[L.sg];
  if (L.segs) atomicAdd(&st.segs, (unsigned long long)L.segs);
  if (kind == 0) {                       // escaped
    unsafeAtomicAdd(&st.esc_P, L.P);
    atomicAdd(&st.n_esc, 1ull);
  } else if (kind == 1) {                // truncated
    unsafeAtomicAdd(&st.trunc_P, L.P);
    atomicAdd(&st.n_trunc, 1ull);
  } else {                               // split
    atomicAdd(&st.splits, 1ull);
  }
}

__device__ __forceinline__ unsigned long long bcast64(unsigned long long v, int src) {
  const unsigned lo = __shfl((unsigned)v, src), hi = __shfl((unsigned)(v >> 32), src);
  return ((unsigned long long)hi << 32) | lo;
}

template <typename R>
__global__ __launch_bounds__(kTraceBlock) void trace_level_kernel(TraceArgs<R> a) {
  using A = Arith<R>;
  const int lane = threadIdx.x & (kWave - 1);
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  if (a.ctr->err & kErrBadInput) return;
  const int level = a.level;
  const unsigned long long n_children = min(a.ctr->count[level], a.capacity);
  const unsigned long long n_seeds =
      (unsigned long long)(a.seed_sg_end - a.seed_sg_begin) * (12ull << (2 * level));
  const unsigned long long total = n_children + n_seeds;
  if (total == 0) return;
  const Tracer<R> T(a);
  Ray<R> L;
  bool active = false;
  unsigned steps = 0;
  unsigned long long w_next = 0, w_end = 0;
  bool drained = false;

  for (;;) {
    // ---- refill idle lanes from the wave's chunk of the level queue ----
    unsigned long long idle = __ballot(!active);
    if (!drained && idle && (__popcll(idle) >= a.refill || idle == ~0ull)) {
      for (;;) {
        idle = __ballot(!active);
        if (!idle) break;
        if (w_next >= w_end) {
          unsigned long long b = 0;
          if (lane == 0) b = atomicAdd(&a.ctr->head[level], (unsigned long long)a.chunk);
          b = bcast64(b, 0);
          if (b >= total) { drained = true; break; }
          w_next = b;
          w_end = min(b + (unsigned long long)a.chunk, total);
        }
        const unsigned long long idx = w_next + __popcll(idle & below);
        const bool take = !active && idx < w_end;
        w_next += __popcll(__ballot(take));
        if (take) {
          if (T.start(L, idx, n_children)) {
            active = true;
            steps = 0;
          } else {
            flush_end(a, L, 0);
          }
        }
      }
    }
    if (!__ballot(active)) {
      if (drained) break;
      continue;
    }
    if (active) {
      // ---- one cell: exit distance, split test, deposit, step ----
      const R te = rmin(L.t0, rmin(L.t1, L.t2));
      const int ax = (L.t0 == te) ? 0 : ((L.t1 == te) ? 1 : 2);
      bool split = false;
      if (level < L.level_max) {
        if constexpr (sizeof(R) == 4) {
          const float u = te * L.hloc;
          const float gap = u * u - L.split_t2;
          const float tol = fmaf(2.0f * u + L.eps_u, L.eps_u, L.split_t2 * 9.6e-7f);
          split = fabsf(gap) <= tol ? T.split_exact(L) : gap > 0.0f;
        } else {
          const double u = te * L.hloc;
          split = ldexp(12.0, 2 * level) < L.four_pi_phi_c * (u * u);
        }
      }
      const unsigned long long smask = __ballot(split);
      if (smask) {
        const int leader = __ffsll((unsigned long long)smask) - 1;
        unsigned long long base = 0;
        if (lane == leader) base = atomicAdd(&a.ctr->count[level + 1], 4ull * (unsigned long long)__popcll(smask));
        base = bcast64(base, leader);
        if (split) {
          const unsigned long long dst = base + 4ull * (unsigned long long)__popcll(smask & below);
          if (dst + 4 <= a.capacity) {
            const double Pc = 0.25 * L.P;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              a.out.pix[dst + k] = 4ull * L.pix + (uint64_t)k;
              a.out.sg[dst + k] = L.sg;
              a.out.r[dst + k] = L.r;
              a.out.P[dst + k] = Pc;
            }
          } else {
            atomicOr(&a.ctr->err, kErrOverflow);
            atomicAdd(&a.ctr->lost_rays, 4ull);
            unsafeAtomicAdd(&a.ctr->lost_P, L.P);
          }
          flush_end(a, L, 2);
          active = false;
        }
      }
      if (!split) {
        const R dr = te - L.r;
        if (dr > (R)0) {
          const R tau = L.kap * L.sigma * dr;
          const double dP = L.P * A::neg_expm1(tau);
          unsafeAtomicAdd(&a.acc_abs[L.lin], dP);
          if (L.eexc != 0.0) unsafeAtomicAdd(&a.acc_heat[L.lin], dP * L.eexc);
          L.P -= dP;
          L.segs++;
          L.r = te;
        }
        // step across the exit face
        int dir;
        if (ax == 0) {
          dir = L.d0 > (R)0 ? 1 : -1;
          L.c0 += dir;
          L.lin += dir;
          L.t0 = A::tplane((R)(L.c0 + (dir > 0)), L.s0, L.d0, L.i0, L.hinv);
        } else if (ax == 1) {
          dir = L.d1 > (R)0 ? 1 : -1;
          L.c1 += dir;
          L.lin += dir * L.n0;
          L.t1 = A::tplane((R)(L.c1 + (dir > 0)), L.s1, L.d1, L.i1, L.hinv);
        } else {
          dir = L.d2 > (R)0 ? 1 : -1;
          L.c2 += dir;
          L.lin += dir * L.n0 * L.n1;
          L.t2 = A::tplane((R)(L.c2 + (dir > 0)), L.s2, L.d2, L.i2, L.hinv);
        }
        if (L.P < L.pmin) {
          flush_end(a, L, 1);
          active = false;
        } else if (++steps > a.max_steps) {
          // cell indices move monotonically, so this bound is never reached by a correct trace
          atomicOr(&a.ctr->err, kErrInternal);
          flush_end(a, L, 0);
          active = false;
        } else {
          const int cax = ax == 0 ? L.c0 : (ax == 1 ? L.c1 : L.c2);
          const int nax = ax == 0 ? L.n0 : (ax == 1 ? L.n1 : L.n2);
          const R k = ((unsigned)cax < (unsigned)nax) ? a.kappa[L.lin] : (R)-1;
          if (k < (R)0) {
            if (!T.settle(L, ax, dir)) {
              flush_end(a, L, 0);
              active = false;
            }
          } else {
            L.kap = k;
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Per-cell kernels
// ---------------------------------------------------------------------------
__device__ __forceinline__ int grid_of(const GridDev* grids, int n_grids, long long cell) {
  int lo = 0, hi = n_grids - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (grids[mid].cell_off <= cell) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ void reset_kernel(Counters* ctr, SgStats* stats, int n_sg, double* prob_abs, int n_prob) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    for (int l = 0; l < kLevels; ++l) { ctr->count[l] = 0; ctr->head[l] = 0; }
    ctr->lost_rays = 0; ctr->lost_P = 0.0; ctr->err = 0;
  }
  if (i < n_sg) stats[i] = SgStats{0.0, 0.0, 0ull, 0ull, 0ull, 0ull};
  if (i < n_prob) prob_abs[i] = 0.0;
}

__global__ void reset_levels_kernel(Counters* ctr) {
  const int l = threadIdx.x;
  if (l < kLevels) { ctr->count[l] = 0; ctr->head[l] = 0; }
}

// Absorber column per root-cell length, input checks, zeroed accumulators.
template <typename R>
__global__ void prep_kernel(const GridDev* grids, int n_grids, const ProblemDev* probs, long long n_cells,
                            R* kappa, double* acc_abs, double* acc_heat, Counters* ctr) {
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n_cells;
       c += (long long)gridDim.x * blockDim.x) {
    const int g = grid_of(grids, n_grids, c);
    const GridDev& G = grids[g];
    const long long local = c - G.cell_off;
    const float nh = G.n_h[local], xh = G.x_hi[local];
    if (!(nh >= 0.0f) || !(xh >= 0.0f) || !(xh <= 1.0f) || !isfinite(nh)) atomicOr(&ctr->err, kErrBadInput);
    const double dx_root = G.is_child ? 2.0 * G.dx_cm : G.dx_cm;
    R k = (R)((double)nh * (double)xh * dx_root);
    if (!G.is_child) {
      // a root cell under a child grid carries -(child + 1)
      const int i = (int)(local % G.nx), j = (int)((local / G.nx) % G.ny), kk = (int)(local / ((long long)G.nx * G.ny));
      for (int q = g + 1; q < n_grids && grids[q].is_child && grids[q].problem == G.problem; ++q) {
        const GridDev& C = grids[q];
        if (i >= C.ox && i < C.ox + C.nx / 2 && j >= C.oy && j < C.oy + C.ny / 2 && kk >= C.oz && kk < C.oz + C.nz / 2)
          k = (R)(-(q + 1));
      }
    }
    kappa[c] = k;
    acc_abs[c] = 0.0;
    acc_heat[c] = 0.0;
  }
}

// k_ph and heating per absorber; per-problem absorbed totals.
__global__ void finalize_kernel(const GridDev* grids, int n_grids, long long n_cells, const double* acc_abs,
                                const double* acc_heat, double* prob_abs, const Counters* ctr) {
  if (ctr->err & kErrBadInput) return;
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n_cells;
       c += (long long)gridDim.x * blockDim.x) {
    const int g = grid_of(grids, n_grids, c);
    const GridDev& G = grids[g];
    const long long local = c - G.cell_off;
    const double nabs = (double)G.n_h[local] * (double)G.x_hi[local];
    const double vol = G.dx_cm * G.dx_cm * G.dx_cm;
    const double ab = acc_abs[c], he = acc_heat[c];
    double k = 0.0, h = 0.0;
    if (nabs > 0.0) {
      k = ab / (nabs * vol);
      h = he / (nabs * vol);
    }
    G.out_kph[local] = k;
    G.out_heat[local] = h;
    if (ab != 0.0) unsafeAtomicAdd(&prob_abs[G.problem], ab);
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers (called by the runtime on its stream).
// ---------------------------------------------------------------------------
hipError_t launch_reset(hipStream_t s, Counters* ctr, SgStats* stats, int n_sg, double* prob_abs, int n_prob) {
  const int n = n_sg > n_prob ? n_sg : n_prob;
  const int blocks = (n > 0 ? n : 1) / 256 + 1;
  hipLaunchKernelGGL(reset_kernel, dim3(blocks), dim3(256), 0, s, ctr, stats, n_sg, prob_abs, n_prob);
  return hipGetLastError();
}

hipError_t launch_reset_levels(hipStream_t s, Counters* ctr) {
  hipLaunchKernelGGL(reset_levels_kernel, dim3(1), dim3(64), 0, s, ctr);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_prep(hipStream_t s, int num_cu, const GridDev* grids, int n_grids, const ProblemDev* probs,
                       long long n_cells, R* kappa, double* acc_abs, double* acc_heat, Counters* ctr) {
  long long blocks = (n_cells + 255) / 256;
  if (blocks > 32LL * num_cu) blocks = 32LL * num_cu;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(prep_kernel<R>, dim3((unsigned)blocks), dim3(256), 0, s, grids, n_grids, probs, n_cells, kappa,
                     acc_abs, acc_heat, ctr);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_trace_level(hipStream_t s, int blocks, const TraceArgs<R>& args) {
  hipLaunchKernelGGL(trace_level_kernel<R>, dim3(blocks), dim3(kTraceBlock), 0, s, args);
  return hipGetLastError();
}

hipError_t launch_finalize(hipStream_t s, int num_cu, const GridDev* grids, int n_grids, long long n_cells,
                           const double* acc_abs, const double* acc_heat, double* prob_abs, const Counters* ctr) {
  long long blocks = (n_cells + 255) / 256;
  if (blocks > 32LL * num_cu) blocks = 32LL * num_cu;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)blocks), dim3(256), 0, s, grids, n_grids, n_cells, acc_abs,
                     acc_heat, prob_abs, ctr);
  return hipGetLastError();
}

template hipError_t launch_prep<float>(hipStream_t, int, const GridDev*, int, const ProblemDev*, long long, float*,
                                       double*, double*, Counters*);
template hipError_t launch_prep<double>(hipStream_t, int, const GridDev*, int, const ProblemDev*, long long, double*,
                                        double*, double*, Counters*);
template hipError_t launch_trace_level<float>(hipStream_t, int, const TraceArgs<float>&);
template hipError_t launch_trace_level<double>(hipStream_t, int, const TraceArgs<double>&);

hipError_t trace_occupancy(int precision, int* blocks_per_cu) {
  if (precision == 0)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, trace_level_kernel<double>, kTraceBlock, 0);
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, trace_level_kernel<float>, kTraceBlock, 0);
}

}  // namespace moray
