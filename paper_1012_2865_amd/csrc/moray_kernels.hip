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
// criterion at each cell exit (Eq. split), and deposits P (1 - e^-tau) into
// the (problem, group) accumulator of the cell (Eqs. dtau, flux, kph; heating
// is the group-weighted sum formed in finalize, Eq. gamma). Deposits combine
// in a per-wave LDS table and reach the float64 accumulators in HBM as
// atomics only when evicted; per-tree ray statistics combine in a per-block
// LDS table. Idle lanes refill from a private chunk of the level queue
// claimed with one atomic. Children of splitting lanes are compacted with a
// wave ballot and written as four consecutive structure-of-arrays records.
#include "moray_device.h"

#include <hip/hip_runtime.h>
#include <cfloat>
#include <cmath>
#include <cstdint>
#include <type_traits>

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

// sin and cos of beta in [0, pi/4]: their Taylor series about 0 (coefficients
// 1/n!) through x^19 and x^20 in Horner form; the first omitted terms are
// below 1e-19 relative there, and the rounding of the evaluation stays within
// 1 ulp (0.67 ulp for sin, 0.87 for cos over 4e6 points against long double).
// Used instead of the general sincos, whose argument reduction for large
// arguments would set the trace kernel's register peak.
__device__ __forceinline__ void sincos_octant(double beta, double& s, double& c) {
  const double x2 = beta * beta;
  double ps = 1.0 / 121645100408832000.0;      // 1/19!
  ps = fma(ps, -x2, 1.0 / 355687428096000.0);  // 1/17!
  ps = fma(ps, -x2, 1.0 / 1307674368000.0);    // 1/15!
  ps = fma(ps, -x2, 1.0 / 6227020800.0);       // 1/13!
  ps = fma(ps, -x2, 1.0 / 39916800.0);         // 1/11!
  ps = fma(ps, -x2, 1.0 / 362880.0);           // 1/9!
  ps = fma(ps, -x2, 1.0 / 5040.0);             // 1/7!
  ps = fma(ps, -x2, 1.0 / 120.0);              // 1/5!
  ps = fma(ps, -x2, 1.0 / 6.0);                // 1/3!
  s = fma(beta * x2, -ps, beta);
  double pc = 1.0 / 2432902008176640000.0;     // 1/20!
  pc = fma(pc, -x2, 1.0 / 6402373705728000.0); // 1/18!
  pc = fma(pc, -x2, 1.0 / 20922789888000.0);   // 1/16!
  pc = fma(pc, -x2, 1.0 / 87178291200.0);      // 1/14!
  pc = fma(pc, -x2, 1.0 / 479001600.0);        // 1/12!
  pc = fma(pc, -x2, 1.0 / 3628800.0);          // 1/10!
  pc = fma(pc, -x2, 1.0 / 40320.0);            // 1/8!
  pc = fma(pc, -x2, 1.0 / 720.0);              // 1/6!
  pc = fma(pc, -x2, 1.0 / 24.0);               // 1/4!
  pc = fma(pc, -x2, 0.5);                      // 1/2!
  c = fma(x2, -pc, 1.0);
}

// I is the integer type of the ring arithmetic: every intermediate is below
// 16 Ns^2, so 32 bits hold it up to level 13.
template <typename I>
__device__ __forceinline__ void healpix_dir_t(int level, uint64_t pix, double& vx, double& vy, double& vz) {
  const I ns = (I)1 << level;
  const int face = (int)(pix >> (2 * level));
  const uint64_t ipf = pix & ((1ull << (2 * level)) - 1ull);
  const I ix = (I)compact_even_bits(ipf);
  const I iy = (I)compact_even_bits(ipf >> 1);
  const int row = face >> 2;                              // 0 north, 1 equator, 2 south
  const I jr = (I)(row + 2) * ns - ix - iy - 1;
  const I jpf = 2 * (face & 3) + (row == 1 ? 0 : 1);
  I nr;
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
    const I m = 2 * (2 * ns - jr);
    z = (double)m / (3.0 * (double)ns);
    sth = sqrt((double)(9 * ns * ns - m * m)) / (3.0 * (double)ns);
    kshift = (int)((jr - ns) & 1);
  }
  I jp = (jpf * nr + ix - iy + 1 + kshift) >> 1;          // the numerator is always even
  if (jp > 4 * nr) jp -= 4 * nr;
  if (jp < 1) jp += 4 * nr;
  const I num = 2 * jp - kshift - 1, den = 2 * nr;
  const I q = num / den, rem = num - q * den;
  double c, s;
  if (2 * rem == den) {
    c = s = sqrt(0.5);
  } else {
    const bool low = 2 * rem < den;
    const I m = low ? rem : den - rem;
    const double beta = ((double)m / (double)den) * (M_PI / 2.0);
    double sb, cb;
    sincos_octant(beta, sb, cb);
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

__device__ void healpix_dir(int level, uint64_t pix, double& vx, double& vy, double& vz) {
  if (level <= 13) healpix_dir_t<int32_t>(level, pix, vx, vy, vz);
  else healpix_dir_t<int64_t>(level, pix, vx, vy, vz);
}

// A point on a cell plane belongs to the upper cell when the direction
// component is >= 0, else to the lower one.
__device__ __forceinline__ int cell_rule(double x, double d) { return d >= 0.0 ? (int)floor(x) : (int)ceil(x) - 1; }
__device__ __forceinline__ int floor_half(int c) { return c >= 0 ? c / 2 : -((-c + 1) / 2); }
template <typename T> __device__ __forceinline__ T sel3(int k, T a, T b, T c) { return k == 0 ? a : (k == 1 ? b : c); }

// One in-order counter covers a wave's vector loads, stores and atomics. A
// load still in flight where a rare path (a ray start, a grid change, a
// float64 split re-check) rejoins the hot loop makes the compiler wait at the
// join for that counter to reach zero, which includes every deposit atomic
// issued since; those paths therefore finish their own loads before rejoining.
__device__ __forceinline__ void finish_vector_loads() { __builtin_amdgcn_s_waitcnt(0x0F70); }  // vmcnt(0) alone

// ---------------------------------------------------------------------------
// Geometry, float64: the definition's expressions (true division, no
// contraction), so every decision equals the reference's.
// ---------------------------------------------------------------------------
struct Geom64 {
  double d0, d1, d2;       // direction
  double s0, s1, s2;       // source in local cells
  double t0, t1, t2;       // distance to the next plane per axis, root cells
  double r;                // radius, root cells
  double hinv, hloc;

  __device__ void set_dir(const double v[3]) { d0 = v[0]; d1 = v[1]; d2 = v[2]; }
  __device__ double dir64(int k) const { return sel3(k, d0, d1, d2); }
  __device__ double src64(int k) const { return sel3(k, s0, s1, s2); }
  __device__ float dirf(int k) const { return (float)sel3(k, d0, d1, d2); }
  __device__ void set_radius(double r64) { r = r64; }
  __device__ double radius64() const { return r; }
  __device__ double plane(double d, double s, int c) const {
    if (d == 0.0) return __builtin_huge_val();
    return (((double)(c + (d > 0.0 ? 1 : 0)) - s) / d) * hinv;
  }
  __device__ void set_frame(const double sl[3], int c0, int c1, int c2, bool child) {
    s0 = sl[0]; s1 = sl[1]; s2 = sl[2];
    hinv = child ? 0.5 : 1.0;
    hloc = child ? 2.0 : 1.0;
    t0 = plane(d0, s0, c0); t1 = plane(d1, s1, c1); t2 = plane(d2, s2, c2);
  }
  __device__ int exit_axis() const {
    int ax = 0;
    double b = t0;
    if (t1 < b) { ax = 1; b = t1; }
    if (t2 < b) ax = 2;
    return ax;
  }
  __device__ double te(int ax) const { return sel3(ax, t0, t1, t2); }
  __device__ double exit64(int ax) const { return te(ax); }
  __device__ double chord(int ax) const { return te(ax) - r; }
  __device__ bool positive(double dr, int) const { return dr > 0.0; }
  __device__ void advance(int ax) { r = te(ax); }
  __device__ double local_u(int ax) const { return te(ax) * hloc; }
  __device__ void step(int ax, int cnew) {
    const double d = sel3(ax, d0, d1, d2), s = sel3(ax, s0, s1, s2);
    const double t = (((double)(cnew + (d > 0.0 ? 1 : 0)) - s) / d) * hinv;   // d != 0 on the exit axis
    t0 = ax == 0 ? t : t0;
    t1 = ax == 1 ? t : t1;
    t2 = ax == 2 ? t : t2;
  }
};

// ---------------------------------------------------------------------------
// Geometry, float32: every plane distance is a pair hi + lo of floats.
// The source coordinate is split into a 2^-12-lattice part q (so b - q is
// exact) and a residual e, |e| <= 2^-13; the reciprocal of the float64
// direction into i + j. Then t = (b - q - e)(i + j) = hi + lo, hi = (b-q) i
// rounded, lo = its exact fma residual + (b-q) j - e i. A pair is within
// about 2^-36 / |d| cells of the float64 distance (e rounded to float and the
// dropped e j), so chords, which are differences of pairs, place every
// segment where float64 would up to that: a plane tie closer than that is a
// segment of that length in either of two cells. hi alone is not the
// distance: near the source e i is comparable to it.
// ---------------------------------------------------------------------------
// The float path keeps each lane's float64 direction in LDS rather than in
// registers: it is read only by the rare exact paths (a split test within
// rounding of its threshold, entering or starting in a child grid), and
// recomputing it from the pixel there would set the kernel's register peak.
__device__ __forceinline__ double* lane_dir() {
  __shared__ double sdir[3][kTraceBlock];
  return &sdir[0][threadIdx.x];
}

struct Geom32 {
  float d0, d1, d2;
  float i0, i1, i2, j0, j1, j2;      // 1/d = i + j
  float q0, q1, q2, e0, e1, e2;      // local source = q + e
  float h0, h1, h2, l0, l1, l2;      // plane distance = h + l (root cells)
  float rh, rl;                      // radius = rh + rl
  float hinv, hloc;

  __device__ void set_dir(const double v[3]) {
    d0 = (float)v[0]; d1 = (float)v[1]; d2 = (float)v[2];
    split_inv(v[0], i0, j0); split_inv(v[1], i1, j1); split_inv(v[2], i2, j2);
    double* vd = lane_dir();
    vd[0] = v[0]; vd[kTraceBlock] = v[1]; vd[2 * kTraceBlock] = v[2];
  }
  static __device__ void split_inv(double d, float& i, float& j) {
    if (d == 0.0) { i = 0.0f; j = 0.0f; return; }
    const double inv = 1.0 / d;
    i = (float)inv;
    j = (float)(inv - (double)i);
  }
  __device__ double dir64(int k) const { return lane_dir()[k * kTraceBlock]; }
  __device__ double src64(int k) const { return (double)sel3(k, q0, q1, q2) + (double)sel3(k, e0, e1, e2); }
  __device__ float dirf(int k) const { return sel3(k, d0, d1, d2); }
  __device__ void set_radius(double r64) { rh = (float)r64; rl = (float)(r64 - (double)rh); }
  __device__ double radius64() const { return (double)rh + (double)rl; }
  __device__ void plane(float d, float i, float j, float q, float e, int c, float& h, float& l) const {
    if (d == 0.0f) { h = __builtin_huge_valf(); l = 0.0f; return; }
    const float bs = (float)(c + (d > 0.0f ? 1 : 0)) - q;     // exact
    const float th = bs * i;
    float tl = fmaf(bs, i, -th);
    tl = fmaf(bs, j, tl);
    tl = fmaf(-e, i, tl);
    h = th * hinv;
    l = tl * hinv;
  }
  static __device__ void split_src(double s, float& q, float& e) {
    const double qd = rint(s * 4096.0) * (1.0 / 4096.0);
    q = (float)qd;
    e = (float)(s - (double)q);
  }
  __device__ void set_frame(const double sl[3], int c0, int c1, int c2, bool child) {
    split_src(sl[0], q0, e0); split_src(sl[1], q1, e1); split_src(sl[2], q2, e2);
    hinv = child ? 0.5f : 1.0f;
    hloc = child ? 2.0f : 1.0f;
    plane(d0, i0, j0, q0, e0, c0, h0, l0);
    plane(d1, i1, j1, q1, e1, c1, h1, l1);
    plane(d2, i2, j2, q2, e2, c2, h2, l2);
  }
  // (ah + al) < (bh + bl), exact enough to order distinct planes
  static __device__ bool lt(float ah, float al, float bh, float bl) { return ((ah - bh) + (al - bl)) < 0.0f; }
  __device__ int exit_axis() const {
    int ax = 0;
    float bh = h0, bl = l0;
    if (lt(h1, l1, bh, bl)) { ax = 1; bh = h1; bl = l1; }
    if (lt(h2, l2, bh, bl)) ax = 2;
    return ax;
  }
  __device__ float chord(int ax) const {
    return (sel3(ax, h0, h1, h2) - rh) + (sel3(ax, l0, l1, l2) - rl);
  }
  // a pair resolves distances to ~2^-46 t: anything below 2^-40 t is a plane tie (dr = 0 in float64)
  __device__ bool positive(float dr, int ax) const { return dr > sel3(ax, h0, h1, h2) * 9.094947e-13f; }
  __device__ void advance(int ax) { rh = sel3(ax, h0, h1, h2); rl = sel3(ax, l0, l1, l2); }
  // The split test's distance takes both halves of the pair: the low half
  // holds the source's off-lattice residual e (t = (b - q - e) / d), which
  // near the source is not small against the high half.
  __device__ float local_u(int ax) const { return (sel3(ax, h0, h1, h2) + sel3(ax, l0, l1, l2)) * hloc; }
  __device__ double exit64(int ax) const { return (double)sel3(ax, h0, h1, h2) + (double)sel3(ax, l0, l1, l2); }
  // The exit axis always has a nonzero direction component (an axis with
  // none is at infinity), so its next plane needs no special case; selects
  // instead of a branch per axis keep the wave converged.
  __device__ void step(int ax, int cnew) {
    const bool a0 = ax == 0, a1 = ax == 1, a2 = ax == 2;
    const float d = sel3(ax, d0, d1, d2), i = sel3(ax, i0, i1, i2), j = sel3(ax, j0, j1, j2);
    const float q = sel3(ax, q0, q1, q2), e = sel3(ax, e0, e1, e2);
    const float bs = (float)(cnew + (d > 0.0f ? 1 : 0)) - q;  // exact
    const float th = bs * i;
    float tl = fmaf(bs, i, -th);
    tl = fmaf(bs, j, tl);
    tl = fmaf(-e, i, tl);
    const float h = th * hinv, l = tl * hinv;
    h0 = a0 ? h : h0; l0 = a0 ? l : l0;
    h1 = a1 ? h : h1; l1 = a1 ? l : l1;
    h2 = a2 ? h : h2; l2 = a2 ? l : l2;
  }
};

template <typename R> struct GeomOf;
template <> struct GeomOf<double> { using type = Geom64; };
template <> struct GeomOf<float> { using type = Geom32; };

// Photons removed in a segment of optical depth tau: dP = P (1 - e^-tau)
// (Eq. flux), P -= dP. Float64 takes the definition literally. Float32 keeps
// both parts accurate to its own precision: 1 - e^-tau as -expm1f for thin
// segments, and for thick ones (tau > ln 2) the transmitted part P e^-tau
// from expf, the absorbed part as the float64 difference, so dP + P_new = P
// holds to float64 rounding either way.
__device__ __forceinline__ double absorb(double& P, double tau) {
  const double dP = P * -expm1(-tau);
  P -= dP;
  return dP;
}
// One exponential core serves both: Cody-Waite reduction x = k ln2 + r with
// |r| <= ln2/2 (ln 2 split so k ln2 is exact) and the Taylor series of
// expm1(r) to r^7 (truncation below 2e-8 relative there). Then
// e^x - 1 = 2^k expm1(r) + (2^k - 1) is accurate for thin segments (k is 0
// or -1) and e^x = 2^k (1 + expm1(r)) for thick ones, without a branch.
__device__ __forceinline__ double absorb(double& P, float tau) {
  const float x = -tau;
  const float k = rintf(x * 1.44269504f);
  const float r = fmaf(-k, 1.42860677e-06f, fmaf(-k, 0.693145752f, x));
  float q = fmaf(r, 1.0f / 5040.0f, 1.0f / 720.0f);
  q = fmaf(r, q, 1.0f / 120.0f);
  q = fmaf(r, q, 1.0f / 24.0f);
  q = fmaf(r, q, 1.0f / 6.0f);
  q = fmaf(r, q, 0.5f);
  q = fmaf(r * r, q, r);                                   // expm1(r)
  const int ki = (int)k;
  const bool thin = tau < 0.6931472f;
  const float p2 = ldexpf(1.0f, ki);
  const float absorbed = -fmaf(p2, q, p2 - 1.0f);          // 1 - e^-tau (thin: k is 0 or -1)
  const float transmitted = ldexpf(1.0f + q, ki);          // e^-tau
  const double Pin = P;
  const double a = Pin * (double)(thin ? absorbed : transmitted);
  P = thin ? Pin - a : a;
  return thin ? a : Pin - a;
}

// Per-lane ray state. The tree fields (source, photon rates, absorber
// accumulator, cross-section, root grid) belong to the lane's current tree
// and are reloaded only when the lane starts a ray of another tree.
template <typename R>
struct Ray {
  typename GeomOf<R>::type g;
  uint64_t pix;
  uint32_t sg;
  int q;                  // grid index
  int c0, c1, c2;         // local cell
  int n0, n1, n2;         // grid dims
  int lin;                // batch-wide cell index
  double P, pmin;
  uint32_t slot0;         // the ray's (problem, group) accumulator of cell lin is acc[slot0 + lin]
  R sigma;
  R kap;                  // absorber column per root-cell length of the current cell
  R split_t;              // float path: split when u^2 > split_t; float64 path: 12*4^l (inf: never)
  double fpp;             // 4 pi phi_c (float64 path)
  unsigned segs;
  // the lane's tree
  uint32_t tree;
  int level;              // HEALPix level of the tree's rays in this launch
  double sx, sy, sz, P0;
  int root, rn0, rn1, rn2, rcell;
  bool cover;             // its deposits are scaled by the covering factor
  uint32_t astride;       // deposit key of cell lin: slot0 + astride * lin (4: a radiation-pressure record)
  double mscale;          // E_ph / c, 0 when the problem does not ask for the momentum
  double rhalt;           // time-dependent rays: radius where the tree's rays halt in this step
  // optically-thin approximation (section 2.4): while the ray is thin, the
  // absorber column it may still cross before its optical depth from the
  // source reaches tau_thin, rem = (tau_thin - tau) / sigma (units of kap x
  // radius), and the tree's constants for it
  bool thin;
  double rem;
  double kap64;           // the current cell's column in float64 (the thin decision's optical depth)
  R split_t_thin;         // split thresholds of thin rays, as split_t and fpp
  double fpp_thin;
  long long mark_base;
  unsigned tsegs;         // the ray's thin segments
};

template <typename R>
struct Tracer {
  const TraceArgs<R>& a;
  __device__ explicit Tracer(const TraceArgs<R>& args) : a(args) {}

  __device__ void root_frame(Ray<R>& L) const {
    L.q = L.root;
    L.n0 = L.rn0; L.n1 = L.rn1; L.n2 = L.rn2;
    const double sl[3] = {L.sx, L.sy, L.sz};
    L.g.set_frame(sl, L.c0, L.c1, L.c2, false);
    L.lin = L.rcell + L.c0 + L.n0 * (L.c1 + L.n1 * L.c2);
  }

  __device__ void child_frame(Ray<R>& L, int q) const {
    const GridDev& G = a.grids[q];
    L.q = q;
    L.n0 = G.nx; L.n1 = G.ny; L.n2 = G.nz;
    const double sl[3] = {2.0 * (L.sx - (double)G.ox), 2.0 * (L.sy - (double)G.oy), 2.0 * (L.sz - (double)G.oz)};
    L.g.set_frame(sl, L.c0, L.c1, L.c2, true);
    L.lin = (int)G.cell_off + L.c0 + G.nx * (L.c1 + G.ny * L.c2);
  }

  // Enter child grid `ch` from root cell (rc0, rc1, rc2) across axis `ax`
  // moving in direction `dir`, at the current radius: along the crossing axis
  // the fine cell follows from the face, along the others from the position,
  // kept among the two fine cells under the root cell.
  __device__ void enter_child(Ray<R>& L, int ch, int rc0, int rc1, int rc2, int ax, int dir) const {
    const GridDev& G = a.grids[ch];
    const int rc[3] = {rc0, rc1, rc2};
    const int o[3] = {G.ox, G.oy, G.oz};
    const double sr[3] = {L.sx, L.sy, L.sz};
    const double r = L.g.radius64();
    int c[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int lo = 2 * (rc[k] - o[k]);
      if (k == ax) {
        c[k] = lo + (dir < 0 ? 1 : 0);
      } else {
        const double dk = L.g.dir64(k);
        const double x = __dadd_rn(sr[k], __dmul_rn(r, dk));
        const int cl = cell_rule(2.0 * (x - (double)o[k]), dk);
        c[k] = cl < lo ? lo : (cl > lo + 1 ? lo + 1 : cl);
      }
    }
    L.c0 = c[0]; L.c1 = c[1]; L.c2 = c[2];
    child_frame(L, ch);
  }

  // After a step along `ax` by `dir` out of the current grid, or into a root
  // cell covered by a child: find the new leaf cell. Returns false when the
  // ray left the root grid.
  __device__ bool settle(Ray<R>& L, int ax, int dir) const {
    const bool inside = find_cell(L, ax, dir);
    finish_vector_loads();
    return inside;
  }
  __device__ bool find_cell(Ray<R>& L, int ax, int dir) const {
    if (L.q == L.root) {
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
    const GridDev& G = a.grids[L.q];
    const int rc0 = G.ox + floor_half(L.c0), rc1 = G.oy + floor_half(L.c1), rc2 = G.oz + floor_half(L.c2);
    if ((unsigned)rc0 >= (unsigned)L.rn0 || (unsigned)rc1 >= (unsigned)L.rn1 || (unsigned)rc2 >= (unsigned)L.rn2)
      return false;
    const int rlin = L.rcell + rc0 + L.rn0 * (rc1 + L.rn1 * rc2);
    const R k = a.kappa[rlin];
    if (k < (R)0) {
      enter_child(L, (int)(-k) - 1, rc0, rc1, rc2, ax, dir);
      L.kap = a.kappa[L.lin];
    } else {
      L.c0 = rc0; L.c1 = rc1; L.c2 = rc2;
      root_frame(L);
      L.kap = k;
    }
    return true;
  }

  // A ray starts in three steps:
  //   fetch  - its queue record (a child) or its tree and pixel (a seed);
  //   tree   - the tree's constants, unless the lane already holds them;
  //   locate - direction, start cell and frame, and that cell's absorber column.
  __device__ void fetch(Ray<R>& L, bool child, unsigned long long idx, double& r64) const {
    if (child) {
      L.sg = a.in.sg[idx];
      L.pix = a.in.pix[idx];
      r64 = a.in.r[idx];
      L.P = a.in.P[idx];
    } else {
      const unsigned long long npix = 12ull << (2 * a.seed_level);
      L.sg = (uint32_t)(a.seed_sg_begin + idx / npix);
      L.pix = idx % npix;
      r64 = 0.0;
      L.P = -__builtin_huge_val();         // the tree's seed rate, set in locate
    }
  }

  __device__ void load_tree(Ray<R>& L) const {
    const SgDev& S = a.sgs[L.sg];
    const int level = S.level_init + (a.gen - S.gen0);
    L.tree = L.sg;
    L.level = level;
    L.sx = S.sx; L.sy = S.sy; L.sz = S.sz;
    L.P0 = S.P0;
    L.pmin = ldexp(S.pmin0, -2 * (level - S.level_init));
    L.slot0 = (uint32_t)S.acc_slot;
    L.root = S.root_grid;
    L.rn0 = S.rnx; L.rn1 = S.rny; L.rn2 = S.rnz;
    L.rcell = (int)S.rcell_off;
    L.cover = S.covering != 0;
    L.astride = S.acc_stride;
    L.mscale = S.mom_scale;
    L.rhalt = S.r_halt;
    const bool can_split = level < S.level_max;
    if constexpr (sizeof(R) == 4) {
      L.sigma = S.sigma32;
      L.split_t = can_split ? ldexpf(S.split_t2_base, 2 * level) : FLT_MAX;
      L.fpp = 0.0;
    } else {
      L.sigma = S.sigma64;
      L.split_t = can_split ? ldexp(12.0, 2 * level) : __builtin_huge_val();
      L.fpp = S.four_pi_phi_c;
    }
  }

  // The optically-thin constants of the lane's tree (after load_tree).
  __device__ void load_thin(Ray<R>& L) const {
    const SgDev& S = a.sgs[L.sg];
    L.mark_base = S.mark_base;
    const bool can_split = L.level < S.level_max;
    if constexpr (sizeof(R) == 4) {
      L.split_t_thin = can_split ? ldexpf(S.split_t2_thin, 2 * L.level) : FLT_MAX;
      L.fpp_thin = 0.0;
    } else {
      L.split_t_thin = L.split_t;
      L.fpp_thin = S.four_pi_phi_thin;
    }
  }

  // Thin state of a fetched ray (before locate). A thin ray has removed no
  // photons, so its rate is its seed's, quartered per level; its queue
  // record holds -(1 + rem) in place of the rate (its parent staged
  // -4 (1 + rem), which the child writer quarters like any rate). A seed is
  // thin when its tree uses the approximation. rem is capped at kRemMax (a
  // zero cross-section), which keeps every record finite.
  static constexpr double kRemMax = 1e300;
  __device__ void thin_start(Ray<R>& L) const {
    L.tsegs = 0;
    const SgDev& S = a.sgs[L.sg];
    if (L.P == -__builtin_huge_val()) {
      L.thin = S.tau_thin > 0.0;
      const double r = S.tau_thin / S.sigma64;
      L.rem = r < kRemMax ? r : kRemMax;
    } else if (L.P < 0.0) {
      L.thin = true;
      L.rem = -L.P - 1.0;
      L.P = ldexp(S.P0, -2 * (L.level - S.level_init));
    } else {
      L.thin = false;
    }
  }

  // Does the ray's current cell hold its source (inside or on its boundary)?
  // Only a cell within sqrt(3) local cells of the source can: nearer than 2
  // the test is taken exactly, on the source's float64 local coordinates.
  __device__ bool holds_source(const Ray<R>& L) const {
    const bool child = L.q != L.root;
    if (L.g.radius64() * (child ? 2.0 : 1.0) >= 2.0) return false;
    double sl[3] = {L.sx, L.sy, L.sz};
    if (child) {
      const GridDev& G = a.grids[L.q];
      sl[0] = 2.0 * (L.sx - (double)G.ox);
      sl[1] = 2.0 * (L.sy - (double)G.oy);
      sl[2] = 2.0 * (L.sz - (double)G.oz);
    }
    const int c[3] = {L.c0, L.c1, L.c2};
    bool in = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) in = in && (double)c[k] <= sl[k] && sl[k] <= (double)c[k] + 1.0;
    return in;
  }

  // Start cell of a fetched ray whose tree constants are loaded. Returns false
  // when the ray starts outside the root grid; otherwise the ray is framed in
  // the root cell holding s + r d and `k` receives that cell's column.
  __device__ bool locate(Ray<R>& L, double r64, R& k) const {
    if (L.P < 0.0) L.P = L.P0;
    L.segs = 0;
    double v[3];
    healpix_dir(L.level, L.pix, v[0], v[1], v[2]);
    L.g.set_dir(v);
    L.g.set_radius(r64);
    const double x0 = __dadd_rn(L.sx, __dmul_rn(r64, v[0]));
    const double x1 = __dadd_rn(L.sy, __dmul_rn(r64, v[1]));
    const double x2 = __dadd_rn(L.sz, __dmul_rn(r64, v[2]));
    L.c0 = cell_rule(x0, v[0]); L.c1 = cell_rule(x1, v[1]); L.c2 = cell_rule(x2, v[2]);
    if ((unsigned)L.c0 >= (unsigned)L.rn0 || (unsigned)L.c1 >= (unsigned)L.rn1 || (unsigned)L.c2 >= (unsigned)L.rn2)
      return false;
    root_frame(L);
    k = a.kappa[L.lin];
    return true;
  }

  // The located ray becomes active: in the root cell, or when that cell is
  // covered by a child grid, in the fine cell under it that holds s + r d
  // (exact in floating point; kept in range regardless).
  __device__ void begin(Ray<R>& L, R k) const {
    if (k >= (R)0) {
      L.kap = k;
      return;
    }
    const int ch = (int)(-k) - 1;
    const GridDev& G = a.grids[ch];
    const double r64 = L.g.radius64();
    const double v[3] = {L.g.dir64(0), L.g.dir64(1), L.g.dir64(2)};
    const double x0 = __dadd_rn(L.sx, __dmul_rn(r64, v[0]));
    const double x1 = __dadd_rn(L.sy, __dmul_rn(r64, v[1]));
    const double x2 = __dadd_rn(L.sz, __dmul_rn(r64, v[2]));
    const int f0 = 2 * (L.c0 - G.ox), f1 = 2 * (L.c1 - G.oy), f2 = 2 * (L.c2 - G.oz);
    L.c0 = min(max(cell_rule(2.0 * (x0 - (double)G.ox), v[0]), f0), f0 + 1);
    L.c1 = min(max(cell_rule(2.0 * (x1 - (double)G.oy), v[1]), f1), f1 + 1);
    L.c2 = min(max(cell_rule(2.0 * (x2 - (double)G.oz), v[2]), f2), f2 + 1);
    child_frame(L, ch);
    L.kap = a.kappa[L.lin];
  }

  // Float64 re-evaluation of the split test for the current cell, in the
  // canonical form 12 * 4^l < (4 pi phi_c) * u^2, u = t_exit in local cells.
  __device__ bool split_exact(const Ray<R>& L, bool thin) const {
    const bool sp = split_exact64(L, thin);
    finish_vector_loads();
    return sp;
  }
  __device__ bool split_exact64(const Ray<R>& L, bool thin) const {
    const SgDev& S = a.sgs[L.sg];
    const bool child = L.q != L.root;
    int o[3] = {0, 0, 0};
    if (child) {
      const GridDev& G = a.grids[L.q];
      o[0] = G.ox; o[1] = G.oy; o[2] = G.oz;
    }
    const double v[3] = {L.g.dir64(0), L.g.dir64(1), L.g.dir64(2)};
    const double h = child ? 2.0 : 1.0;
    const double s[3] = {L.sx, L.sy, L.sz};
    const int c[3] = {L.c0, L.c1, L.c2};
    double te = __builtin_huge_val();
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (v[k] == 0.0) continue;
      const double sl = child ? h * (s[k] - (double)o[k]) : s[k];
      const double b = (double)(c[k] + (v[k] > 0.0 ? 1 : 0));
      const double t = ((b - sl) / v[k]) / h;
      te = t < te ? t : te;
    }
    const double u = te * h;
    return ldexp(12.0, 2 * L.level) < (thin ? S.four_pi_phi_thin : S.four_pi_phi_c) * (u * u);
  }

  // thin: the ray is optically thin in this cell and is split against
  // min(1, phi_c) rays per cell face (section 2.4)
  __device__ bool split_test(const Ray<R>& L, int ax, bool thin = false) const {
    if constexpr (sizeof(R) == 4) {
      const float u = L.g.local_u(ax);
      const float t = thin ? L.split_t_thin : L.split_t;
      const float gap = u * u - t;
      const float tol = t * 9.6e-7f;           // 16 float ulp: beyond every rounding of u^2
      if (gap > tol) return true;
      if (gap < -tol) return false;
      return split_exact(L, thin);
    } else {
      const double u = L.g.local_u(ax);
      return L.split_t < (thin ? L.fpp_thin : L.fpp) * (u * u);
    }
  }

  // Covering factor of the segment that starts at the current radius R_0 and
  // has chord dr (root cells), section 2.3: D_edge = 1/2 - max_i D_c,i is
  // the distance from the segment's midpoint to the nearest face of its cell,
  // L_pix = R_0 theta_pix the pixel's width at entry (theta_pix =
  // sqrt(4 pi / N_pix) = sqrt(pi/3) 2^-l), both in local cells, and
  // f_c = (1/2 + D_edge / L_pix)^2, at most 1 (1 also for R_0 = 0). Float64
  // throughout, from the float64 direction and source.
  __device__ double covering_factor(const Ray<R>& L, double dr) const {
    const double h = (double)L.g.hloc;
    const double r0 = L.g.radius64();
    const double rmid = (r0 + 0.5 * dr) * h;
    const int c[3] = {L.c0, L.c1, L.c2};
    double dmax = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double d = fabs(L.g.src64(k) + rmid * L.g.dir64(k) - ((double)c[k] + 0.5));
      dmax = d > dmax ? d : dmax;
    }
    const double lpix = r0 * h * ldexp(1.0233267079464885, -L.level);   // sqrt(pi/3) = 1.02332670794648848...
    if (!(lpix > 0.0)) return 1.0;
    const double f = 0.5 + (0.5 - dmax) / lpix;
    return f * f >= 1.0 ? 1.0 : f * f;
  }
};

// Per-tree statistics of finished rays (segments, splits, escaped and
// truncated rays with their photon rates), combined per block in LDS: a lane
// whose ray ends adds to its tree's entry with LDS atomics, and the block adds
// each entry to the tree's global counters once, when all its waves are done.
// Consecutive rays of a lane seldom share a tree, and a global atomic per ray
// end would sit in the same in-order memory counter as the next absorber
// gather. A tree that finds no free entry among its kTallyProbes probes adds
// to the global counters directly: those are atomics on its tree's counters,
// one address that every ray end of the tree on the device then shares (two
// probes left enough trees of the 64-grid batch without an entry to take its
// step from 37.1 to 42.5 ms; 16 and 32 probes measured alike, a probe of
// the whole table slower). THIN adds a fifth count, the ray's optically thin
// segments (the rays of one tree tend to end together, and one global atomic
// per ray end on the tree's counter serialised at the memory side).
template <bool THIN>
struct TallyTable {
  static constexpr int kRows = THIN ? 5 : 4;
  uint32_t* key;                 // kTallySlots tree indices (kNoTree: free)
  unsigned long long* cnt;       // [kRows][kTallySlots]: segs, splits, n_esc, n_trunc(, thin_segs)
  double* sum;                   // [2][kTallySlots]: esc_P, trunc_P

  // all threads of the block; followed by a block barrier
  __device__ void init() {
    __shared__ uint32_t skey[kTallySlots];
    __shared__ unsigned long long scnt[kRows * kTallySlots];
    __shared__ double ssum[2 * kTallySlots];
    key = skey; cnt = scnt; sum = ssum;
    for (int i = threadIdx.x; i < kTallySlots; i += blockDim.x) {
      key[i] = kNoTree;
#pragma unroll
      for (int r = 0; r < kRows; ++r) cnt[r * kTallySlots + i] = 0ull;
      sum[i] = sum[kTallySlots + i] = 0.0;
    }
  }
  // kind: 0 escaped, 1 truncated, 2 split, 3 halted (its segments only: the
  // photons it holds are summed from the halt list)
  __device__ void add(SgStats* stats, uint32_t sg, unsigned segs, double P, int kind, unsigned tsegs = 0u) {
    const uint32_t h0 = (sg * 0x9E3779B1u) >> (32 - kTallyLog2);
    int slot = -1;
#pragma unroll
    for (int probe = 0; probe < kTallyProbes; ++probe) {
      const uint32_t h = (h0 + probe) & (kTallySlots - 1);
      uint32_t k = __hip_atomic_load(&key[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      if (k == kNoTree) {
        uint32_t seen = kNoTree;
        __hip_atomic_compare_exchange_strong(&key[h], &seen, sg, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_WORKGROUP);
        k = seen == kNoTree ? sg : seen;
      }
      if (k == sg) {
        slot = (int)h;
        break;
      }
    }
    const int c = kind == 2 ? 1 : kind + 2;
    if (slot >= 0) {
      __hip_atomic_fetch_add(&cnt[slot], (unsigned long long)segs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      if (kind < 3)
        __hip_atomic_fetch_add(&cnt[c * kTallySlots + slot], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      if (kind < 2)
        __hip_atomic_fetch_add(&sum[kind * kTallySlots + slot], P, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      if (THIN && tsegs)
        __hip_atomic_fetch_add(&cnt[4 * kTallySlots + slot], (unsigned long long)tsegs, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
    } else {
      SgStats& st = stats[sg];
      if (segs) atomicAdd(&st.segs, (unsigned long long)segs);
      if (THIN && tsegs) atomicAdd(&st.thin_segs, (unsigned long long)tsegs);
      if (kind == 2) {
        atomicAdd(&st.splits, 1ull);
      } else if (kind == 3) {
      } else if (kind == 0) {
        atomicAdd(&st.n_esc, 1ull);
        unsafeAtomicAdd(&st.esc_P, P);
      } else {
        atomicAdd(&st.n_trunc, 1ull);
        unsafeAtomicAdd(&st.trunc_P, P);
      }
    }
  }
  // all threads of the block, after a block barrier that follows every add
  __device__ void flush(SgStats* stats) const {
    for (int i = threadIdx.x; i < kTallySlots; i += blockDim.x) {
      const uint32_t k = key[i];
      if (k == kNoTree) continue;
      SgStats& st = stats[k];
      if (cnt[i]) atomicAdd(&st.segs, cnt[i]);
      if (cnt[kTallySlots + i]) atomicAdd(&st.splits, cnt[kTallySlots + i]);
      if (cnt[2 * kTallySlots + i]) {
        atomicAdd(&st.n_esc, cnt[2 * kTallySlots + i]);
        unsafeAtomicAdd(&st.esc_P, sum[i]);
      }
      if (cnt[3 * kTallySlots + i]) {
        atomicAdd(&st.n_trunc, cnt[3 * kTallySlots + i]);
        unsafeAtomicAdd(&st.trunc_P, sum[kTallySlots + i]);
      }
      if (THIN && cnt[4 * kTallySlots + i]) atomicAdd(&st.thin_segs, cnt[4 * kTallySlots + i]);
    }
  }
};

__device__ __forceinline__ unsigned long long bcast64(unsigned long long v, int src) {
  const unsigned lo = __shfl((unsigned)v, src), hi = __shfl((unsigned)(v >> 32), src);
  return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ int uniform32(int v) { return __builtin_amdgcn_readfirstlane(v); }
// A wave-uniform 64-bit value (the first active lane's) in scalar registers.
__device__ __forceinline__ unsigned long long uniform64(unsigned long long v) {
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ uint32_t cache_index(uint32_t key) {
  return (key * 0x9E3779B1u) >> (32 - kCacheLog2);
}

// Every global store or atomic a wave issues stays outstanding in the same
// in-order counter as its loads, so the next gather of an absorber column
// may wait for it, and float64 atomics are performed at the memory side. The
// trace therefore stages its writes in LDS and issues them in bulk: deposits
// combine in a per-wave cache, evicted sums collect in a per-wave buffer
// drained 64 atomics per instruction, and split parents collect in a per-wave
// stage whose children are written together.

// Deposit combining: each wave keeps a direct-mapped table of (accumulator
// slot, float64 sum) in LDS. The rays of a wave come from one small patch of
// HEALPix pixels, so each cell of their cone receives several of their
// deposits a few steps apart; those add up in LDS and reach the float64
// accumulator in HBM only when the entry is evicted or the launch ends.
// Within an iteration every lane first compares its key, matching lanes add,
// and only then may a lane claim the entry for a new key (one winner per
// entry via compare-and-swap), so every deposit lands in its own cell's sum.
template <bool CACHE>
struct DepositCache;

template <>
struct DepositCache<false> {
  __device__ void init(int) {}
  __device__ void add(double* acc, uint32_t key, double v, bool has, int) { if (has) unsafeAtomicAdd(&acc[key], v); }
  __device__ bool want_drain() const { return false; }
  __device__ void drain(double*, int) {}
  __device__ void flush(double*, int) {}
};

template <>
struct DepositCache<true> {
  uint32_t* key;
  double* val;
  uint32_t* ekey;         // evicted sums waiting for their global atomic
  double* eval;
  int ecount;             // wave-uniform

  __device__ void init(int lane) {
    __shared__ uint32_t skey[kTraceBlock / kWave][kCacheEntries];
    __shared__ double sval[kTraceBlock / kWave][kCacheEntries];
    __shared__ uint32_t sekey[kTraceBlock / kWave][kEvictCap];
    __shared__ double seval[kTraceBlock / kWave][kEvictCap];
    const int wv = threadIdx.x / kWave;
    key = skey[wv];
    val = sval[wv];
    ekey = sekey[wv];
    eval = seval[wv];
    ecount = 0;
    for (int e = lane; e < kCacheEntries; e += kWave) key[e] = kNoSlot;
    __builtin_amdgcn_wave_barrier();
  }
  __device__ bool want_drain() const { return ecount >= kEvictCap - kWave; }
  // one global atomic instruction per 64 buffered sums
  __device__ void drain(double* acc, int lane) {
    __builtin_amdgcn_wave_barrier();
    for (int i = lane; i < ecount; i += kWave) unsafeAtomicAdd(&acc[ekey[i]], eval[i]);
    ecount = 0;
    __builtin_amdgcn_wave_barrier();
  }
  // Every lane of the wave calls this (uniform control flow); one pass per
  // call. Lanes whose key is in the table add to its sum; the others claim
  // their entry by compare-and-swap. A winner swaps its deposit in and passes
  // the entry's old sum to the eviction buffer. A lane that loses the claim
  // sees the winner's key in the failed swap: if it is its own key (two rays
  // of one tree entering the same cell) it adds to the new sum once the
  // winner has swapped, otherwise it passes its deposit to the eviction
  // buffer. The phases are separated by wave barriers: per thread the
  // branches are exclusive, and without a convergent barrier between them
  // the compiler may merge them into one if/else and reorder the LDS ops.
  __device__ void add(double* acc, uint32_t k_new, double v, bool has, int lane) {
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    if (!__ballot(has)) return;
    if (ecount > kEvictCap - kWave) drain(acc, lane);     // room for this call's evictions
    uint32_t h = 0, k = kNoSlot;
    bool match = false;
    if (has) {
      h = cache_index(k_new);
      k = __hip_atomic_load(&key[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      match = k == k_new;
    }
    __builtin_amdgcn_wave_barrier();
    if (match) __hip_atomic_fetch_add(&val[h], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __builtin_amdgcn_wave_barrier();
    const bool claim = has && !match;
    bool won = false, join = false;
    if (claim) {
      uint32_t seen = k;
      won = __hip_atomic_compare_exchange_strong(&key[h], &seen, k_new, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_WORKGROUP);
      join = !won && seen == k_new;
    }
    __builtin_amdgcn_wave_barrier();
    const bool out = claim && !join && (!won || k != kNoSlot);
    const unsigned long long omask = __ballot(out);
    uint32_t ok = k_new;
    double ov = v;
    if (won) {
      // the adds of this call precede the exchange, so the old sum is complete
      ov = __hip_atomic_exchange(&val[h], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      ok = k;
    }
    __builtin_amdgcn_wave_barrier();
    if (join) __hip_atomic_fetch_add(&val[h], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (out) {
      const int e = ecount + __popcll(omask & below);
      ekey[e] = ok;
      eval[e] = ov;
    }
    ecount += __popcll(omask);
    __builtin_amdgcn_wave_barrier();
  }
  __device__ void flush(double* acc, int lane) {
    drain(acc, lane);
    for (int e = lane; e < kCacheEntries; e += kWave) {
      const uint32_t k = key[e];
      if (k != kNoSlot) unsafeAtomicAdd(&acc[k], val[e]);
    }
  }
};

// Radiation pressure: a problem that asks for the momentum keeps one 32-byte
// record per (group, cell), [absorbed rate, momentum x, y, z], so a segment
// makes one deposit of four sums under one key. Keys at or above rec_base
// are such records; below it they are the plain one-sum slots of the other
// problems of the batch. Evicted records are drained with (entry, component)
// spread over consecutive lanes, so the four float64 atomics of a record go
// out in one instruction to one 32-byte-aligned piece of a cache line.
constexpr int kCache4Log2 = 8;                 // entries of the 4-sum table per wave
constexpr int kCache4Entries = 1 << kCache4Log2;

template <bool CACHE>
struct DepositCache4;

template <>
struct DepositCache4<false> {
  uint32_t rec_base;
  __device__ void init(int, uint32_t rb) { rec_base = rb; }
  __device__ void add(double* acc, uint32_t key, const double (&v)[4], bool has, int) {
    if (!has) return;
    unsafeAtomicAdd(&acc[key], v[0]);
    if (key >= rec_base) {
      unsafeAtomicAdd(&acc[key + 1], v[1]);
      unsafeAtomicAdd(&acc[key + 2], v[2]);
      unsafeAtomicAdd(&acc[key + 3], v[3]);
    }
  }
  __device__ bool want_drain() const { return false; }
  __device__ void drain(double*, int) {}
  __device__ void flush(double*, int) {}
};

__device__ __forceinline__ uint32_t cache4_index(uint32_t key) {
  return (key * 0x9E3779B1u) >> (32 - kCache4Log2);
}

template <>
struct DepositCache4<true> {
  uint32_t* key;
  double* val;            // [4][kCache4Entries]
  uint32_t* ekey;
  double* eval;           // [4][kEvictCap]
  int ecount;
  uint32_t rec_base;

  __device__ void init(int lane, uint32_t rb) {
    __shared__ uint32_t skey[kTraceBlock / kWave][kCache4Entries];
    __shared__ double sval[kTraceBlock / kWave][4 * kCache4Entries];
    __shared__ uint32_t sekey[kTraceBlock / kWave][kEvictCap];
    __shared__ double seval[kTraceBlock / kWave][4 * kEvictCap];
    const int wv = threadIdx.x / kWave;
    key = skey[wv];
    val = sval[wv];
    ekey = sekey[wv];
    eval = seval[wv];
    ecount = 0;
    rec_base = rb;
    for (int e = lane; e < kCache4Entries; e += kWave) key[e] = kNoSlot;
    __builtin_amdgcn_wave_barrier();
  }
  __device__ bool want_drain() const { return ecount >= kEvictCap - kWave; }
  // (entry, component) pairs over consecutive lanes: a record's four sums in one instruction
  __device__ void drain(double* acc, int lane) {
    __builtin_amdgcn_wave_barrier();
    for (int j = lane; j < 4 * ecount; j += kWave) {
      const int i = j >> 2, k = j & 3;
      const uint32_t kk = ekey[i];
      if (k == 0 || kk >= rec_base) unsafeAtomicAdd(&acc[kk + k], eval[k * kEvictCap + i]);
    }
    ecount = 0;
    __builtin_amdgcn_wave_barrier();
  }
  // The protocol of the one-sum table (DepositCache<true>::add) with four
  // sums per entry.
  __device__ void add(double* acc, uint32_t k_new, const double (&v)[4], bool has, int lane) {
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    if (!__ballot(has)) return;
    if (ecount > kEvictCap - kWave) drain(acc, lane);
    uint32_t h = 0, k = kNoSlot;
    bool match = false;
    if (has) {
      h = cache4_index(k_new);
      k = __hip_atomic_load(&key[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      match = k == k_new;
    }
    __builtin_amdgcn_wave_barrier();
    if (match) {
#pragma unroll
      for (int c = 0; c < 4; ++c)
        __hip_atomic_fetch_add(&val[c * kCache4Entries + h], v[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    __builtin_amdgcn_wave_barrier();
    const bool claim = has && !match;
    bool won = false, join = false;
    if (claim) {
      uint32_t seen = k;
      won = __hip_atomic_compare_exchange_strong(&key[h], &seen, k_new, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_WORKGROUP);
      join = !won && seen == k_new;
    }
    __builtin_amdgcn_wave_barrier();
    const bool out = claim && !join && (!won || k != kNoSlot);
    const unsigned long long omask = __ballot(out);
    uint32_t ok = k_new;
    double ov[4] = {v[0], v[1], v[2], v[3]};
    if (won) {
#pragma unroll
      for (int c = 0; c < 4; ++c)
        ov[c] = __hip_atomic_exchange(&val[c * kCache4Entries + h], v[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      ok = k;
    }
    __builtin_amdgcn_wave_barrier();
    if (join) {
#pragma unroll
      for (int c = 0; c < 4; ++c)
        __hip_atomic_fetch_add(&val[c * kCache4Entries + h], v[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    if (out) {
      const int e = ecount + __popcll(omask & below);
      ekey[e] = ok;
#pragma unroll
      for (int c = 0; c < 4; ++c) eval[c * kEvictCap + e] = ov[c];
    }
    ecount += __popcll(omask);
    __builtin_amdgcn_wave_barrier();
  }
  __device__ void flush(double* acc, int lane) {
    drain(acc, lane);
    for (int j = lane; j < 4 * kCache4Entries; j += kWave) {
      const int e = j >> 2, c = j & 3;
      const uint32_t kk = key[e];
      if (kk != kNoSlot && (c == 0 || kk >= rec_base)) unsafeAtomicAdd(&acc[kk + c], val[c * kCache4Entries + e]);
    }
  }
};

// Split parents waiting for their children to be written: the children of a
// stage go to the wave's current segment of the next level's queue (its home
// segment at first) through blocks of slots it reserves with one atomic, in
// coalesced stores (lane c writes child c), four consecutive records per
// parent. A segment that is full sends the wave on to the next one, so the
// splits of a few neighbouring pixel ranges (the rays towards a grid's
// corners, say) can fill one segment without losing children while the
// queue has room elsewhere; only when every segment is full are children
// lost (an overflow, which the host answers by tracing in smaller chunks).
struct SplitStage {
  uint64_t* pix;
  uint32_t* sg;
  double* r;
  double* P;
  int count;                                    // wave-uniform
  int wseg;                                     // segment of the wave's current reservation
  unsigned long long o_next, o_end;             // the wave's reserved slots of segment wseg

  __device__ void init(int home) {
    __shared__ uint64_t spix[kTraceBlock / kWave][kStageCap];
    __shared__ uint32_t ssg[kTraceBlock / kWave][kStageCap];
    __shared__ double sr[kTraceBlock / kWave][kStageCap];
    __shared__ double sP[kTraceBlock / kWave][kStageCap];
    const int wv = threadIdx.x / kWave;
    pix = spix[wv]; sg = ssg[wv]; r = sr[wv]; P = sP[wv];
    count = 0;
    wseg = home;
    o_next = o_end = 0;
  }
  template <typename R>
  __device__ void write(const TraceArgs<R>& a, int lane) {
    __builtin_amdgcn_wave_barrier();
    const unsigned long long need = 4ull * (unsigned long long)count;
    unsigned long long done = 0;
    int full = 0;                                           // segments found full in this call
    while (done < need) {
      if (o_next >= o_end) {
        const unsigned long long want = need - done;
        const unsigned long long grab = want > a.reserve ? want : a.reserve;
        unsigned long long fresh = 0;
        if (lane == 0) fresh = atomicAdd(&a.ctr->count[a.cout][wseg], grab);
        fresh = bcast64(fresh, 0);
        if (fresh >= a.seg_cap) {
          if (++full >= a.nseg) break;                      // every segment is full
          wseg = (wseg + 1) & (a.nseg - 1);
          continue;
        }
        o_next = fresh;
        o_end = fresh + grab < a.seg_cap ? fresh + grab : a.seg_cap;
      }
      const unsigned long long n = need - done < o_end - o_next ? need - done : o_end - o_next;
      const unsigned long long base = (unsigned long long)wseg * a.seg_cap + o_next;
      for (unsigned long long c = lane; c < n; c += kWave) {
        const unsigned long long k = done + c;
        const int p = (int)(k >> 2);
        a.out.pix[base + c] = 4ull * pix[p] + (k & 3);
        a.out.sg[base + c] = sg[p];
        a.out.r[base + c] = r[p];
        a.out.P[base + c] = 0.25 * P[p];
      }
      o_next += n;
      done += n;
    }
    if (done < need) {
      for (unsigned long long k = done + lane; k < need; k += kWave) {
        if (k == done) atomicOr(&a.ctr->err, kErrOverflow);
        atomicAdd(&a.ctr->lost_rays, 1ull);
        unsafeAtomicAdd(&a.ctr->lost_P, 0.25 * P[k >> 2]);
      }
    }
    count = 0;
    __builtin_amdgcn_wave_barrier();
  }
  // all lanes of the wave, at its end: the unused slots of its last
  // reservation become empty slots
  template <typename R>
  __device__ void close(const TraceArgs<R>& a, int lane) const {
    for (unsigned long long i = o_next + lane; i < o_end; i += kWave)
      a.out.sg[(unsigned long long)wseg * a.seg_cap + i] = kNoTree;
  }
};

// PHYS selects the optional physics some tree of the launch asks for:
// kPhysCover scales deposits by the covering factor (section 2.3), kPhysRadp
// adds the absorbed momentum E_ph dP / c n to three more sums per cell
// (radiation pressure, section 2.5.4), kPhysHalt halts every ray at its
// tree's radius r_halt (time-dependent rays, section 2.1 and section 3.1
// step 3j): the segment in that cell ends there and the ray, with the
// photons it still carries, goes to the halt list for the next step.
// kPhysThin applies the optically-thin approximation (section 2.4, Eq.
// optthin): a ray whose optical depth from its source stays below tau_thin
// through a cell removes no photons there, is split against min(1, phi_c)
// rays per cell face, and sets its tree's mark on the cell (a byte; the rate
// sigma P / (Omega_ray r_cell^2) is the same for every thin ray of a tree,
// so finalize adds it once per marked tree); in a cell that holds the source
// it adds its general deposit to the cell's second sum instead.
// PHYS = 0 is the plain trace.
constexpr int kPhysCover = 1, kPhysRadp = 2, kPhysHalt = 4, kPhysThin = 8;

// Waves per SIMD the register budget is set for: three (at most 168 VGPRs),
// which the LDS of a block (four waves) also allows; two for the
// radiation-pressure variant with its four-sum deposit table, whose LDS
// leaves room for two blocks per CU.
template <typename R, bool CACHE, int PHYS>
__global__ __launch_bounds__(kTraceBlock) __attribute__((amdgpu_waves_per_eu(CACHE && (PHYS & kPhysRadp) ? 2 : 3)))
void trace_level_kernel(TraceArgs<R> a) {
  constexpr bool COVER = (PHYS & kPhysCover) != 0, RADP = (PHYS & kPhysRadp) != 0, HALT = (PHYS & kPhysHalt) != 0;
  constexpr bool THIN = (PHYS & kPhysThin) != 0;
  static_assert(!(THIN && (RADP || HALT)), "the optically-thin approximation is a single-pass option");
  const int lane = threadIdx.x & (kWave - 1);
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  __shared__ int s_bad;
  TallyTable<THIN> tally;
  tally.init();
  if (threadIdx.x == 0) s_bad = (a.ctr->err & kErrBadInput) != 0;
  __syncthreads();
  if (s_bad) return;      // the whole block
  const int K = a.nseg;                      // a power of two
  const int kshift = __ffs(K) - 1;
  const unsigned long long npix = 12ull << (2 * a.seed_level);
  const unsigned long long n_seeds = (unsigned long long)(a.seed_sg_end - a.seed_sg_begin) * npix;
  const unsigned long long* cnt_in = a.ctr->count[a.cin];
  unsigned long long* head_in = a.ctr->head[a.cin];
  // rays claimed per atomic: the launch's setting, halved while the level
  // holds less than one claim for every wave of the launch, down to one ray
  // per lane, so that a level of few rays spreads over the waves instead of
  // queueing several rays behind each lane of a few of them
  // (kept in LDS: the claim path alone reads it, and a scalar register held
  // through the step loop would push the loop's own values out of theirs)
  __shared__ unsigned s_chunk[kTraceBlock / kWave];
  {
    unsigned long long n = lane < K ? min(cnt_in[lane], a.seg_cap) : 0ull;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
      const unsigned lo = __shfl_xor((unsigned)n, o), hi = __shfl_xor((unsigned)(n >> 32), o);
      n += ((unsigned long long)hi << 32) | lo;
    }
    n += n_seeds;
    const unsigned long long waves = (unsigned long long)gridDim.x * (kTraceBlock / kWave);
    unsigned chunk = (unsigned)a.chunk;
    while (chunk >= 2u * kWave && (unsigned long long)chunk * waves > n) chunk >>= 1;
    s_chunk[threadIdx.x / kWave] = chunk;   // every lane holds the same sum and stores the same value
  }
  // the wave's home segment: it claims there first and writes children there
  const int home = (int)((blockIdx.x * (kTraceBlock / kWave) + threadIdx.x / kWave) % (unsigned)K);
  const Tracer<R> T(a);
  Ray<R> L;
  int ended = -1;          // kind of the lane's ray that ended and is not yet tallied
  // with radiation pressure one deposit carries four sums (one table entry each)
  std::conditional_t<RADP, DepositCache4<CACHE>, DepositCache<CACHE>> cache;
  if constexpr (RADP) cache.init(lane, a.rec_base);
  else cache.init(lane);
  SplitStage stage;
  stage.init(home);
  bool active = false;
  unsigned steps = 0;
  L.tree = kNoTree;
  // the wave's current claim: [w_next, w_end) of segment w_seg, whose first
  // w_nch indices are queue slots and the rest seed numbers from w_slo on
  unsigned long long w_next = 0, w_end = 0, w_nch = 0, w_slo = 0;
  int w_seg = home;
  bool drained = false;
  // time-dependent rays: the wave's reserved block [h_next, h_end) of the
  // halt list, and the rays it halted in this launch
  unsigned long long h_next = 0, h_end = 0, h_count = 0;
  // the step's two uniform operands, held in vector registers in the float
  // kernels: their scalar registers are full, and from there the operands
  // were reloaded (a kernel-argument load and lane reads of spilled scalars)
  // at every step; the float64 kernels have no vector registers to spare
  uint64_t kappa_v = (uint64_t)a.kappa;
  unsigned max_steps_v = a.max_steps;
  if constexpr (sizeof(R) == 4) asm volatile("" : "+v"(kappa_v), "+v"(max_steps_v));
  const __attribute__((address_space(1))) R* const kappa_step = (const __attribute__((address_space(1))) R*)kappa_v;
  // the float kernel with the optically-thin approximation gathers the
  // float64 columns instead (the same values before rounding to float), so
  // that its thin decisions see the optical depth the float64 path sees
  constexpr bool K64 = THIN && sizeof(R) == 4;
  uint64_t kappa64_v = (uint64_t)a.kappa64;
  if constexpr (K64) asm volatile("" : "+v"(kappa64_v));
  const __attribute__((address_space(1))) double* const kappa64_step =
      (const __attribute__((address_space(1))) double*)kappa64_v;

  for (;;) {
    if (ended >= 0) {
      tally.add(a.stats, HALT ? L.sg % a.tree_fold : L.sg, L.segs, L.P, ended, THIN ? L.tsegs : 0u);
      ended = -1;
    }
    // ---- refill idle lanes from the wave's claim on the level queue ----
    // Every idle lane first gets its queue slot or seed number (claiming as
    // many chunks as that takes), then all of them start in one pass; lanes
    // whose slot turns out empty wait for the next refill.
    const unsigned long long idle = __ballot(!active);
    if (!drained && idle && (__popcll(idle) >= a.refill || idle == ~0ull)) {
      unsigned long long left = idle;
      bool take = false, child = false;
      unsigned long long q = 0;
      while (left) {
        if (w_next >= w_end) {
          // Claim a chunk: from the wave's current segment while it has rays
          // left; once it is used up, every lane reads one segment's counters
          // (one round trip for all of them), the wave picks the first segment
          // with rays left after it, and claims there with one atomic; a claim
          // that finds the segment used up in the meantime looks again. No
          // segment with rays left: the level is drained.
          bool got = false;
          for (;;) {
            // the current segment first: one load while it lasts
            {
              const unsigned long long c_nch = min(cnt_in[w_seg], a.seg_cap);
              const unsigned long long c_slo = ((unsigned long long)w_seg * n_seeds) >> kshift;
              const unsigned long long c_size = c_nch + ((((unsigned long long)w_seg + 1) * n_seeds) >> kshift) - c_slo;
              const unsigned long long seen =
                  uniform64(__hip_atomic_load(&head_in[w_seg], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
              if (seen < c_size) {
                unsigned long long b = 0;
                const unsigned long long chunk = uniform32((int)s_chunk[threadIdx.x / kWave]);
                if (lane == 0) b = atomicAdd(&head_in[w_seg], chunk);
                b = bcast64(b, 0);
                if (b < c_size) {
                  w_nch = c_nch;
                  w_slo = c_slo;
                  w_next = b;
                  w_end = min(b + chunk, c_size);
                  got = true;
                  break;
                }
              }
            }
            bool has = false;
            if (lane < K) {
              const unsigned long long size = min(cnt_in[lane], a.seg_cap) +
                                              ((((unsigned long long)lane + 1) * n_seeds) >> kshift) -
                                              (((unsigned long long)lane * n_seeds) >> kshift);
              has = __hip_atomic_load(&head_in[lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < size;
            }
            const unsigned long long live = __ballot(has);
            if (!live) break;
            const unsigned long long ahead = live & (~0ull << w_seg);
            const int sg = uniform32((int)__ffsll((long long)(ahead ? ahead : live)) - 1);
            // the chosen segment's slots and seeds, once more for the whole wave
            const unsigned long long s_nch = min(cnt_in[sg], a.seg_cap);
            const unsigned long long s_slo = ((unsigned long long)sg * n_seeds) >> kshift;
            const unsigned long long s_size = s_nch + ((((unsigned long long)sg + 1) * n_seeds) >> kshift) - s_slo;
            unsigned long long b = 0;
            const unsigned long long chunk = uniform32((int)s_chunk[threadIdx.x / kWave]);
            if (lane == 0) b = atomicAdd(&head_in[sg], chunk);
            b = bcast64(b, 0);
            w_seg = sg;
            if (b < s_size) {
              w_nch = s_nch;
              w_slo = s_slo;
              w_next = b;
              w_end = min(b + chunk, s_size);
              got = true;
              break;
            }
          }
          if (!got) { drained = true; break; }
        }
        const unsigned long long idx = w_next + __popcll(left & below);
        const bool mine = ((left >> lane) & 1ull) && idx < w_end;
        if (mine) {
          take = true;
          child = idx < w_nch;
          q = child ? (unsigned long long)w_seg * a.seg_cap + idx : w_slo + (idx - w_nch);
        }
        const unsigned long long got_mask = __ballot(mine);
        w_next += __popcll(got_mask);
        left &= ~got_mask;
      }
      if (take) {
        double r64;
        T.fetch(L, child, q, r64);
        if (L.sg != kNoTree) {
          if (L.sg != L.tree) {
            T.load_tree(L);
            if constexpr (THIN) T.load_thin(L);
          }
          if constexpr (THIN) T.thin_start(L);
          R k;
          if (T.locate(L, r64, k)) {
            T.begin(L, k);
            if constexpr (K64) L.kap64 = a.kappa64[L.lin];
            else if constexpr (THIN) L.kap64 = (double)L.kap;
            active = true;
            steps = 0;
          } else {
            ended = 0;                     // starts outside the root grid: escaped at once
          }
        }
      }
      finish_vector_loads();
    }
    if (!__ballot(active)) {
      if (drained) break;
      continue;
    }
    // ---- one cell: exit plane, split test, deposit, step ----
    int ax = 0;
    bool split = false;
    int e_dir = 0, e_cnew = 0, e_lin = 0;
    bool e_in = false;
    R kpre = (R)0;
    double kpre64 = 0.0;
    bool thin_here = false;
    double tc64 = 0.0;
    if (active) {
      ax = L.g.exit_axis();
      // the next cell is known from the exit axis alone: its column is
      // gathered now, under the split test, the deposit and its combining
      // (an index outside the grid reads cell 0 of the batch, unused)
      e_dir = L.g.dirf(ax) > 0.0f ? 1 : -1;
      e_cnew = sel3(ax, L.c0, L.c1, L.c2) + e_dir;
      e_in = (unsigned)e_cnew < (unsigned)sel3(ax, L.n0, L.n1, L.n2);
      e_lin = L.lin + e_dir * sel3(ax, 1, L.n0, L.n0 * L.n1);
      if constexpr (K64) {
        kpre64 = kappa64_step[e_in ? e_lin : 0];
      } else {
        kpre = kappa_step[e_in ? e_lin : 0];
      }
      if constexpr (THIN) {
        // optically thin in this cell: the optical depth on leaving it, in
        // float64, below tau_thin
        if (L.thin) {
          const double dr64 = L.g.exit64(ax) - L.g.radius64();
          tc64 = dr64 > 0.0 ? L.kap64 * dr64 : 0.0;
          thin_here = tc64 < L.rem;
        }
        split = T.split_test(L, ax, thin_here);
      } else {
        split = T.split_test(L, ax);
      }
    }
    const unsigned long long smask = __ballot(split);
    if (smask) {
      if (split) {
        const int e = stage.count + __popcll(smask & below);
        stage.pix[e] = L.pix;
        stage.sg[e] = L.sg;
        stage.r[e] = L.g.radius64();
        // a thin ray's children carry its remaining column as -(1 + rem)
        stage.P[e] = (THIN && L.thin) ? -4.0 * (1.0 + L.rem) : L.P;
        ended = 2;
        active = false;
      }
      stage.count += __popcll(smask);
    }
    bool dep = false, moved = false;
    uint32_t dkey = 0;
    double dval = 0.0, mval = 0.0;
    int s_ax = 0, s_dir = 0;
    bool halt = false;
    if (active) {
      R dr = L.g.chord(ax);
      bool pos = L.g.positive(dr, ax);
      if constexpr (HALT) {
        // the ray reaches its halting radius inside this cell: the segment ends there
        if (L.g.exit64(ax) > L.rhalt) {
          halt = true;
          dr = (R)(L.rhalt - L.g.radius64());
          pos = dr > (R)0;
        }
      }
      if (THIN && pos && thin_here) {
        // thin: no photons removed
        if (T.holds_source(L)) {
          double Pc = L.P;
          dval = absorb(Pc, L.kap * L.sigma * dr);
          if constexpr (COVER) {
            if (L.cover) dval *= T.covering_factor(L, (double)dr);
          }
          dkey = L.slot0 + L.astride * (uint32_t)L.lin + 1u;
          dep = true;
        } else if (sizeof(R) == 4 || (double)dr > L.g.exit64(ax) * 0x1p-40) {
          // the tree's mark on the cell: a plain byte store (every thin ray
          // of the tree that crosses the cell stores the same 1); a segment
          // shorter than 2^-40 of its exit radius (a ray through an edge or
          // a corner) does not cross the cell, which the float path's
          // plane-tie test already decides
          a.mark[L.mark_base + (long long)L.lin] = 1;
        }
        L.rem -= tc64;
        L.segs++;
        L.tsegs++;
        L.g.advance(ax);
      } else if (pos) {
        const R tau = L.kap * L.sigma * dr;
        dval = absorb(L.P, tau);
        if constexpr (THIN) L.thin = false;
        if constexpr (RADP) {
          // the absorbed radiation itself, before any covering-factor scaling
          mval = dval * L.mscale;
        }
        if constexpr (COVER) {
          if (L.cover) dval *= T.covering_factor(L, (double)dr);
        }
        dkey = (RADP || THIN) ? L.slot0 + L.astride * (uint32_t)L.lin : L.slot0 + (uint32_t)L.lin;
        dep = true;
        L.segs++;
        if (HALT && halt) L.g.set_radius(L.rhalt);
        else L.g.advance(ax);
      }
    }
    if (active && !(HALT && halt)) {
      // step across the exit face
      const int dir = e_dir;
      const int cnew = e_cnew;
      L.c0 = ax == 0 ? cnew : L.c0;
      L.c1 = ax == 1 ? cnew : L.c1;
      L.c2 = ax == 2 ? cnew : L.c2;
      L.lin = e_lin;
      L.g.step(ax, cnew);
      if (L.P < L.pmin) {
        ended = 1;
        active = false;
      } else if (++steps > max_steps_v) {
        // cell indices move monotonically, so this bound is never reached by a correct trace
        atomicOr(&a.ctr->err, kErrInternal);
        ended = 0;
        active = false;
      } else {
        s_ax = ax;
        s_dir = dir;
        moved = true;
      }
    }
    if constexpr (HALT) {
      // halted rays of the wave take consecutive records of its reserved
      // block of the halt list, and of a new block (one atomic per
      // kHaltBlock records) once that is full: a counter every wave of the
      // device shares is not touched at every halt
      const unsigned long long hm = __ballot(halt);
      if (hm) {
        const unsigned long long n = (unsigned long long)__popcll(hm);
        const unsigned long long room = h_end - h_next;
        unsigned long long nb = 0;
        if (n > room) {
          if (lane == 0) nb = atomicAdd(&a.ctr->halt_count, (unsigned long long)kHaltBlock);
          nb = bcast64(nb, 0);
        }
        if (halt) {
          const unsigned long long rank = (unsigned long long)__popcll(hm & below);
          const unsigned long long i = rank < room ? h_next + rank : nb + (rank - room);
          if (i < a.halt_cap) {
            a.halt.pix[i] = L.pix;
            a.halt.sg[i] = L.sg;
            a.halt.r[i] = dep ? L.rhalt : L.g.radius64();
            a.halt.P[i] = L.P;
            a.halt_lev[i] = a.gen;
          } else {
            atomicOr(&a.ctr->err, kErrOverflow);
          }
          ended = 3;
          active = false;
        }
        if (n > room) {
          h_next = nb + (n - room);
          h_end = nb + (unsigned long long)kHaltBlock;
        } else {
          h_next += n;
        }
        h_count += n;
      }
    }
    if constexpr (RADP) {
      // the momentum rate along the ray, from the float64 direction (zero
      // for a problem that does not ask for it: its key is a one-sum slot)
      double v[4] = {dval, 0.0, 0.0, 0.0};
      if (dep && mval != 0.0) {
        v[1] = mval * L.g.dir64(0);
        v[2] = mval * L.g.dir64(1);
        v[3] = mval * L.g.dir64(2);
      }
      cache.add(a.acc, dkey, v, dep, lane);
    } else {
      cache.add(a.acc, dkey, dval, dep, lane);
    }
    // the gathered column is taken on every path, so that no load is in
    // flight across the loop's back edge
    // the gather completes here, on every path: left in flight across the
    // loop's back edge it would make the compiler drain the whole counter
    if constexpr (K64) {
      asm volatile("" ::"v"(kpre64));
      kpre = (R)kpre64;
    } else {
      asm volatile("" ::"v"(kpre));
    }
    const bool kneg = moved && (!e_in || kpre < (R)0);
    L.kap = (moved && !kneg) ? kpre : L.kap;
    if constexpr (THIN) L.kap64 = (moved && !kneg) ? (K64 ? kpre64 : (double)kpre) : L.kap64;
    if (kneg && !T.settle(L, s_ax, s_dir)) {
      ended = 0;
      active = false;
    }
    if constexpr (K64) {
      if (kneg && active) {
        L.kap64 = a.kappa64[L.lin];
        finish_vector_loads();
      }
    } else if constexpr (THIN) {
      if (kneg) L.kap64 = (double)L.kap;
    }
    // bulk writes, only when a buffer is nearly full
    if (stage.count >= kStageFlush) stage.write(a, lane);
    if (cache.want_drain()) cache.drain(a.acc, lane);
  }
  if (stage.count) stage.write(a, lane);
  cache.flush(a.acc, lane);
  if (ended >= 0) {
    tally.add(a.stats, HALT ? L.sg % a.tree_fold : L.sg, L.segs, L.P, ended, THIN ? L.tsegs : 0u);
  }
  if constexpr (HALT) {
    // the unfilled rest of the wave's last block: empty records (no photons,
    // a level above every real one); the level's count once per wave
    for (unsigned long long i = h_next + lane; i < h_end; i += kWave)
      if (i < a.halt_cap) {
        a.halt.pix[i] = 0;
        a.halt.sg[i] = 0;
        a.halt.r[i] = 0.0;
        a.halt.P[i] = 0.0;
        a.halt_lev[i] = kHaltHole;
      }
    if (lane == 0 && h_count) atomicAdd(&a.ctr->halt_levels[a.gen], h_count);
  }
  // unused slots of the wave's last reserved block become empty slots
  stage.close(a, lane);
  __syncthreads();
  tally.flush(a.stats);
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

__global__ void reset_kernel(Counters* ctr, SgStats* stats, int n_sg) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kLevels * kSegMax) {
    (&ctr->count[0][0])[i] = 0;
    (&ctr->head[0][0])[i] = 0;
  }
  if (i == 0) {
    ctr->lost_rays = 0; ctr->lost_P = 0.0; ctr->err = 0;
  }
  if (i < kLevels) ctr->halt_levels[i] = 0;
  if (i == 0) ctr->halt_count = 0;
  if (i < n_sg) stats[i] = SgStats{0.0, 0.0, 0ull, 0ull, 0ull, 0ull};
}

__global__ void reset_levels_kernel(Counters* ctr) {
  for (int i = threadIdx.x; i < kLevels * kSegMax; i += blockDim.x) {
    (&ctr->count[0][0])[i] = 0;
    (&ctr->head[0][0])[i] = 0;
  }
}

// Before a launch of the serving engine: the input queue's claim counters and
// the output queue's write counters start at zero; earlier overflow flags are
// cleared (the host has read them).
__global__ void reset_generation_kernel(Counters* ctr, int cin, int cout) {
  for (int s = threadIdx.x; s < kSegMax; s += blockDim.x) {
    ctr->head[cin][s] = 0;
    ctr->count[cout][s] = 0;
  }
  if (threadIdx.x == 0) {
    ctr->err &= ~kErrOverflow;
    ctr->lost_rays = 0;
    ctr->lost_P = 0.0;
  }
}

__global__ void reset_stats_kernel(SgStats* stats, int first, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) stats[first + i] = SgStats{0.0, 0.0, 0ull, 0ull, 0ull, 0ull};
}

// Absorber column per root-cell length, input checks, zeroed accumulators.
// `grids` holds the n_grids grids (grid-table indices grid_base...) whose
// cells fill [cell_begin, cell_end) of the batch-wide numbering.
template <typename R>
__global__ void prep_kernel(const GridDev* grids, int n_grids, int grid_base, const ProblemDev* probs,
                            long long cell_begin, long long cell_end, R* kappa, double* acc, Counters* ctr,
                            uint8_t* mark, double* kappa64) {
  for (long long c = cell_begin + blockIdx.x * (long long)blockDim.x + threadIdx.x; c < cell_end;
       c += (long long)gridDim.x * blockDim.x) {
    const int g = grid_of(grids, n_grids, c);
    const GridDev& G = grids[g];
    const ProblemDev& P = probs[G.problem];
    const long long local = c - G.cell_off;
    const float nh = G.n_h[local], xh = G.x_hi[local];
    if (!(nh >= 0.0f) || !(xh >= 0.0f) || !(xh <= 1.0f) || !isfinite(nh)) atomicOr(&ctr->err, kErrBadInput);
    const double dx_root = G.is_child ? 2.0 * G.dx_cm : G.dx_cm;
    double k64 = (double)nh * (double)xh * dx_root;
    // children follow their root in the grid table
    if (!G.is_child && g + 1 < n_grids && grids[g + 1].is_child && grids[g + 1].problem == G.problem) {
      // a root cell under a child grid carries -(child + 1)
      const int i = (int)(local % G.nx), j = (int)((local / G.nx) % G.ny), kk = (int)(local / ((long long)G.nx * G.ny));
      for (int q = g + 1; q < n_grids && grids[q].is_child && grids[q].problem == G.problem; ++q) {
        const GridDev& C = grids[q];
        if (i >= C.ox && i < C.ox + C.nx / 2 && j >= C.oy && j < C.oy + C.ny / 2 && kk >= C.oz && kk < C.oz + C.nz / 2)
          k64 = (double)(-(grid_base + q + 1));
      }
    }
    kappa[c] = (R)k64;
    if (kappa64) kappa64[c] = k64;
    const long long base = P.acc_off + P.acc_stride * (c - P.cell_off), gstride = P.acc_stride * P.n_cells;
    for (int gr = 0; gr < P.n_groups; ++gr)
      for (int k = 0; k < P.acc_stride; ++k) acc[base + gr * gstride + k] = 0.0;
    for (int t = 0; t < P.mark_trees; ++t) mark[P.mark_off + t * P.n_cells + (c - P.cell_off)] = 0;
  }
}

// k_ph = sum_g absorbed_g / (n_H x_HI V); heating = sum_g absorbed_g (E_g - E_ion) / (n_H x_HI V);
// with radiation pressure, accel = (absorbed momentum rate) / (m_H n_H V) per component;
// with the optically-thin approximation, the thin deposits in cells that hold a source join the
// absorbed sums of k_ph and heating (not the absorbed total), and every tree marked on the cell
// adds its rate thin_coef / r^2 (r from its source to the cell centre, root cells) to k_ph and
// that times (E_g - E_ion) to the heating (section 2.4, Eq. optthin), whatever n_H x_HI is;
// per-block sums of the absorbed rate (no atomics).
__global__ __launch_bounds__(kFinalBlock) void finalize_kernel(const GridDev* grids, const ProblemDev* probs,
                                                               const FinalBlock* blocks, const double* acc,
                                                               const double* eexc, double* partial,
                                                               const Counters* ctr, const SgDev* sgs,
                                                               const uint8_t* mark) {
  __shared__ double red[kFinalBlock / kWave];
  if (ctr->err & kErrBadInput) return;
  const FinalBlock B = blocks[blockIdx.x];
  const GridDev& G = grids[B.grid];
  const ProblemDev& P = probs[G.problem];
  const double vol = G.dx_cm * G.dx_cm * G.dx_cm;
  double sum = 0.0;
  for (int t = threadIdx.x; t < B.count; t += kFinalBlock) {
    const long long local = B.first + t;
    const long long c = G.cell_off + local;
    const long long base = P.acc_off + P.acc_stride * (c - P.cell_off), gstride = P.acc_stride * P.n_cells;
    double ab = 0.0, he = 0.0, tab = 0.0, the = 0.0;
    double mom[3] = {0.0, 0.0, 0.0};
    for (int gr = 0; gr < P.n_groups; ++gr) {
      const double v = acc[base + gr * gstride];
      ab += v;
      he += v * eexc[P.eexc_off + gr];
      if (P.acc_stride == 2) {
        const double w = acc[base + gr * gstride + 1];
        tab += w;
        the += w * eexc[P.eexc_off + gr];
      }
      if (P.acc_stride == 4)
        for (int d = 0; d < 3; ++d) mom[d] += acc[base + gr * gstride + 1 + d];
    }
    double kt = 0.0, ht = 0.0;
    if (P.mark_trees > 0) {
      const int i = (int)(local % G.nx), j = (int)((local / G.nx) % G.ny);
      const int kk = (int)(local / ((long long)G.nx * G.ny));
      const double cx = G.is_child ? (double)G.ox + 0.5 * ((double)i + 0.5) : (double)i + 0.5;
      const double cy = G.is_child ? (double)G.oy + 0.5 * ((double)j + 0.5) : (double)j + 0.5;
      const double cz = G.is_child ? (double)G.oz + 0.5 * ((double)kk + 0.5) : (double)kk + 0.5;
      for (int t = 0; t < P.mark_trees; ++t) {
        if (!mark[P.mark_off + t * P.n_cells + (c - P.cell_off)]) continue;
        const SgDev& S = sgs[P.sg_first + t];
        const double dx0 = cx - S.sx, dx1 = cy - S.sy, dx2 = cz - S.sz;
        const double kv = S.thin_coef / (dx0 * dx0 + dx1 * dx1 + dx2 * dx2);
        kt += kv;
        ht += kv * eexc[P.eexc_off + t % P.n_groups];
      }
    }
    const double nabs = (double)G.n_h[local] * (double)G.x_hi[local];
    double k = kt, h = ht;
    if (nabs > 0.0) {
      k = (ab + tab) / (nabs * vol) + kt;
      h = (he + the) / (nabs * vol) + ht;
    }
    G.out_kph[local] = k;
    G.out_heat[local] = h;
    if (P.acc_stride == 4 && G.out_acc) {
      const double rho = kHydrogenMassG * (double)G.n_h[local];
      for (int d = 0; d < 3; ++d) G.out_acc[d * P.n_cells + local] = rho > 0.0 ? mom[d] / (rho * vol) : 0.0;
    }
    sum += ab;
  }
  for (int off = kWave / 2; off > 0; off >>= 1) sum += __shfl_down(sum, off);
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kFinalBlock / kWave; ++w) s += red[w];
    partial[blockIdx.x] = s;
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers (called by the runtime on its stream).
// ---------------------------------------------------------------------------
hipError_t launch_reset(hipStream_t s, Counters* ctr, SgStats* stats, int n_sg) {
  const int n = n_sg > kLevels * kSegMax ? n_sg : kLevels * kSegMax;
  const int blocks = n / 256 + 1;
  hipLaunchKernelGGL(reset_kernel, dim3(blocks), dim3(256), 0, s, ctr, stats, n_sg);
  return hipGetLastError();
}

hipError_t launch_reset_generation(hipStream_t s, Counters* ctr, int cin, int cout) {
  hipLaunchKernelGGL(reset_generation_kernel, dim3(1), dim3(kSegMax), 0, s, ctr, cin, cout);
  return hipGetLastError();
}

hipError_t launch_reset_stats(hipStream_t s, SgStats* stats, int first, int count) {
  if (count < 1) return hipSuccess;
  hipLaunchKernelGGL(reset_stats_kernel, dim3((count + 255) / 256), dim3(256), 0, s, stats, first, count);
  return hipGetLastError();
}

hipError_t launch_reset_levels(hipStream_t s, Counters* ctr) {
  hipLaunchKernelGGL(reset_levels_kernel, dim3(1), dim3(256), 0, s, ctr);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_prep(hipStream_t s, int num_cu, const GridDev* grids, int n_grids, int grid_base,
                       const ProblemDev* probs, long long cell_begin, long long cell_end, R* kappa, double* acc,
                       Counters* ctr, uint8_t* mark, double* kappa64) {
  long long blocks = (cell_end - cell_begin + 255) / 256;
  if (blocks > 32LL * num_cu) blocks = 32LL * num_cu;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(prep_kernel<R>, dim3((unsigned)blocks), dim3(256), 0, s, grids, n_grids, grid_base, probs,
                     cell_begin, cell_end, kappa, acc, ctr, mark, kappa64);
  return hipGetLastError();
}

// Blocks per CU a kernel can keep resident (looked up once per kernel).
template <typename K>
static int resident_blocks(K kernel, int& memo) {
  if (memo <= 0) {
    int n = 0;
    memo = (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, kTraceBlock, 0) == hipSuccess && n > 0) ? n : 1;
  }
  return memo;
}

// `blocks` is sized for the plain kernel's residency; a variant that keeps
// fewer blocks per CU resident (the radiation-pressure table takes more LDS)
// is launched with proportionally fewer, so its grid stays persistent.
template <typename R, int PHYS>
static void launch_phys(hipStream_t s, int blocks, const TraceArgs<R>& args, bool cache) {
  if (cache) {
    static int plain = 0, mine = 0;
    const int p = resident_blocks(trace_level_kernel<R, true, 0>, plain);
    const int m = resident_blocks(trace_level_kernel<R, true, PHYS>, mine);
    if (m < p) blocks = (blocks * m + p - 1) / p;
    hipLaunchKernelGGL((trace_level_kernel<R, true, PHYS>), dim3(blocks), dim3(kTraceBlock), 0, s, args);
  } else {
    hipLaunchKernelGGL((trace_level_kernel<R, false, PHYS>), dim3(blocks), dim3(kTraceBlock), 0, s, args);
  }
}

template <typename R>
hipError_t launch_trace_level(hipStream_t s, int blocks, const TraceArgs<R>& args, bool cache, bool cover,
                              bool radp, bool thin) {
  if (thin && radp) return hipErrorInvalidValue;
  if (thin && cover) launch_phys<R, kPhysThin | kPhysCover>(s, blocks, args, cache);
  else if (thin) launch_phys<R, kPhysThin>(s, blocks, args, cache);
  else if (cover && radp) launch_phys<R, kPhysCover | kPhysRadp>(s, blocks, args, cache);
  else if (cover) launch_phys<R, kPhysCover>(s, blocks, args, cache);
  else if (radp) launch_phys<R, kPhysRadp>(s, blocks, args, cache);
  else launch_phys<R, 0>(s, blocks, args, cache);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_trace_level_halt(hipStream_t s, int blocks, const TraceArgs<R>& args, bool cache) {
  launch_phys<R, kPhysHalt>(s, blocks, args, cache);
  return hipGetLastError();
}

// Time-dependent rays: the rays of HEALPix level `level` among the n_pool
// rays halted in the previous step join level queue q (counter row `row`).
// Each wave pass takes 64 records and puts its matching ones, with one
// atomic, at the end of one of the queue's nseg segments (a power of two),
// chosen by the pass; a segment that is full flags an overflow.
__global__ __launch_bounds__(256) void prefill_level_kernel(RayQueue pool, const int* __restrict__ pool_lev,
                                                            unsigned long long n_pool, int level, RayQueue q,
                                                            unsigned long long seg_cap, int nseg, Counters* ctr,
                                                            int row) {
  const int lane = threadIdx.x & (kWave - 1);
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const unsigned long long waves = (unsigned long long)gridDim.x * (blockDim.x / kWave);
  const unsigned long long wave = blockIdx.x * (unsigned long long)(blockDim.x / kWave) + threadIdx.x / kWave;
  for (unsigned long long w = wave; w * kWave < n_pool; w += waves) {
    const unsigned long long i = w * kWave + lane;
    const bool mine = i < n_pool && pool_lev[i] == level;
    const unsigned long long m = __ballot(mine);
    if (!m) continue;
    const int seg = (int)(w & (unsigned long long)(nseg - 1));
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(&ctr->count[row][seg], (unsigned long long)__popcll(m));
    base = bcast64(base, 0);
    if (mine) {
      const unsigned long long pos = base + __popcll(m & below);
      if (pos < seg_cap) {
        const unsigned long long o = (unsigned long long)seg * seg_cap + pos;
        q.pix[o] = pool.pix[i];
        q.sg[o] = pool.sg[i];
        q.r[o] = pool.r[i];
        q.P[o] = pool.P[i];
      } else {
        atomicOr(&ctr->err, kErrOverflow);
      }
    }
  }
}

// Serving: rays of removed problems leave the queue between two launches.
// Block b walks segment b % nseg (blocks share a segment by their quotient)
// over its written slots and empties every record whose tree index lies in
// one of the n ranges [lo[i], hi[i]).
struct DropRanges {
  int n;
  int lo[kDropRanges], hi[kDropRanges];
};

__global__ __launch_bounds__(256) void drop_trees_kernel(uint32_t* __restrict__ sg, const Counters* __restrict__ ctr,
                                                         int row, unsigned long long seg_cap, int nseg, DropRanges r) {
  const int seg = (int)(blockIdx.x % (unsigned)nseg);
  const unsigned long long part = blockIdx.x / (unsigned)nseg, parts = gridDim.x / (unsigned)nseg;
  const unsigned long long cnt = ctr->count[row][seg] < seg_cap ? ctr->count[row][seg] : seg_cap;
  uint32_t* q = sg + (unsigned long long)seg * seg_cap;
  for (unsigned long long i = part * 256ull + threadIdx.x; i < cnt; i += parts * 256ull) {
    const uint32_t t = q[i];
    bool drop = false;
    for (int k = 0; k < r.n; ++k) drop = drop || ((int)t >= r.lo[k] && (int)t < r.hi[k]);
    if (t != kNoTree && drop) q[i] = kNoTree;
  }
}

// Per-block sums of v[0..n) (the photons the halted rays hold).
__global__ __launch_bounds__(256) void sum_blocks_kernel(const double* __restrict__ v, unsigned long long n,
                                                         double* __restrict__ part) {
  __shared__ double red[256 / kWave];
  double s = 0.0;
  for (unsigned long long i = blockIdx.x * 256ull + threadIdx.x; i < n; i += (unsigned long long)gridDim.x * 256ull)
    s += v[i];
  for (int off = kWave / 2; off > 0; off >>= 1) s += __shfl_down(s, off);
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < 256 / kWave; ++w) t += red[w];
    part[blockIdx.x] = t;
  }
}

hipError_t launch_sum_blocks(hipStream_t s, int blocks, const double* v, unsigned long long n, double* part) {
  hipLaunchKernelGGL(sum_blocks_kernel, dim3(blocks), dim3(256), 0, s, v, n, part);
  return hipGetLastError();
}

hipError_t launch_drop_trees(hipStream_t s, uint32_t* sg, const Counters* ctr, int row, unsigned long long seg_cap,
                             int nseg, const int* lo, const int* hi, int n) {
  if (n <= 0) return hipSuccess;
  if (n > kDropRanges || nseg < 1) return hipErrorInvalidValue;
  DropRanges r{};
  r.n = n;
  for (int k = 0; k < n; ++k) {
    r.lo[k] = lo[k];
    r.hi[k] = hi[k];
  }
  hipLaunchKernelGGL(drop_trees_kernel, dim3((unsigned)nseg * 16u), dim3(256), 0, s, sg, ctr, row, seg_cap, nseg, r);
  return hipGetLastError();
}

hipError_t launch_prefill_level(hipStream_t s, int num_cu, const RayQueue& pool, const int* pool_lev,
                                unsigned long long n_pool, int level, const RayQueue& q, unsigned long long seg_cap,
                                int nseg, Counters* ctr, int row) {
  if (n_pool == 0) return hipSuccess;
  unsigned long long blocks = (n_pool + 255) / 256;
  if (blocks > 16ull * (unsigned long long)num_cu) blocks = 16ull * (unsigned long long)num_cu;
  hipLaunchKernelGGL(prefill_level_kernel, dim3((unsigned)blocks), dim3(256), 0, s, pool, pool_lev, n_pool, level, q,
                     seg_cap, nseg, ctr, row);
  return hipGetLastError();
}

hipError_t launch_finalize(hipStream_t s, int n_blocks, const GridDev* grids, const ProblemDev* probs,
                           const FinalBlock* blocks, const double* acc, const double* eexc, double* partial,
                           const Counters* ctr, const SgDev* sgs, const uint8_t* mark) {
  if (n_blocks < 1) return hipSuccess;
  hipLaunchKernelGGL(finalize_kernel, dim3(n_blocks), dim3(kFinalBlock), 0, s, grids, probs, blocks, acc, eexc,
                     partial, ctr, sgs, mark);
  return hipGetLastError();
}

template hipError_t launch_prep<float>(hipStream_t, int, const GridDev*, int, int, const ProblemDev*, long long,
                                       long long, float*, double*, Counters*, uint8_t*, double*);
template hipError_t launch_prep<double>(hipStream_t, int, const GridDev*, int, int, const ProblemDev*, long long,
                                        long long, double*, double*, Counters*, uint8_t*, double*);
template hipError_t launch_trace_level<float>(hipStream_t, int, const TraceArgs<float>&, bool, bool, bool, bool);
template hipError_t launch_trace_level<double>(hipStream_t, int, const TraceArgs<double>&, bool, bool, bool, bool);
template hipError_t launch_trace_level_halt<float>(hipStream_t, int, const TraceArgs<float>&, bool);
template hipError_t launch_trace_level_halt<double>(hipStream_t, int, const TraceArgs<double>&, bool);

hipError_t trace_occupancy(int precision, bool cache, int* blocks_per_cu) {
  if (precision == 0)
    return cache ? hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, trace_level_kernel<double, true, 0>, kTraceBlock, 0)
                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, trace_level_kernel<double, false, 0>, kTraceBlock, 0);
  return cache ? hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, trace_level_kernel<float, true, 0>, kTraceBlock, 0)
               : hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, trace_level_kernel<float, false, 0>, kTraceBlock, 0);
}

}  // namespace moray
