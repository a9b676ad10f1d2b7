// model.hpp -- device-side physics of one transport step (toy electromagnetic
// shower in a slab calorimeter), random numbers and elementary functions.
//
// Everything here is __host__ __device__ so the same source can also be built
// for the host by the test harness; the library itself only runs it on gfx950.
//
// Units: mm, MeV.  The calorimeter has 50 layers along z, each a 2.3 mm absorber
// (X0 5.6 mm, dE/dx 1.27 MeV/mm) and a 5.7 mm gap (X0 140 mm, dE/dx 0.21
// MeV/mm), transverse half-width 200 mm.  Volume v = 2*layer + (v is a gap).
//
// Bitwise agreement with an independent CPU implementation needs: the same
// named algorithms for log/exp/sincos (atanh series, Taylor series, Cody-Waite
// reduction), IEEE correctly-rounded + - * / sqrt, no FMA contraction
// (-ffp-contract=off) and the same source-order evaluation.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define AD_HD __host__ __device__ __forceinline__

// Random-number blocks that several divergent paths of a step use are drawn once
// per step, by every lane, before the paths split: a wavefront then runs the
// Philox rounds once instead of once per path that any of its lanes takes.
// ADEPT_RNG_PER_PATH=1 builds the form that draws them on each path (same
// numbers, same results), to measure what the hoisting saves; 0 in normal builds.
#ifndef ADEPT_RNG_PER_PATH
#define ADEPT_RNG_PER_PATH 0
#endif

namespace adept {

enum : int { ELECTRON = 0, POSITRON = 1, GAMMA = 2 };
enum : int { LIM_RANGE = 0, LIM_PHYS = 1, LIM_GEOM = 2 };
constexpr int kNumVol = 100;
constexpr int kNumLayer = 50;
constexpr int kOutside = -1;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
// as 1, 2, 3", SC'11): 10 rounds of two 32x32->64 multiplies, the key bumped
// by the Weyl constants between rounds.
// ---------------------------------------------------------------------------
struct U4 {
  uint32_t x, y, z, w;
};

// Three-way XOR: one gfx950 v_bitop3_b32 (truth table 0x96, the parity of its
// three inputs) where the compiler would issue two v_xor_b32.
AD_HD uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
#if defined(__HIP_DEVICE_COMPILE__)
  uint32_t r;
  asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
#else
  return a ^ b ^ c;
#endif
}

// U: rounds per loop iteration (a divisor of 10), a tuning choice of the
// precision policy.  Fully unrolled, the round keys of each inlined call fold
// into distinct constants that crowd the scalar registers; a short loop keeps
// two of them.  The result does not depend on U.
template <int U = 10>
AD_HD U4 philox(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll U
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    // fully unrolled, the first round's counter words are often constants (block
    // index, zero) that plain XORs fold; the three-input form takes registers only
    const bool fold = U == 10 && r == 0;
    const uint32_t h1 = (uint32_t)(p1 >> 32), h0 = (uint32_t)(p0 >> 32);
    const U4 n = {fold ? (h1 ^ c.y ^ k0) : xor3(h1, c.y, k0), (uint32_t)p1, fold ? (h0 ^ c.w ^ k1) : xor3(h0, c.w, k1),
                  (uint32_t)p0};
    c = n;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// Block j of the stream of track (seed, id) at its own step n.
template <int U = 10>
AD_HD U4 track_block(uint32_t seed, uint64_t id, uint32_t n, uint32_t j) {
  return philox<U>(U4{n, j, (uint32_t)(id >> 32), 0u}, seed, (uint32_t)id);
}

// The k-th track created by (seed, id) at its step n: top bit set, the rest from
// the first two words of block 2 + k.
template <int U = 10>
AD_HD uint64_t child_id(uint32_t seed, uint64_t id, uint32_t n, uint32_t k) {
  const U4 r = track_block<U>(seed, id, n, 2u + k);
  return (1ull << 63) | ((uint64_t)(r.x & 0x7FFFFFFFu) << 32) | (uint64_t)r.y;
}

// Uniforms strictly inside (0, 1).
AD_HD double u01(uint32_t r) { return ((double)r + 0.5) * 0x1p-32; }
AD_HD float u01f(uint32_t r) { return ((float)(r >> 9) + 0.5f) * 0x1p-23f; }

// ---------------------------------------------------------------------------
// Elementary functions, one template per format.
// ---------------------------------------------------------------------------
template <class R>
struct Fmt;

template <>
struct Fmt<double> {
  // Cody-Waite splits: ln 2 rounded to 42 significant bits and pi/2 to 33
  // bits, plus the nearest double of the remainder.
  static constexpr double ln2_hi = 0x1.62e42fefa38p-1, ln2_lo = 0x1.ef35793c7673p-45;
  static constexpr double pio2_hi = 0x1.921fb544p+0, pio2_lo = 0x1.0b4611a626331p-34;
  static constexpr double inv_ln2 = 1.4426950408889634, two_over_pi = 0.6366197723675814;
  static constexpr double sqrt_half = 0.7071067811865476, pi = 3.14159265358979323846;
  static constexpr int log_terms = 11, exp_terms = 13, trig_terms = 8;
  AD_HD static double frexp_(double x, int* e) { return frexp(x, e); }
  AD_HD static double ldexp_(double x, int e) { return ldexp(x, e); }
  AD_HD static double rint_(double x) { return rint(x); }
  AD_HD static double sqrt_(double x) { return sqrt(x); }
};

template <>
struct Fmt<float> {
  static constexpr float ln2_hi = 0x1.62e4p-1f, ln2_lo = 0x1.7f7d1cp-20f;
  static constexpr float pio2_hi = 0x1.922p+0f, pio2_lo = -0x1.2aeef4p-18f;
  static constexpr float inv_ln2 = 1.44269504f, two_over_pi = 0.636619772f;
  static constexpr float sqrt_half = 0.707106781f, pi = 3.14159265358979323846f;
  static constexpr int log_terms = 5, exp_terms = 7, trig_terms = 4;
  AD_HD static float frexp_(float x, int* e) { return frexpf(x, e); }
  AD_HD static float ldexp_(float x, int e) { return ldexpf(x, e); }
  AD_HD static float rint_(float x) { return rintf(x); }
  AD_HD static float sqrt_(float x) { return sqrtf(x); }
};

// 1 / (2j+1), 1 / j!, 1 / (2j)!, 1 / (2j+1)!: each rounded once from an exact
// integer denominator (all factorials used are below 2^53).
template <class R>
AD_HD R inv_odd(int j) {
  return (R)1 / (R)(2 * j + 1);
}
template <class R>
AD_HD R inv_fact(int j) {
  double f = 1.0;
  for (int i = 2; i <= j; ++i) f *= (double)i;
  return (R)1 / (R)f;
}

// log x: x = m 2^e with m in (sqrt(1/2), sqrt(2)]; log m = 2 f sum_j f^(2j)/(2j+1)
// with f = (m-1)/(m+1) (Horner in f^2); result e*ln2_hi + (e*ln2_lo + log m).
template <class R>
AD_HD R plog(R x) {
  using F = Fmt<R>;
  int e;
  R m = F::frexp_(x, &e);
  if (!(m > F::sqrt_half)) {
    m = m * (R)2;
    e = e - 1;
  }
  const R f = (m - (R)1) / (m + (R)1);
  const R s = f * f;
  R p = inv_odd<R>(F::log_terms);
#pragma unroll
  for (int j = F::log_terms - 1; j >= 0; --j) p = p * s + inv_odd<R>(j);
  const R lm = (f + f) * p;
  const R de = (R)e;
  return de * F::ln2_hi + (de * F::ln2_lo + lm);
}

// exp x: k = rint(x / ln 2); r = (x - k ln2_hi) - k ln2_lo; Taylor series of e^r
// in Horner form; scale by 2^k.
template <class R>
AD_HD R pexp(R x) {
  using F = Fmt<R>;
  const R k = F::rint_(x * F::inv_ln2);
  const R r = (x - k * F::ln2_hi) - k * F::ln2_lo;
  R p = inv_fact<R>(F::exp_terms);
#pragma unroll
  for (int j = F::exp_terms - 1; j >= 0; --j) p = p * r + inv_fact<R>(j);
  return F::ldexp_(p, (int)k);
}

// sin and cos for |x| <= 8: q = rint(x 2/pi); r reduced with the two-part pi/2;
// sin r = r * sum (-r^2)^j / (2j+1)!, cos r = sum (-r^2)^j / (2j)!; quadrant q mod 4.
template <class R>
AD_HD void psincos(R x, R* so, R* co) {
  using F = Fmt<R>;
  const R q = F::rint_(x * F::two_over_pi);
  const R r = (x - q * F::pio2_hi) - q * F::pio2_lo;
  const R z = r * r;
  R ps = inv_fact<R>(2 * F::trig_terms + 1);
  R pc = inv_fact<R>(2 * F::trig_terms);
#pragma unroll
  for (int j = F::trig_terms - 1; j >= 0; --j) {
    ps = ps * (-z) + inv_fact<R>(2 * j + 1);
    pc = pc * (-z) + inv_fact<R>(2 * j);
  }
  const R S = r * ps, C = pc;
  switch (((int)q) & 3) {
    case 0: *so = S; *co = C; break;
    case 1: *so = C; *co = -S; break;
    case 2: *so = -S; *co = -C; break;
    default: *so = -C; *co = S; break;
  }
}

template <class R>
AD_HD R rmax(R a, R b) {
  return a > b ? a : b;
}
template <class R>
AD_HD R rmin(R a, R b) {
  return a < b ? a : b;
}

// Knuth's TwoSum: s + e == a + b exactly.
template <class R>
AD_HD void two_sum(R a, R b, R* s, R* e) {
  const R t = a + b;
  const R bb = t - a;
  *e = (a - (t - bb)) + (b - bb);
  *s = t;
}

// ---------------------------------------------------------------------------
// Geometry
// ---------------------------------------------------------------------------
AD_HD double zlo(int v) {
  const int l = v >> 1;
  return (v & 1) ? 8.0 * (double)l + 2.3 : 8.0 * (double)l;
}
AD_HD double zhi(int v) {
  const int l = v >> 1;
  return (v & 1) ? 8.0 * (double)(l + 1) : 8.0 * (double)l + 2.3;
}

// Volume of a point known to be inside the calorimeter.
AD_HD int locate(double z) {
  const int l = (int)floor(z / 8.0);
  return 2 * l + (z >= 8.0 * (double)l + 2.3 ? 1 : 0);
}

AD_HD double axis_dist(double p, double d, double lo, double hi) {
  double t;
  if (d > 0.0) t = (hi - p) / d;
  else if (d < 0.0) t = (lo - p) / d;
  else t = __builtin_inf();
  return t > 0.0 ? t : 0.0;
}

// True if the transverse distance (num / d, num = plane - p) cannot be strictly
// below s: |num| > s |d| (1 + 2^-40) implies fl(num / d) > s whatever the
// roundings (each below 2^-53 relative), so the division can be skipped.
AD_HD bool cannot_beat(double p, double d, double s) {
  if (d == 0.0) return true;  // +inf never replaces
  const double num = d > 0.0 ? 200.0 - p : -200.0 - p;
  const double an = d > 0.0 ? num : -num;
  const double ad = d > 0.0 ? d : -d;
  return an > s * ad * (1.0 + 0x1p-40);
}

// Distance to the slab boundary; ties resolved z, then x, then y.  The x and y
// distances are only divided out when they might win (same result bit for bit
// as evaluating all three).
AD_HD double distance(const double p[3], const double d[3], int v, int* axis) {
  double s = axis_dist(p[2], d[2], zlo(v), zhi(v));
  int a = 2;
  if (!cannot_beat(p[0], d[0], s)) {
    const double tx = axis_dist(p[0], d[0], -200.0, 200.0);
    if (tx < s) { s = tx; a = 0; }
  }
  if (!cannot_beat(p[1], d[1], s)) {
    const double ty = axis_dist(p[1], d[1], -200.0, 200.0);
    if (ty < s) { s = ty; a = 1; }
  }
  *axis = a;
  return s;
}

// Snap the crossed coordinate to its plane; return the new volume or kOutside.
AD_HD int cross(double p[3], const double d[3], int v, int axis) {
  if (axis == 2) {
    if (d[2] > 0.0) {
      p[2] = zhi(v);
      return v + 1 > kNumVol - 1 ? kOutside : v + 1;
    }
    p[2] = zlo(v);
    return v - 1 < 0 ? kOutside : v - 1;
  }
  if (axis == 0) p[0] = d[0] > 0.0 ? 200.0 : -200.0;
  else p[1] = d[1] > 0.0 ? 200.0 : -200.0;
  return kOutside;
}

// ---------------------------------------------------------------------------
// Precision policies.  FP64: everything binary64.  Mixed: direction, energy and
// interaction length stored and stepped in binary32; position, boundary
// distance, limiter comparison, continuous-loss subtraction and all deposits in
// binary64.
// ---------------------------------------------------------------------------
struct PolicyF64 {
  using R = double;  // stepping / sampling / angle type
  static constexpr bool mixed = false;
  static constexpr int philox_unroll = 5;  // measured fastest for this policy
  // tracks a lane of the step kernel holds per tile (the parked outputs of the
  // first take LDS: 148 B per lane here, so the batched tally cache is kept small)
  AD_HD static constexpr int tracks_per_lane(int block) { return block >= 1024 ? 2 : 1; }
  static constexpr int tally_cache_bits = 9;
  AD_HD static R uni(uint32_t r) { return u01(r); }
};
struct PolicyMixed {
  using R = float;
  static constexpr bool mixed = true;
  static constexpr int philox_unroll = 10;
  AD_HD static constexpr int tracks_per_lane(int block) { return block >= 1024 ? 2 : 1; }
  static constexpr int tally_cache_bits = 11;
  AD_HD static R uni(uint32_t r) { return u01f(r); }
};

template <class R>
struct Consts;
template <>
struct Consts<double> {
  AD_HD static double x0(int m) { return m ? 140.0 : 5.6; }
  AD_HD static double dedx(int m) { return m ? 0.21 : 1.27; }
  AD_HD static double lpair(int m) { return m ? 180.0 : 7.2; }
  AD_HD static double lcomp(int m) { return m ? 280.0 : 11.2; }
  static constexpr double me = 0.511, pairth = 1.022, cut_e = 1.0, cut_g = 0.1, kmin = 1.0, msc = 13.6;
};
template <>
struct Consts<float> {
  AD_HD static float x0(int m) { return m ? 140.0f : 5.6f; }
  AD_HD static float dedx(int m) { return m ? 0.21f : 1.27f; }
  AD_HD static float lpair(int m) { return m ? 180.0f : 7.2f; }
  AD_HD static float lcomp(int m) { return m ? 280.0f : 11.2f; }
  static constexpr float me = 0.511f, pairth = 1.022f, cut_e = 1.0f, cut_g = 0.1f, kmin = 1.0f, msc = 13.6f;
};

// A track in registers.
template <class R>
struct Track {
  double pos[3];
  R dir[3];
  R E;
  R nl;
  uint64_t id;
  uint64_t parent;
  uint32_t seed;
  uint32_t ctr;
  int32_t vol;
  uint32_t event;
};

// Up to three tracks created by one step.  dsel: 0 = the stepping track's
// (post-step) direction, 1 = +d, 2 = -d (annihilation axis).  psel: 0 = parent
// is the stepping track, 1 = parent is the virtual positron vid.
template <class R>
struct Creations {
  int n;
  // per slot s, bits [8s, 8s+7): type (2 bits), dsel (2), psel (1), k (2);
  // bits [24, 26): k of the virtual positron
  uint32_t meta;
  R E[3];
  R d[3];

  AD_HD int type(int s) const { return (int)((meta >> (8 * s)) & 3u); }
  AD_HD int dsel(int s) const { return (int)((meta >> (8 * s + 2)) & 3u); }
  AD_HD int psel(int s) const { return (int)((meta >> (8 * s + 4)) & 1u); }
  AD_HD uint32_t kid(int s) const { return (meta >> (8 * s + 5)) & 3u; }
  AD_HD uint32_t vk() const { return (meta >> 24) & 3u; }

  // Append one creation (type, direction select, parent select, energy, index k
  // of the creation among its parent's creations at this step).  Slots are
  // addressed with constant indices only so the arrays stay in registers.
  AD_HD void push(int ty, int ds, int ps, R e, uint32_t k) {
    meta |= (uint32_t)(ty | (ds << 2) | (ps << 4) | (int)(k << 5)) << (8 * n);
#pragma unroll
    for (int s = 0; s < 3; ++s) E[s] = n == s ? e : E[s];  // value selects, no pointer selects
    n += 1;
  }
};

// Ids of creation slot i of a step of track (seed, id) at counter n: a slot
// whose parent is the stepping track has id child_id(seed, id, n, k); one whose
// parent is a virtual positron (created below the cut and annihilated at once)
// has parent vid = child_id(seed, id, n, vk) and id child_id(seed, vid, 0, k).
// Recomputed where the record is written instead of being carried in registers.
template <int U = 10, class R>
AD_HD uint64_t creation_parent(const Creations<R>& cr, int i, uint32_t seed, uint64_t id, uint32_t n) {
  return cr.psel(i) ? child_id<U>(seed, id, n, cr.vk()) : id;
}
template <int U = 10, class R>
AD_HD uint64_t creation_id(const Creations<R>& cr, int i, uint32_t seed, uint64_t parent, uint32_t n) {
  return child_id<U>(seed, parent, cr.psel(i) ? 0u : n, cr.kid(i));
}

// Deposits of one step, handed to the tally stage.
struct Deposits {
  double cont;       // continuous loss, pre-step volume, step midpoint
  double cut;        // local deposits (below-cut source or creations), pre-step volume, post-step point
  double escaped;
  double round;
  double mid[2];     // x, y of the step midpoint
};

// Creation path: structural id; sub-cut tracks deposit at once (a sub-cut
// positron annihilates immediately as a virtual track with counter 0).
template <class P>
struct Creator {
  using R = typename P::R;
  uint32_t seed;
  uint64_t id;
  uint32_t n;
  int k;
};

// Annihilation of positron X0 at rest; b is block 1 of X0's stream.
template <class P>
AD_HD void annihilate(const U4& b, const Creator<P>& X0, int* kidx, int psel, Creations<typename P::R>& out) {
  using R = typename P::R;
  using F = Fmt<R>;
  const R c = (R)2 * P::uni(b.y) - (R)1;
  const R st = F::sqrt_(rmax((R)0, (R)1 - c * c));
  const R ph = ((R)2 * F::pi) * P::uni(b.z);
  R sp, cp;
  psincos<R>(ph, &sp, &cp);
  out.d[0] = st * cp;
  out.d[1] = st * sp;
  out.d[2] = c;
  out.push(GAMMA, 1, psel, Consts<R>::me, (uint32_t)(*kidx)++);
  out.push(GAMMA, 2, psel, Consts<R>::me, (uint32_t)(*kidx)++);
}

template <class P>
AD_HD void create(const Creator<P>& X, int* kidx, int type, typename P::R E, Creations<typename P::R>& out,
                  Deposits& dep) {
  using R = typename P::R;
  const uint32_t k = (uint32_t)(*kidx)++;
  const bool subcut = type == GAMMA ? (E < Consts<R>::cut_g) : (E < Consts<R>::cut_e);
  if (subcut) {
    dep.cut += (double)E;
    if (type == POSITRON) {
      Creator<P> V{X.seed, child_id<P::philox_unroll>(X.seed, X.id, X.n, k), 0u, 0};
      int k2 = 0;
      out.meta |= k << 24;
      annihilate<P>(track_block<P::philox_unroll>(V.seed, V.id, V.n, 1u), V, &k2, 1, out);
    }
    return;
  }
  out.push(type, 0, 0, E, k);
}

// Rotation taking z-hat to u, applied to (dx, dy, dz); no renormalisation.
template <class R>
AD_HD void rotate(R u[3], R dx, R dy, R dz) {
  using F = Fmt<R>;
  const R ux = u[0], uy = u[1], uz = u[2];
  const R up = F::sqrt_(ux * ux + uy * uy);
  if (up > (R)0) {
    u[0] = (ux * uz * dx - uy * dy) / up + ux * dz;
    u[1] = (uy * uz * dx + ux * dy) / up + uy * dz;
    u[2] = -up * dx + uz * dz;
  } else if (uz > (R)0) {
    u[0] = dx; u[1] = dy; u[2] = dz;
  } else {
    u[0] = -dx; u[1] = dy; u[2] = -dz;
  }
}

// One step of an electron or positron.  Returns true if it survives.
template <class P>
AD_HD bool step_charged(Track<typename P::R>& t, int type, Creations<typename P::R>& out, Deposits& dep) {
  using R = typename P::R;
  using F = Fmt<R>;
  using C = Consts<R>;
  const uint32_t n = t.ctr;
  const U4 a = track_block<P::philox_unroll>(t.seed, t.id, n, 0u);
  const Creator<P> X{t.seed, t.id, n, 0};
  int kidx = 0;
  const int v = t.vol, m = v & 1;
  const R E0 = t.E;
  R nl = t.nl;
  if (nl < (R)0) nl = -plog<R>(P::uni(a.x));
  const R lam = C::x0(m);
  const R s_phys = nl * lam;
  const R s_range = E0 / C::dedx(m);
  double dd[3] = {(double)t.dir[0], (double)t.dir[1], (double)t.dir[2]};
  int axis;
  const double s_geom = distance(t.pos, dd, v, &axis);
  const double sp = (double)s_phys, sr = (double)s_range;
  int lim;
  double s;
  if (sr <= sp && sr <= s_geom) { lim = LIM_RANGE; s = sr; }
  else if (sp <= s_geom) { lim = LIM_PHYS; s = sp; }
  else { lim = LIM_GEOM; s = s_geom; }
  double p0[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    p0[i] = t.pos[i];
    t.pos[i] = p0[i] + s * dd[i];
  }
  const int v1 = lim == LIM_GEOM ? cross(t.pos, dd, v, axis) : v;
  R E1;
  if (P::mixed) {
    E1 = (lim == LIM_RANGE) ? (R)0 : (R)rmax((double)E0 - Consts<double>::dedx(m) * s, 0.0);
    double d, e;
    two_sum((double)E0, -(double)E1, &d, &e);
    dep.cont = d;
    dep.round += e;
  } else {
    E1 = (lim == LIM_RANGE) ? (R)0 : (R)rmax((double)E0 - Consts<double>::dedx(m) * s, 0.0);
    dep.cont = (double)E0 - (double)E1;
  }
  dep.mid[0] = 0.5 * (p0[0] + t.pos[0]);
  dep.mid[1] = 0.5 * (p0[1] + t.pos[1]);
  const R sr_ = (R)s;
  nl = (lim == LIM_PHYS) ? (R)0 : rmax(nl - sr_ / lam, (R)0);
  if (v1 == kOutside) {
    dep.escaped += (double)E1;
    if (type == POSITRON) dep.escaped += 2.0 * (double)C::me;
    return false;
  }
  // Block 1 serves the interaction-length resample after a brem and the
  // annihilation direction; one of the two occurs in nearly every wavefront, so
  // it is drawn once here rather than on each path.
#if !ADEPT_RNG_PER_PATH
  const U4 b = track_block<P::philox_unroll>(t.seed, t.id, n, 1u);
#endif
  if (E1 < C::cut_e) {
    dep.cut += (double)E1;
    t.vol = v1;
#if ADEPT_RNG_PER_PATH
    if (type == POSITRON) annihilate<P>(track_block<P::philox_unroll>(t.seed, t.id, n, 1u), X, &kidx, 0, out);
#else
    if (type == POSITRON) annihilate<P>(b, X, &kidx, 0, out);
#endif
    return false;
  }
  const R th0 = (C::msc / E0) * F::sqrt_(sr_ / lam);
  const R th = rmin(th0 * F::sqrt_((R)(-2) * plog<R>(P::uni(a.y))), F::pi);
  const R ph = ((R)2 * F::pi) * P::uni(a.z);
  R sth, cth, sph, cph;
  psincos<R>(th, &sth, &cth);
  psincos<R>(ph, &sph, &cph);
  rotate<R>(t.dir, sth * cph, sth * sph, cth);
  R E = E1;
  if (lim == LIM_PHYS) {
    R k = C::kmin * pexp<R>(P::uni(a.w) * plog<R>(E1 / C::kmin));
    k = rmin(rmax(k, C::kmin), E1);
    const R E2 = E1 - k;
    k = E1 - E2;
    create<P>(X, &kidx, GAMMA, k, out, dep);
#if ADEPT_RNG_PER_PATH
    const U4 b = track_block<P::philox_unroll>(t.seed, t.id, n, 1u);
#endif
    nl = -plog<R>(P::uni(b.x));
    E = E2;
    if (E2 < C::cut_e) {
      dep.cut += (double)E2;
      t.vol = v1;
      if (type == POSITRON) annihilate<P>(b, X, &kidx, 0, out);
      return false;
    }
  }
  t.E = E;
  t.nl = nl;
  t.vol = v1;
  t.ctr = n + 1;
  return true;
}

// One step of a photon.  Returns true if it survives.
template <class P>
AD_HD bool step_photon(Track<typename P::R>& t, Creations<typename P::R>& out, Deposits& dep) {
  using R = typename P::R;
  using C = Consts<R>;
  const uint32_t n = t.ctr;
  const Creator<P> X{t.seed, t.id, n, 0};
  int kidx = 0;
  const int v = t.vol, m = v & 1;
  const R E = t.E;
  R nl = t.nl;
  // Block 0 gives the initial interaction length and the interaction's split.
  // Almost every wavefront holds a new photon and an interacting one, so the
  // block is drawn once for all lanes instead of on each of the two paths.
#if ADEPT_RNG_PER_PATH
  if (nl < (R)0) nl = -plog<R>(P::uni(track_block<P::philox_unroll>(t.seed, t.id, n, 0u).x));
#else
  const U4 a = track_block<P::philox_unroll>(t.seed, t.id, n, 0u);
  if (nl < (R)0) nl = -plog<R>(P::uni(a.x));
#endif
  const bool pair = E > C::pairth;
  const R lam = pair ? C::lpair(m) : C::lcomp(m);
  const R s_phys = nl * lam;
  double dd[3] = {(double)t.dir[0], (double)t.dir[1], (double)t.dir[2]};
  int axis;
  const double s_geom = distance(t.pos, dd, v, &axis);
  const int lim = ((double)s_phys <= s_geom) ? LIM_PHYS : LIM_GEOM;
  const double s = lim == LIM_PHYS ? (double)s_phys : s_geom;
#pragma unroll
  for (int i = 0; i < 3; ++i) t.pos[i] = t.pos[i] + s * dd[i];
  const int v1 = lim == LIM_GEOM ? cross(t.pos, dd, v, axis) : v;
  nl = (lim == LIM_PHYS) ? (R)0 : rmax(nl - (R)s / lam, (R)0);
  if (v1 == kOutside) {
    dep.escaped += (double)E;
    return false;
  }
  t.vol = v1;
#if ADEPT_RNG_PER_PATH
  uint32_t a3 = 0;
  if (lim == LIM_PHYS) a3 = track_block<P::philox_unroll>(t.seed, t.id, n, 0u).w;
#else
  const uint32_t a3 = a.w;
#endif
  if (lim == LIM_PHYS && pair) {
    R T, r;
    two_sum<R>(E, -C::pairth, &T, &r);
    dep.round += (double)r;
    R Tm = P::uni(a3) * T;
    const R Tp = T - Tm;
    Tm = T - Tp;
    create<P>(X, &kidx, ELECTRON, Tm, out, dep);
    create<P>(X, &kidx, POSITRON, Tp, out, dep);
    return false;
  }
  R Enew = E;
  if (lim == LIM_PHYS) {
    const U4 b = track_block<P::philox_unroll>(t.seed, t.id, n, 1u);
    R T = P::uni(a3) * E;
    const R Ep = E - T;
    T = E - Ep;
    create<P>(X, &kidx, ELECTRON, T, out, dep);
    nl = -plog<R>(P::uni(b.x));
    Enew = Ep;
    if (Ep < C::cut_g) {
      dep.cut += (double)Ep;
      return false;
    }
  }
  t.E = Enew;
  t.nl = nl;
  t.ctr = n + 1;
  return true;
}

}  // namespace adept
