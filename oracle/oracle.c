/*
 * oracle.c -- plain CPU reference of the per-iteration track-transport step.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by tests/, by the smoke check and by the
 * CPU-baseline leg of the benchmark; never by the product path.  It is
 * deliberately slow and sequential: one iteration processes every active
 * track in the canonical order (all electrons, then positrons, then photons;
 * within a type in current-buffer order), appends each source's outputs in
 * order (survivor first, then its creations in creation order) and only then
 * builds the next iteration's buffers.  Tallies use Neumaier-compensated sums.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math (no FMA
 * contraction, IEEE binary64/binary32 arithmetic in source order).
 *
 * Model (units: mm, MeV):
 *  - calorimeter: 50 layers along z, each a 2.3 mm absorber (X0 5.6 mm,
 *    dE/dx 1.27 MeV/mm) followed by a 5.7 mm gap (X0 140 mm, dE/dx 0.21
 *    MeV/mm); transverse half-width 200 mm.  Volume v = 2*layer + (gap).
 *  - e+-: one interaction length ~ Exp(1) in units of the current material's
 *    X0 (bremsstrahlung); continuous loss dE/dx * step; Gaussian multiple
 *    scattering of projected width 13.6/E * sqrt(step/X0) (space angle
 *    Rayleigh-distributed, clamped at pi); bremsstrahlung photon energy
 *    k ~ 1/k on [1 MeV, E]; positrons annihilate at rest into two
 *    back-to-back 0.511 MeV photons.
 *  - photons: pair production (mean free path 9/7 X0) above 1.022 MeV, the
 *    kinetic energy split uniformly between e- and e+; otherwise Compton
 *    scattering (mean free path 2 X0) with energy transfer uniform in [0, E].
 *  - cuts: e+- below 1 MeV and photons below 0.1 MeV deposit locally.
 *  - randomness: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) keyed by
 *    (event seed, track id) with the track's own step count as counter.
 */
#include "oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Constants.  Binary64 values are the nearest doubles of the decimal         */
/* literals, binary32 values the nearest floats of the same literals.         */
/* ------------------------------------------------------------------------- */
#define NLAYER 50
#define NVOL 100
#define OUTSIDE (-1)

static const double kX0[2] = {5.6, 140.0};
static const double kDEDX[2] = {1.27, 0.21};
static const double kLPAIR[2] = {7.2, 180.0};   /* 9/7 X0 */
static const double kLCOMP[2] = {11.2, 280.0};  /* 2 X0 */
static const float kX0f[2] = {5.6f, 140.0f};
static const float kDEDXf[2] = {1.27f, 0.21f};
static const float kLPAIRf[2] = {7.2f, 180.0f};
static const float kLCOMPf[2] = {11.2f, 280.0f};
static const double kME = 0.511, kPAIRTH = 1.022, kCUTE = 1.0, kCUTG = 0.1, kKMIN = 1.0, kMSC = 13.6;
static const float kMEf = 0.511f, kPAIRTHf = 1.022f, kCUTEf = 1.0f, kCUTGf = 0.1f, kKMINf = 1.0f, kMSCf = 13.6f;
static const double kPI = 3.14159265358979323846;
static const float kPIf = 3.14159265358979323846f;
static const double kHALFW = 200.0;

/* Cody-Waite split constants.  LN2_HI: ln 2 rounded to 42 significant bits;
 * PIO2_HI: pi/2 rounded to 33 bits; the binary32 HI parts to 16 bits.  Each
 * LO part is the nearest value to (exact - HI). */
static const double kLN2_HI = 0x1.62e42fefa38p-1, kLN2_LO = 0x1.ef35793c7673p-45;
static const double kPIO2_HI = 0x1.921fb544p+0, kPIO2_LO = 0x1.0b4611a626331p-34;
static const double kINV_LN2 = 1.4426950408889634, kTWO_OVER_PI = 0.6366197723675814;
static const double kSQRT_HALF = 0.7071067811865476;
static const float kLN2_HIf = 0x1.62e4p-1f, kLN2_LOf = 0x1.7f7d1cp-20f;
static const float kPIO2_HIf = 0x1.922p+0f, kPIO2_LOf = -0x1.2aeef4p-18f;
static const float kINV_LN2f = 1.44269504f, kTWO_OVER_PIf = 0.636619772f, kSQRT_HALFf = 0.707106781f;

void or_constants(double *d, float *f) {
  d[0] = kLN2_HI; d[1] = kLN2_LO; d[2] = kPIO2_HI; d[3] = kPIO2_LO; d[4] = kINV_LN2;
  d[5] = kTWO_OVER_PI; d[6] = kSQRT_HALF; d[7] = kPI;
  f[0] = kLN2_HIf; f[1] = kLN2_LOf; f[2] = kPIO2_HIf; f[3] = kPIO2_LOf; f[4] = kINV_LN2f;
  f[5] = kTWO_OVER_PIf; f[6] = kSQRT_HALFf; f[7] = kPIf;
}

/* max/min as used throughout the model: (a > b) ? a : b and (a < b) ? a : b. */
static double dmax(double a, double b) { return a > b ? a : b; }
static double dmin(double a, double b) { return a < b ? a : b; }
static float fmaxx(float a, float b) { return a > b ? a : b; }
static float fminn(float a, float b) { return a < b ? a : b; }

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 and uniforms                                                  */
/* ------------------------------------------------------------------------- */
/* Ten rounds; round i uses key + i * (0x9E3779B9, 0xBB67AE85).  One round:
 * (hi0, lo0) = 0xD2511F53 * c0, (hi1, lo1) = 0xCD9E8D57 * c2 (64-bit products),
 * new counter = (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0). */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Block j of a track at its step n: counter (n, j, hi32(id), 0), key (seed, lo32(id)). */
static void track_block(uint32_t seed, uint64_t id, uint32_t n, uint32_t j, uint32_t out[4]) {
  uint32_t ctr[4] = {n, j, (uint32_t)(id >> 32), 0u};
  uint32_t key[2] = {seed, (uint32_t)id};
  or_philox4x32_10(ctr, key, out);
}

/* Uniform in (0,1): (r + 1/2) 2^-32 in binary64; (floor(r/2^9) + 1/2) 2^-23 in binary32. */
double or_u01(uint32_t r) { return ((double)r + 0.5) * 0x1p-32; }
float or_u01f(uint32_t r) { return ((float)(r >> 9) + 0.5f) * 0x1p-23f; }

/* Id of the k-th track created by a parent at its step n: 2^63 | ((r0 << 32 | r1) mod 2^63),
 * (r0, r1) the first two words of the parent's block 2 + k. */
uint64_t or_child_id(uint32_t seed, uint64_t parent_id, uint32_t n, uint32_t k) {
  uint32_t r[4];
  track_block(seed, parent_id, n, 2u + k, r);
  uint64_t v = ((uint64_t)r[0] << 32) | (uint64_t)r[1];
  return (UINT64_C(1) << 63) | (v & ((UINT64_C(1) << 63) - 1));
}

/* ------------------------------------------------------------------------- */
/* Elementary functions from named textbook methods (evaluated in source      */
/* order, no contraction), so that two independent implementations agree bit */
/* for bit.                                                                   */
/* ------------------------------------------------------------------------- */
/* log: x = m 2^e with m in (sqrt(1/2), sqrt(2)]; f = (m-1)/(m+1); log m = 2f * sum_{j=0..N}
 * f^(2j)/(2j+1) (the atanh series, Horner in f^2, N = 11 in binary64, 5 in binary32);
 * log x = e*LN2_HI + (e*LN2_LO + log m) (Cody-Waite). */
double or_log(double x) {
  int e;
  double m = frexp(x, &e); /* m in [0.5, 1) */
  if (!(m > kSQRT_HALF)) {
    m = m * 2.0;
    e = e - 1;
  }
  double f = (m - 1.0) / (m + 1.0);
  double s = f * f;
  double p = 1.0 / 23.0;
  for (int j = 10; j >= 0; --j) p = p * s + 1.0 / (double)(2 * j + 1);
  double lm = (f + f) * p;
  double de = (double)e;
  return de * kLN2_HI + (de * kLN2_LO + lm);
}

float or_logf(float x) {
  int e;
  float m = frexpf(x, &e);
  if (!(m > kSQRT_HALFf)) {
    m = m * 2.0f;
    e = e - 1;
  }
  float f = (m - 1.0f) / (m + 1.0f);
  float s = f * f;
  float p = 1.0f / 11.0f;
  for (int j = 4; j >= 0; --j) p = p * s + 1.0f / (float)(2 * j + 1);
  float lm = (f + f) * p;
  float fe = (float)e;
  return fe * kLN2_HIf + (fe * kLN2_LOf + lm);
}

/* exp: k = rint(x/ln 2) (ties to even); r = (x - k LN2_HI) - k LN2_LO;
 * exp r = sum_{j=0..N} r^j/j! (Horner, N = 13 / 7); result = exp(r) 2^k. */
double or_exp(double x) {
  double k = rint(x * kINV_LN2);
  double r = (x - k * kLN2_HI) - k * kLN2_LO;
  double fact[14];
  fact[0] = 1.0;
  for (int j = 1; j <= 13; ++j) fact[j] = fact[j - 1] * (double)j; /* exact up to 13! */
  double p = 1.0 / fact[13];
  for (int j = 12; j >= 0; --j) p = p * r + 1.0 / fact[j];
  return ldexp(p, (int)k);
}

float or_expf(float x) {
  float k = rintf(x * kINV_LN2f);
  float r = (x - k * kLN2_HIf) - k * kLN2_LOf;
  float fact[8];
  fact[0] = 1.0f;
  for (int j = 1; j <= 7; ++j) fact[j] = fact[j - 1] * (float)j;
  float p = 1.0f / fact[7];
  for (int j = 6; j >= 0; --j) p = p * r + 1.0f / fact[j];
  return ldexpf(p, (int)k);
}

/* sincos for |x| <= 8: q = rint(x 2/pi); r = (x - q PIO2_HI) - q PIO2_LO;
 * sin r = r * sum_{j=0..8} (-r^2)^j/(2j+1)!, cos r = sum_{j=0..8} (-r^2)^j/(2j)!
 * (binary32: j = 0..4); the quadrant q mod 4 selects (S,C), (C,-S), (-S,-C), (-C,S). */
void or_sincos(double x, double *so, double *co) {
  double q = rint(x * kTWO_OVER_PI);
  double r = (x - q * kPIO2_HI) - q * kPIO2_LO;
  double z = r * r;
  double fact[18];
  fact[0] = 1.0;
  for (int j = 1; j <= 17; ++j) fact[j] = fact[j - 1] * (double)j; /* exact up to 17! */
  double ps = 1.0 / fact[17];            /* j = 8, sign + */
  for (int j = 7; j >= 0; --j) ps = ps * (-z) + 1.0 / fact[2 * j + 1];
  double pc = 1.0 / fact[16];
  for (int j = 7; j >= 0; --j) pc = pc * (-z) + 1.0 / fact[2 * j];
  double S = r * ps, C = pc;
  int quad = ((int)q) & 3;
  switch (quad) {
    case 0: *so = S; *co = C; break;
    case 1: *so = C; *co = -S; break;
    case 2: *so = -S; *co = -C; break;
    default: *so = -C; *co = S; break;
  }
}

void or_sincosf(float x, float *so, float *co) {
  float q = rintf(x * kTWO_OVER_PIf);
  float r = (x - q * kPIO2_HIf) - q * kPIO2_LOf;
  float z = r * r;
  float fact[10];
  fact[0] = 1.0f;
  for (int j = 1; j <= 9; ++j) fact[j] = fact[j - 1] * (float)j;
  float ps = 1.0f / fact[9];
  for (int j = 3; j >= 0; --j) ps = ps * (-z) + 1.0f / fact[2 * j + 1];
  float pc = 1.0f / fact[8];
  for (int j = 3; j >= 0; --j) pc = pc * (-z) + 1.0f / fact[2 * j];
  float S = r * ps, C = pc;
  int quad = ((int)q) & 3;
  switch (quad) {
    case 0: *so = S; *co = C; break;
    case 1: *so = C; *co = -S; break;
    case 2: *so = -S; *co = -C; break;
    default: *so = -C; *co = S; break;
  }
}

/* Knuth's TwoSum: s + err == a + b exactly. */
static void two_sum(double a, double b, double *s, double *err) {
  double t = a + b;
  double bb = t - a;
  *err = (a - (t - bb)) + (b - bb);
  *s = t;
}
static void two_sumf(float a, float b, float *s, float *err) {
  float t = a + b;
  float bb = t - a;
  *err = (a - (t - bb)) + (b - bb);
  *s = t;
}

/* ------------------------------------------------------------------------- */
/* Geometry                                                                   */
/* ------------------------------------------------------------------------- */
static double plane_lo(int v) {
  int l = v >> 1;
  return (v & 1) ? 8.0 * (double)l + 2.3 : 8.0 * (double)l;
}
static double plane_hi(int v) {
  int l = v >> 1;
  return (v & 1) ? 8.0 * (double)(l + 1) : 8.0 * (double)l + 2.3;
}

/* Volume of a point: requires 0 <= z < 400 and |x|, |y| <= 200. */
int or_locate(const double pos[3], int32_t *volume) {
  if (!(pos[2] >= 0.0 && pos[2] < 400.0 && fabs(pos[0]) <= kHALFW && fabs(pos[1]) <= kHALFW)) return OR_E_INVALID;
  int l = (int)floor(pos[2] / 8.0);
  *volume = 2 * l + (pos[2] >= 8.0 * (double)l + 2.3 ? 1 : 0);
  return OR_OK;
}

/* Distance to the boundary of the current slab along dir.  Per axis: moving up,
 * (plane_hi - p)/d; moving down, (plane_lo - p)/d; not moving, +inf; each
 * clamped at 0.  The smallest wins with ties resolved z, then x, then y. */
double or_distance(const double p[3], const double d[3], int32_t v, int32_t *axis) {
  double t[3];
  const double lo[3] = {-kHALFW, -kHALFW, plane_lo(v)};
  const double hi[3] = {kHALFW, kHALFW, plane_hi(v)};
  for (int i = 0; i < 3; ++i) {
    double ti;
    if (d[i] > 0.0) ti = (hi[i] - p[i]) / d[i];
    else if (d[i] < 0.0) ti = (lo[i] - p[i]) / d[i];
    else ti = INFINITY;
    t[i] = ti > 0.0 ? ti : 0.0;
  }
  double s = t[2];
  int a = 2;
  if (t[0] < s) { s = t[0]; a = 0; }
  if (t[1] < s) { s = t[1]; a = 1; }
  *axis = a;
  return s;
}

/* Boundary crossing: the crossed coordinate is set to the plane value; a z
 * plane moves to the neighbouring volume, which is OUTSIDE beyond the ends;
 * a transverse plane leaves the calorimeter. */
static int cross(double p[3], const double d[3], int v, int axis) {
  if (axis == 2) {
    if (d[2] > 0.0) {
      p[2] = plane_hi(v);
      return v + 1 > NVOL - 1 ? OUTSIDE : v + 1;
    }
    p[2] = plane_lo(v);
    return v - 1 < 0 ? OUTSIDE : v - 1;
  }
  p[axis] = d[axis] > 0.0 ? kHALFW : -kHALFW;
  return OUTSIDE;
}

/* ------------------------------------------------------------------------- */
/* Layouts (paper Sec. 3-4): byte address of (slot, leaf) in one buffer.      */
/* ------------------------------------------------------------------------- */
/* Leaves: 0-2 pos, 3-5 dir, 6 E, 7 numIALeft, 8 trackId, 9 parentId, 10 rngSeed,
 * 11 rngCtr, 12 volume, 13 event. */
static const uint32_t kSizeD[14] = {8, 8, 8, 8, 8, 8, 8, 8, 8, 8, 4, 4, 4, 4};
static const uint32_t kSizeM[14] = {8, 8, 8, 4, 4, 4, 4, 4, 8, 8, 4, 4, 4, 4};
static const uint32_t kAosOffD[14] = {0, 8, 16, 24, 32, 40, 48, 56, 64, 72, 80, 84, 88, 92};
static const uint32_t kAosOffM[14] = {0, 8, 16, 24, 28, 32, 36, 40, 48, 56, 64, 68, 72, 76};

uint32_t or_leaf_size(int prec, int leaf) { return prec == OR_MIXED ? kSizeM[leaf] : kSizeD[leaf]; }

static uint64_t align256(uint64_t x) { return (x + 255u) & ~(uint64_t)255u; }

static uint64_t soa_start(int prec, uint64_t C, int leaf) {
  uint64_t a = 0;
  for (int j = 1; j <= leaf; ++j) a = align256(a + C * (uint64_t)or_leaf_size(prec, j - 1));
  return a;
}

/* AoS: slot*stride + offset (stride 96 binary64 record, 80 mixed record with 4
 * bytes of padding after numIALeft).  SoA: one array per leaf, each starting at
 * a 256-byte boundary.  AoSoA-N: blocks of N records, leaf-major inside a block
 * (Sec. 4: "AABBCC" for N = 2), unpadded record size R = 96 / 76. */
uint64_t or_leaf_addr(int mapping, uint32_t N, int prec, uint64_t C, uint64_t slot, int leaf) {
  uint32_t size = or_leaf_size(prec, leaf);
  if (mapping == OR_AOS) {
    uint64_t stride = prec == OR_MIXED ? 80 : 96;
    return slot * stride + (prec == OR_MIXED ? kAosOffM[leaf] : kAosOffD[leaf]);
  }
  if (mapping == OR_SOA) return soa_start(prec, C, leaf) + slot * size;
  uint64_t R = 0, pre = 0;
  for (int j = 0; j < 14; ++j) {
    if (j < leaf) pre += or_leaf_size(prec, j);
    R += or_leaf_size(prec, j);
  }
  return (slot / N) * (uint64_t)N * R + (uint64_t)N * pre + (slot % N) * size;
}

uint64_t or_buffer_bytes(int mapping, uint32_t N, int prec, uint64_t C) {
  if (mapping == OR_AOS) return C * (prec == OR_MIXED ? 80 : 96);
  if (mapping == OR_SOA) return align256(soa_start(prec, C, 13) + C * or_leaf_size(prec, 13));
  (void)N;
  return C * (prec == OR_MIXED ? 76 : 96);
}

/* ------------------------------------------------------------------------- */
/* Simulation state                                                           */
/* ------------------------------------------------------------------------- */
typedef struct { double s, c; } nsum; /* Neumaier compensated sum */
static void nadd(nsum *a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
  else a->c += (x - t) + a->s;
  a->s = t;
}
static double nval(const nsum *a) { return a->s + a->c; }

typedef struct {
  or_track trk;
  int type;
  int survivor;   /* 1: the source track itself */
  uint32_t slot;  /* sparse survivor: its slot */
} outrec;

struct or_sim {
  int scheme, prec;
  uint64_t C;
  uint32_t n_events;
  uint32_t *seeds;
  /* dense: two arrays per type, cur[t] selects the current one; sparse: slot array [t][0] */
  or_track *buf[3][2];
  uint64_t bufcap[3][2];
  int cur[3];
  uint64_t n[3];
  uint32_t *list_cur[3], *list_next[3];
  uint32_t *ring[3];
  uint64_t head[3], count[3];
  uint8_t *touched[3];
  /* tallies */
  nsum *cont, *cut, *escaped, *round, *ein, *cells;
  uint32_t nx, ny;
  double pitch;
  /* instrumentation */
  int instr_on;
  uint64_t instr_last;
  uint64_t rw[3][2][14][2];
  uint32_t *slotleaf[3][2];
  /* admission */
  int adm_on;
  double alpha, kappa[3];
  uint64_t hold;           /* iterations an admitted event keeps its projected peak reserved */
  uint64_t *ev_admit_iter; /* per staged event group: iterations done when it was admitted */
  uint64_t g_old;          /* first group whose reservation may still be held */
  double reserved[3];
  or_primary *staged;
  uint64_t n_staged;
  uint64_t *ev_first, *ev_count; /* per staged event group */
  double *ev_energy;
  uint32_t *ev_id;
  uint64_t n_groups, next_group;
  /* stats */
  uint64_t iter, steps[3], peak[3], slots_hw[3], error_iter;
  or_ledger led;
  int status;
  /* scratch outputs of one iteration */
  outrec *out;
  uint64_t n_out, cap_out;
  uint32_t *kills[3];
  uint64_t n_kills[3], cap_kills[3];
};

static int cells_on(const or_sim *S) { return S->cells != NULL; }

or_sim *or_create(int scheme, int prec, uint64_t C, uint32_t n_events, const uint32_t *seeds) {
  if ((scheme != OR_SPARSE && scheme != OR_DENSE) || (prec != OR_FP64 && prec != OR_MIXED)) return NULL;
  if (C == 0 || C > (UINT64_C(1) << 31) || n_events == 0) return NULL;
  or_sim *S = (or_sim *)calloc(1, sizeof(or_sim));
  if (!S) return NULL;
  S->scheme = scheme;
  S->prec = prec;
  S->C = C;
  S->n_events = n_events;
  S->seeds = (uint32_t *)malloc(sizeof(uint32_t) * n_events);
  memcpy(S->seeds, seeds, sizeof(uint32_t) * n_events);
  S->cont = (nsum *)calloc((size_t)n_events * NVOL, sizeof(nsum));
  S->cut = (nsum *)calloc((size_t)n_events * NVOL, sizeof(nsum));
  S->escaped = (nsum *)calloc(n_events, sizeof(nsum));
  S->round = (nsum *)calloc(n_events, sizeof(nsum));
  S->ein = (nsum *)calloc(n_events, sizeof(nsum));
  for (int t = 0; t < 3; ++t) {
    if (scheme == OR_SPARSE) {
      S->buf[t][0] = (or_track *)calloc(C, sizeof(or_track));
      S->bufcap[t][0] = C;
      S->list_cur[t] = (uint32_t *)malloc(sizeof(uint32_t) * C);
      S->list_next[t] = (uint32_t *)malloc(sizeof(uint32_t) * C);
      S->ring[t] = (uint32_t *)malloc(sizeof(uint32_t) * C);
      S->touched[t] = (uint8_t *)calloc(C, 1);
      if (!S->buf[t][0] || !S->list_cur[t] || !S->list_next[t] || !S->ring[t] || !S->touched[t]) {
        or_destroy(S);
        return NULL;
      }
      for (uint64_t i = 0; i < C; ++i) S->ring[t][i] = (uint32_t)i;
      S->head[t] = 0;
      S->count[t] = C;
    }
  }
  return S;
}

void or_destroy(or_sim *S) {
  if (!S) return;
  for (int t = 0; t < 3; ++t) {
    for (int b = 0; b < 2; ++b) {
      free(S->buf[t][b]);
      free(S->slotleaf[t][b]);
    }
    free(S->list_cur[t]);
    free(S->list_next[t]);
    free(S->ring[t]);
    free(S->touched[t]);
    free(S->kills[t]);
  }
  free(S->seeds);
  free(S->cont); free(S->cut); free(S->escaped); free(S->round); free(S->ein); free(S->cells);
  free(S->staged); free(S->ev_first); free(S->ev_count); free(S->ev_energy); free(S->ev_id);
  free(S->ev_admit_iter);
  free(S->out);
  free(S);
}

int or_set_scoring(or_sim *S, uint32_t nx, uint32_t ny, double pitch) {
  if (nx == 0 || ny == 0 || !(pitch > 0.0)) return OR_E_INVALID;
  free(S->cells);
  S->cells = (nsum *)calloc((size_t)NLAYER * nx * ny, sizeof(nsum));
  if (!S->cells) return OR_E_NOMEM;
  S->nx = nx; S->ny = ny; S->pitch = pitch;
  return OR_OK;
}

int or_set_instrumented(or_sim *S, int on, uint64_t last_iter) {
  S->instr_on = on;
  S->instr_last = last_iter;
  if (on) {
    for (int t = 0; t < 3; ++t)
      for (int b = 0; b < 2; ++b)
        if (!S->slotleaf[t][b] && (b == 0 || S->scheme == OR_DENSE)) {
          S->slotleaf[t][b] = (uint32_t *)calloc(S->C * 14, sizeof(uint32_t));
          if (!S->slotleaf[t][b]) return OR_E_NOMEM;
        }
  }
  return OR_OK;
}

int or_set_admission(or_sim *S, int on, double alpha, const double kappa[3], uint64_t hold_iters) {
  S->adm_on = on;
  S->alpha = alpha;
  S->hold = hold_iters;
  for (int t = 0; t < 3; ++t) S->kappa[t] = kappa[t];
  return OR_OK;
}

/* ---- instrumentation: counting is active for every operation that starts
 * while fewer than last_iter iterations are done (injection before the first
 * iteration is "iteration 0"). */
static int counting(const or_sim *S) { return S->instr_on && S->iter < S->instr_last; }

static void count_leaf(or_sim *S, int type, int b, uint64_t slot, int leaf, int write) {
  S->rw[type][b][leaf][write] += 1;
  S->slotleaf[type][b][slot * 14 + (uint64_t)leaf] += 1;
}
/* Every source track reads its 13 leaves other than parentId exactly once. */
static void count_source_reads(or_sim *S, int type, int b, uint64_t slot) {
  for (int l = 0; l < 14; ++l)
    if (l != 9) count_leaf(S, type, b, slot, l, 0);
}
static void count_full_write(or_sim *S, int type, int b, uint64_t slot) {
  for (int l = 0; l < 14; ++l) count_leaf(S, type, b, slot, l, 1);
}
/* Sparse survivor, written in place: e+-: pos, dir, E, numIALeft, rngCtr, volume;
 * photons: pos, E, numIALeft, rngCtr, volume. */
static void count_sparse_survivor(or_sim *S, int type, uint64_t slot) {
  static const int ch[10] = {0, 1, 2, 3, 4, 5, 6, 7, 11, 12};
  static const int ph[7] = {0, 1, 2, 6, 7, 11, 12};
  if (type == OR_GAMMA)
    for (int i = 0; i < 7; ++i) count_leaf(S, type, 0, slot, ph[i], 1);
  else
    for (int i = 0; i < 10; ++i) count_leaf(S, type, 0, slot, ch[i], 1);
}

/* ---- tallies */
static void cell_add(or_sim *S, int v, double x, double y, double e) {
  if (!cells_on(S)) return;
  double half = (0.5 * (double)S->nx) * S->pitch;
  double fx = floor((x + half) / S->pitch);
  double halfy = (0.5 * (double)S->ny) * S->pitch;
  double fy = floor((y + halfy) / S->pitch);
  uint32_t ix = fx < 0.0 ? 0u : (fx > (double)(S->nx - 1) ? S->nx - 1 : (uint32_t)fx);
  uint32_t iy = fy < 0.0 ? 0u : (fy > (double)(S->ny - 1) ? S->ny - 1 : (uint32_t)fy);
  nadd(&S->cells[((uint64_t)(v >> 1) * S->nx + ix) * S->ny + iy], e);
}
static void tally_cont(or_sim *S, uint32_t ev, int v, double e, const double mid[3]) {
  nadd(&S->cont[(uint64_t)ev * NVOL + (uint64_t)v], e);
  cell_add(S, v, mid[0], mid[1], e);
}
static void tally_cut(or_sim *S, uint32_t ev, int v, double e, const double at[3]) {
  nadd(&S->cut[(uint64_t)ev * NVOL + (uint64_t)v], e);
  cell_add(S, v, at[0], at[1], e);
}

/* ---- outputs of one step */
typedef struct {
  int n;
  int type[3];
  or_track trk[3];
} creations;

typedef struct {
  uint32_t seed, event;
  uint64_t id;
  uint32_t n;  /* step counter of the creator at this step */
  int k;       /* next creation index */
} creator;

static void annihilate(or_sim *S, creator *X, const double pos[3], int v, creations *out);

/* Creation path: the k-th creation of X gets its structural id; sub-cut tracks
 * deposit locally (a sub-cut positron annihilates at once as a virtual track
 * with that id and counter 0); all others are buffered with numIALeft unset. */
static void create(or_sim *S, creator *X, int type, double E, const double pos[3], const double dir[3], int v,
                   creations *out) {
  uint64_t id = or_child_id(X->seed, X->id, X->n, (uint32_t)X->k);
  X->k += 1;
  int subcut;
  if (S->prec == OR_MIXED) subcut = (type == OR_GAMMA) ? ((float)E < kCUTGf) : ((float)E < kCUTEf);
  else subcut = (type == OR_GAMMA) ? (E < kCUTG) : (E < kCUTE);
  S->led.created[type] += 1;
  if (subcut) {
    tally_cut(S, X->event, v, E, pos);
    if (type == OR_POSITRON) {
      S->led.annihilated += 1;
      creator V = {X->seed, X->event, id, 0u, 0};
      annihilate(S, &V, pos, v, out);
    } else {
      S->led.cut[type] += 1;
    }
    return;
  }
  or_track *t = &out->trk[out->n];
  out->type[out->n] = type;
  out->n += 1;
  for (int i = 0; i < 3; ++i) {
    t->pos[i] = pos[i];
    t->dir[i] = dir[i];
  }
  t->E = E;
  t->numIALeft = -1.0;
  t->trackId = id;
  t->parentId = X->id;
  t->rngSeed = X->seed;
  t->rngCtr = 0;
  t->volume = v;
  t->event = X->event;
}

/* Annihilation at rest of X at its step n: cos(theta) = 2U(b1) - 1, phi = 2 pi U(b2),
 * d = (sin theta cos phi, sin theta sin phi, cos theta); photons of m_e along +d, then -d. */
static void annihilate(or_sim *S, creator *X, const double pos[3], int v, creations *out) {
  S->led.n_annihilation += 1;
  uint32_t b[4];
  track_block(X->seed, X->id, X->n, 1u, b);
  double d[3], md[3], Eg;
  if (S->prec == OR_MIXED) {
    float c = 2.0f * or_u01f(b[1]) - 1.0f;
    float st = sqrtf(fmaxx(0.0f, 1.0f - c * c));
    float ph = (2.0f * kPIf) * or_u01f(b[2]);
    float sp, cp;
    or_sincosf(ph, &sp, &cp);
    float df[3] = {st * cp, st * sp, c};
    for (int i = 0; i < 3; ++i) {
      d[i] = (double)df[i];
      md[i] = (double)(-df[i]);
    }
    Eg = (double)kMEf;
  } else {
    double c = 2.0 * or_u01(b[1]) - 1.0;
    double st = sqrt(dmax(0.0, 1.0 - c * c));
    double ph = (2.0 * kPI) * or_u01(b[2]);
    double sp, cp;
    or_sincos(ph, &sp, &cp);
    d[0] = st * cp; d[1] = st * sp; d[2] = c;
    for (int i = 0; i < 3; ++i) md[i] = -d[i];
    Eg = kME;
  }
  create(S, X, OR_GAMMA, Eg, pos, d, v, out);
  create(S, X, OR_GAMMA, Eg, pos, md, v, out);
}

static double rest2(const or_sim *S) { return S->prec == OR_MIXED ? 2.0 * (double)kMEf : 2.0 * kME; }

enum { LIM_RANGE = 0, LIM_PHYS = 1, LIM_GEOM = 2 };

/* Rotation taking z-hat to u applied to d (no renormalisation). */
static void rotate_d(double u[3], double dx, double dy, double dz) {
  double ux = u[0], uy = u[1], uz = u[2];
  double up = sqrt(ux * ux + uy * uy);
  if (up > 0.0) {
    u[0] = (ux * uz * dx - uy * dy) / up + ux * dz;
    u[1] = (uy * uz * dx + ux * dy) / up + uy * dz;
    u[2] = -up * dx + uz * dz;
  } else if (uz > 0.0) {
    u[0] = dx; u[1] = dy; u[2] = dz;
  } else {
    u[0] = -dx; u[1] = dy; u[2] = -dz;
  }
}
static void rotate_f(float u[3], float dx, float dy, float dz) {
  float ux = u[0], uy = u[1], uz = u[2];
  float up = sqrtf(ux * ux + uy * uy);
  if (up > 0.0f) {
    u[0] = (ux * uz * dx - uy * dy) / up + ux * dz;
    u[1] = (uy * uz * dx + ux * dy) / up + uy * dz;
    u[2] = -up * dx + uz * dz;
  } else if (uz > 0.0f) {
    u[0] = dx; u[1] = dy; u[2] = dz;
  } else {
    u[0] = -dx; u[1] = dy; u[2] = -dz;
  }
}

/* Advance by s along dir; on a geometry-limited step snap and change volume. */
static int advance(double pos[3], double p0[3], const double dir[3], double s, int v, int lim, int axis) {
  for (int i = 0; i < 3; ++i) {
    p0[i] = pos[i];
    pos[i] = p0[i] + s * dir[i];
  }
  return lim == LIM_GEOM ? cross(pos, dir, v, axis) : v;
}

/* An electron below the cut stops (its energy is already booked); a positron
 * annihilates at rest into two photons. */
static void charged_death(or_sim *S, int type, creator *X, const double pos[3], int v1, creations *out) {
  if (type == OR_POSITRON) {
    S->led.annihilated += 1;
    annihilate(S, X, pos, v1, out);
  } else {
    S->led.cut[type] += 1;
  }
}

/* ---- e+- step, binary64 policy.  Returns 1 if the track survives. */
static int step_charged_d(or_sim *S, int type, or_track *t, creations *out) {
  const uint32_t n = t->rngCtr;
  uint32_t a[4], b[4];
  track_block(t->rngSeed, t->trackId, n, 0, a);
  track_block(t->rngSeed, t->trackId, n, 1, b);
  creator X = {t->rngSeed, t->event, t->trackId, n, 0};
  const int v = t->volume, m = v & 1;
  const uint32_t ev = t->event;
  const double E0 = t->E;
  double nl = t->numIALeft;
  if (nl < 0.0) nl = -or_log(or_u01(a[0]));
  const double lam = kX0[m];
  const double s_phys = nl * lam;
  int32_t axis;
  const double s_geom = or_distance(t->pos, t->dir, v, &axis);
  const double s_range = E0 / kDEDX[m];
  int lim;
  double s;
  if (s_range <= s_phys && s_range <= s_geom) { lim = LIM_RANGE; s = s_range; }
  else if (s_phys <= s_geom) { lim = LIM_PHYS; s = s_phys; }
  else { lim = LIM_GEOM; s = s_geom; }
  double p0[3];
  const int v1 = advance(t->pos, p0, t->dir, s, v, lim, axis);
  /* continuous loss; E0 - E1 is exact (Dekker's Fast2Sum lemma) */
  const double E1 = (lim == LIM_RANGE) ? 0.0 : dmax(E0 - kDEDX[m] * s, 0.0);
  const double dep = E0 - E1;
  double mid[3] = {0.5 * (p0[0] + t->pos[0]), 0.5 * (p0[1] + t->pos[1]), 0.5 * (p0[2] + t->pos[2])};
  tally_cont(S, ev, v, dep, mid);
  nl = (lim == LIM_PHYS) ? 0.0 : dmax(nl - s / lam, 0.0);
  if (v1 == OUTSIDE) {
    nadd(&S->escaped[ev], E1);
    if (type == OR_POSITRON) nadd(&S->escaped[ev], rest2(S));
    S->led.escaped[type] += 1;
    return 0;
  }
  if (E1 < kCUTE) {
    tally_cut(S, ev, v, E1, t->pos);
    charged_death(S, type, &X, t->pos, v1, out);
    return 0;
  }
  /* multiple scattering with the pre-step energy */
  const double th0 = (kMSC / E0) * sqrt(s / lam);
  const double th = dmin(th0 * sqrt(-2.0 * or_log(or_u01(a[1]))), kPI);
  const double ph = (2.0 * kPI) * or_u01(a[2]);
  double sth, cth, sph, cph;
  or_sincos(th, &sth, &cth);
  or_sincos(ph, &sph, &cph);
  rotate_d(t->dir, sth * cph, sth * sph, cth);
  double E = E1;
  if (lim == LIM_PHYS) {
    double k = kKMIN * or_exp(or_u01(a[3]) * or_log(E1 / kKMIN));
    k = dmin(dmax(k, kKMIN), E1);
    const double E2 = E1 - k;
    k = E1 - E2;
    S->led.n_brem += 1;
    create(S, &X, OR_GAMMA, k, t->pos, t->dir, v1, out);
    nl = -or_log(or_u01(b[0]));
    E = E2;
    if (E2 < kCUTE) {
      tally_cut(S, ev, v, E2, t->pos);
      charged_death(S, type, &X, t->pos, v1, out);
      return 0;
    }
  }
  t->E = E;
  t->numIALeft = nl;
  t->volume = v1;
  t->rngCtr = n + 1;
  return 1;
}

/* ---- e+- step, mixed policy: binary32 for stepping, sampling and angles;
 * binary64 for the position, the boundary distance and the deposits. */
static int step_charged_m(or_sim *S, int type, or_track *t, creations *out) {
  const uint32_t n = t->rngCtr;
  uint32_t a[4], b[4];
  track_block(t->rngSeed, t->trackId, n, 0, a);
  track_block(t->rngSeed, t->trackId, n, 1, b);
  creator X = {t->rngSeed, t->event, t->trackId, n, 0};
  const int v = t->volume, m = v & 1;
  const uint32_t ev = t->event;
  const float E0 = (float)t->E;
  float nl = (float)t->numIALeft;
  if (nl < 0.0f) nl = -or_logf(or_u01f(a[0]));
  const float lam = kX0f[m];
  const float s_phys = nl * lam;
  int32_t axis;
  const double s_geom = or_distance(t->pos, t->dir, v, &axis);
  const float s_range = E0 / kDEDXf[m];
  const double sp = (double)s_phys, sr = (double)s_range;
  int lim;
  double s;
  if (sr <= sp && sr <= s_geom) { lim = LIM_RANGE; s = sr; }
  else if (sp <= s_geom) { lim = LIM_PHYS; s = sp; }
  else { lim = LIM_GEOM; s = s_geom; }
  double p0[3];
  const int v1 = advance(t->pos, p0, t->dir, s, v, lim, axis);
  const float E1 = (lim == LIM_RANGE) ? 0.0f : (float)dmax((double)E0 - kDEDX[m] * s, 0.0);
  double dep, err;
  two_sum((double)E0, -(double)E1, &dep, &err);
  double mid[3] = {0.5 * (p0[0] + t->pos[0]), 0.5 * (p0[1] + t->pos[1]), 0.5 * (p0[2] + t->pos[2])};
  tally_cont(S, ev, v, dep, mid);
  nadd(&S->round[ev], err);
  const float sf = (float)s;
  nl = (lim == LIM_PHYS) ? 0.0f : fmaxx(nl - sf / lam, 0.0f);
  if (v1 == OUTSIDE) {
    nadd(&S->escaped[ev], (double)E1);
    if (type == OR_POSITRON) nadd(&S->escaped[ev], rest2(S));
    S->led.escaped[type] += 1;
    return 0;
  }
  if (E1 < kCUTEf) {
    tally_cut(S, ev, v, (double)E1, t->pos);
    charged_death(S, type, &X, t->pos, v1, out);
    return 0;
  }
  const float th0 = (kMSCf / E0) * sqrtf(sf / lam);
  const float th = fminn(th0 * sqrtf(-2.0f * or_logf(or_u01f(a[1]))), kPIf);
  const float ph = (2.0f * kPIf) * or_u01f(a[2]);
  float sth, cth, sph, cph;
  or_sincosf(th, &sth, &cth);
  or_sincosf(ph, &sph, &cph);
  float u[3] = {(float)t->dir[0], (float)t->dir[1], (float)t->dir[2]};
  rotate_f(u, sth * cph, sth * sph, cth);
  for (int i = 0; i < 3; ++i) t->dir[i] = (double)u[i];
  float E = E1;
  if (lim == LIM_PHYS) {
    float k = kKMINf * or_expf(or_u01f(a[3]) * or_logf(E1 / kKMINf));
    k = fminn(fmaxx(k, kKMINf), E1);
    const float E2 = E1 - k;
    k = E1 - E2;
    S->led.n_brem += 1;
    create(S, &X, OR_GAMMA, (double)k, t->pos, t->dir, v1, out);
    nl = -or_logf(or_u01f(b[0]));
    E = E2;
    if (E2 < kCUTEf) {
      tally_cut(S, ev, v, (double)E2, t->pos);
      charged_death(S, type, &X, t->pos, v1, out);
      return 0;
    }
  }
  t->E = (double)E;
  t->numIALeft = (double)nl;
  t->volume = v1;
  t->rngCtr = n + 1;
  return 1;
}

/* ---- photon step, binary64 policy */
static int step_photon_d(or_sim *S, or_track *t, creations *out) {
  const uint32_t n = t->rngCtr;
  uint32_t a[4], b[4];
  track_block(t->rngSeed, t->trackId, n, 0, a);
  track_block(t->rngSeed, t->trackId, n, 1, b);
  creator X = {t->rngSeed, t->event, t->trackId, n, 0};
  const int v = t->volume, m = v & 1;
  const uint32_t ev = t->event;
  const double E = t->E;
  double nl = t->numIALeft;
  if (nl < 0.0) nl = -or_log(or_u01(a[0]));
  const int pair = E > kPAIRTH;
  const double lam = pair ? kLPAIR[m] : kLCOMP[m];
  const double s_phys = nl * lam;
  int32_t axis;
  const double s_geom = or_distance(t->pos, t->dir, v, &axis);
  const int lim = (s_phys <= s_geom) ? LIM_PHYS : LIM_GEOM;
  const double s = lim == LIM_PHYS ? s_phys : s_geom;
  double p0[3];
  const int v1 = advance(t->pos, p0, t->dir, s, v, lim, axis);
  nl = (lim == LIM_PHYS) ? 0.0 : dmax(nl - s / lam, 0.0);
  if (v1 == OUTSIDE) {
    nadd(&S->escaped[ev], E);
    S->led.escaped[OR_GAMMA] += 1;
    return 0;
  }
  if (lim == LIM_PHYS && pair) {
    S->led.n_pair += 1;
    S->led.absorbed += 1;
    double T, r;
    two_sum(E, -kPAIRTH, &T, &r);
    nadd(&S->round[ev], r);
    double Tm = or_u01(a[3]) * T;
    const double Tp = T - Tm;
    Tm = T - Tp;
    create(S, &X, OR_ELECTRON, Tm, t->pos, t->dir, v1, out);
    create(S, &X, OR_POSITRON, Tp, t->pos, t->dir, v1, out);
    return 0;
  }
  double Enew = E;
  if (lim == LIM_PHYS) {
    S->led.n_compton += 1;
    double T = or_u01(a[3]) * E;
    const double Ep = E - T;
    T = E - Ep;
    create(S, &X, OR_ELECTRON, T, t->pos, t->dir, v1, out);
    nl = -or_log(or_u01(b[0]));
    Enew = Ep;
    if (Ep < kCUTG) {
      tally_cut(S, ev, v, Ep, t->pos);
      S->led.cut[OR_GAMMA] += 1;
      return 0;
    }
  }
  t->E = Enew;
  t->numIALeft = nl;
  t->volume = v1;
  t->rngCtr = n + 1;
  return 1;
}

/* ---- photon step, mixed policy */
static int step_photon_m(or_sim *S, or_track *t, creations *out) {
  const uint32_t n = t->rngCtr;
  uint32_t a[4], b[4];
  track_block(t->rngSeed, t->trackId, n, 0, a);
  track_block(t->rngSeed, t->trackId, n, 1, b);
  creator X = {t->rngSeed, t->event, t->trackId, n, 0};
  const int v = t->volume, m = v & 1;
  const uint32_t ev = t->event;
  const float E = (float)t->E;
  float nl = (float)t->numIALeft;
  if (nl < 0.0f) nl = -or_logf(or_u01f(a[0]));
  const int pair = E > kPAIRTHf;
  const float lam = pair ? kLPAIRf[m] : kLCOMPf[m];
  const float s_phys = nl * lam;
  int32_t axis;
  const double s_geom = or_distance(t->pos, t->dir, v, &axis);
  const int lim = ((double)s_phys <= s_geom) ? LIM_PHYS : LIM_GEOM;
  const double s = lim == LIM_PHYS ? (double)s_phys : s_geom;
  double p0[3];
  const int v1 = advance(t->pos, p0, t->dir, s, v, lim, axis);
  nl = (lim == LIM_PHYS) ? 0.0f : fmaxx(nl - (float)s / lam, 0.0f);
  if (v1 == OUTSIDE) {
    nadd(&S->escaped[ev], (double)E);
    S->led.escaped[OR_GAMMA] += 1;
    return 0;
  }
  if (lim == LIM_PHYS && pair) {
    S->led.n_pair += 1;
    S->led.absorbed += 1;
    float T, r;
    two_sumf(E, -kPAIRTHf, &T, &r);
    nadd(&S->round[ev], (double)r);
    float Tm = or_u01f(a[3]) * T;
    const float Tp = T - Tm;
    Tm = T - Tp;
    create(S, &X, OR_ELECTRON, (double)Tm, t->pos, t->dir, v1, out);
    create(S, &X, OR_POSITRON, (double)Tp, t->pos, t->dir, v1, out);
    return 0;
  }
  float Enew = E;
  if (lim == LIM_PHYS) {
    S->led.n_compton += 1;
    float T = or_u01f(a[3]) * E;
    const float Ep = E - T;
    T = E - Ep;
    create(S, &X, OR_ELECTRON, (double)T, t->pos, t->dir, v1, out);
    nl = -or_logf(or_u01f(b[0]));
    Enew = Ep;
    if (Ep < kCUTGf) {
      tally_cut(S, ev, v, (double)Ep, t->pos);
      S->led.cut[OR_GAMMA] += 1;
      return 0;
    }
  }
  t->E = (double)Enew;
  t->numIALeft = (double)nl;
  t->volume = v1;
  t->rngCtr = n + 1;
  return 1;
}

static int step_track(or_sim *S, int type, or_track *t, creations *out) {
  out->n = 0;
  if (type == OR_GAMMA) return S->prec == OR_MIXED ? step_photon_m(S, t, out) : step_photon_d(S, t, out);
  return S->prec == OR_MIXED ? step_charged_m(S, type, t, out) : step_charged_d(S, type, t, out);
}

/* ------------------------------------------------------------------------- */
/* Buffers (paper Sec. 2)                                                     */
/* ------------------------------------------------------------------------- */
static int push_out(or_sim *S, const or_track *t, int type, int survivor, uint32_t slot) {
  if (S->n_out == S->cap_out) {
    uint64_t nc = S->cap_out ? 2 * S->cap_out : 1024;
    outrec *p = (outrec *)realloc(S->out, nc * sizeof(outrec));
    if (!p) return OR_E_NOMEM;
    S->out = p;
    S->cap_out = nc;
  }
  outrec *o = &S->out[S->n_out++];
  o->trk = *t;
  o->type = type;
  o->survivor = survivor;
  o->slot = slot;
  return OR_OK;
}

static int push_kill(or_sim *S, int type, uint32_t slot) {
  if (S->n_kills[type] == S->cap_kills[type]) {
    uint64_t nc = S->cap_kills[type] ? 2 * S->cap_kills[type] : 1024;
    uint32_t *p = (uint32_t *)realloc(S->kills[type], nc * sizeof(uint32_t));
    if (!p) return OR_E_NOMEM;
    S->kills[type] = p;
    S->cap_kills[type] = nc;
  }
  S->kills[type][S->n_kills[type]++] = slot;
  return OR_OK;
}

static int dense_reserve(or_sim *S, int type, int b, uint64_t n) {
  if (n <= S->bufcap[type][b]) return OR_OK;
  uint64_t nc = S->bufcap[type][b] ? S->bufcap[type][b] : 1024;
  while (nc < n) nc *= 2;
  if (nc > S->C) nc = S->C;
  or_track *p = (or_track *)realloc(S->buf[type][b], nc * sizeof(or_track));
  if (!p) return OR_E_NOMEM;
  S->buf[type][b] = p;
  S->bufcap[type][b] = nc;
  return OR_OK;
}

static int fail_capacity(or_sim *S, uint64_t iter) {
  S->status = OR_E_CAPACITY;
  S->error_iter = iter;
  return OR_E_CAPACITY;
}

/* Append the collected creations (injection, no survivors) after the current
 * entries of each type: dense at index n[type], sparse into slots taken from
 * the front of the free ring and appended to the current list. */
static int place_appended(or_sim *S, int count_on, uint64_t err_iter) {
  uint64_t add[3] = {0, 0, 0};
  for (uint64_t i = 0; i < S->n_out; ++i) add[S->out[i].type] += 1;
  for (int t = 0; t < 3; ++t) {
    if (S->scheme == OR_DENSE ? (S->n[t] + add[t] > S->C) : (add[t] > S->count[t])) return fail_capacity(S, err_iter);
  }
  for (int t = 0; t < 3; ++t)
    if (S->scheme == OR_DENSE && dense_reserve(S, t, S->cur[t], S->n[t] + add[t]) != OR_OK) return OR_E_NOMEM;
  uint64_t j[3] = {0, 0, 0};
  for (uint64_t i = 0; i < S->n_out; ++i) {
    const outrec *o = &S->out[i];
    int t = o->type;
    if (S->scheme == OR_DENSE) {
      uint64_t idx = S->n[t] + j[t];
      S->buf[t][S->cur[t]][idx] = o->trk;
      if (count_on) count_full_write(S, t, S->cur[t], idx);
      if (idx + 1 > S->slots_hw[t]) S->slots_hw[t] = idx + 1;
    } else {
      uint32_t slot = S->ring[t][(S->head[t] + j[t]) % S->C];
      S->buf[t][0][slot] = o->trk;
      S->list_cur[t][S->n[t] + j[t]] = slot;
      if (count_on) count_full_write(S, t, 0, slot);
      if (!S->touched[t][slot]) {
        S->touched[t][slot] = 1;
        S->slots_hw[t] += 1;
      }
    }
    j[t] += 1;
  }
  for (int t = 0; t < 3; ++t) {
    if (S->scheme == OR_SPARSE) {
      S->head[t] = (S->head[t] + add[t]) % S->C;
      S->count[t] -= add[t];
    }
    S->n[t] += add[t];
  }
  S->n_out = 0;
  return OR_OK;
}

static int validate(const or_sim *S, const or_primary *p) {
  if (p->type < 0 || p->type > 2 || p->event >= S->n_events) return OR_E_INVALID;
  if (!isfinite(p->E) || !(p->E > 0.0) || !isfinite(p->numIALeft)) return OR_E_INVALID;
  for (int i = 0; i < 3; ++i)
    if (!isfinite(p->pos[i]) || !isfinite(p->dir[i])) return OR_E_INVALID;
  int32_t v;
  if (or_locate(p->pos, &v) != OR_OK) return OR_E_INVALID;
  if ((p->trackId >> 63) != 0) return OR_E_INVALID;
  return OR_OK;
}

/* Primaries go through the creation path in input order: the primary is its
 * own creator (id as given, counter 0); a sub-cut primary deposits locally and
 * a sub-cut primary positron annihilates with its own block 1 at counter 0.
 * Under the mixed policy E, dir and numIALeft are rounded to binary32 and the
 * energy residual is booked to the rounding tally. */
static int inject_range(or_sim *S, const or_primary *p, uint64_t n) {
  const int count_on = counting(S);
  S->n_out = 0;
  for (uint64_t i = 0; i < n; ++i) {
    const or_primary *q = &p[i];
    int32_t v;
    or_locate(q->pos, &v);
    const uint32_t ev = q->event;
    creations cr;
    cr.n = 0;
    or_track t;
    memset(&t, 0, sizeof(t));
    for (int k = 0; k < 3; ++k) {
      t.pos[k] = q->pos[k];
      t.dir[k] = S->prec == OR_MIXED ? (double)(float)q->dir[k] : q->dir[k];
    }
    t.E = S->prec == OR_MIXED ? (double)(float)q->E : q->E;
    t.numIALeft = S->prec == OR_MIXED ? (double)(float)q->numIALeft : q->numIALeft;
    t.trackId = q->trackId;
    t.parentId = UINT64_MAX;
    t.rngSeed = S->seeds[ev];
    t.rngCtr = 0;
    t.volume = v;
    t.event = ev;
    nadd(&S->ein[ev], q->E);
    if (q->type == OR_POSITRON) nadd(&S->ein[ev], rest2(S));
    if (S->prec == OR_MIXED) nadd(&S->round[ev], q->E - t.E);
    int subcut;
    if (S->prec == OR_MIXED) subcut = (q->type == OR_GAMMA) ? ((float)t.E < kCUTGf) : ((float)t.E < kCUTEf);
    else subcut = (q->type == OR_GAMMA) ? (t.E < kCUTG) : (t.E < kCUTE);
    S->led.primaries[q->type] += 1;
    if (subcut) {
      tally_cut(S, ev, v, t.E, t.pos);
      if (q->type == OR_POSITRON) {
        S->led.annihilated += 1;
        creator X = {t.rngSeed, ev, t.trackId, 0u, 0};
        annihilate(S, &X, t.pos, v, &cr);
      } else {
        S->led.cut[q->type] += 1;
      }
      for (int k = 0; k < cr.n; ++k)
        if (push_out(S, &cr.trk[k], cr.type[k], 0, 0) != OR_OK) return OR_E_NOMEM;
    } else {
      if (push_out(S, &t, q->type, 0, 0) != OR_OK) return OR_E_NOMEM;
    }
  }
  return place_appended(S, count_on, S->iter + 1);
}

int or_inject(or_sim *S, const or_primary *p, uint64_t n) {
  if (S->status != OR_OK) return OR_E_STATE;
  for (uint64_t i = 0; i < n; ++i)
    if (validate(S, &p[i]) != OR_OK) return OR_E_INVALID;
  return inject_range(S, p, n);
}

/* Staged primaries are admitted whole events at a time before an iteration.
 * They must be grouped by event in non-decreasing event order. */
int or_stage(or_sim *S, const or_primary *p, uint64_t n) {
  if (S->status != OR_OK) return OR_E_STATE;
  for (uint64_t i = 0; i < n; ++i) {
    if (validate(S, &p[i]) != OR_OK) return OR_E_INVALID;
    if (i > 0 && p[i].event < p[i - 1].event) return OR_E_INVALID;
  }
  free(S->staged); free(S->ev_first); free(S->ev_count); free(S->ev_energy); free(S->ev_id);
  free(S->ev_admit_iter);
  S->staged = (or_primary *)malloc(n * sizeof(or_primary) + 1);
  memcpy(S->staged, p, n * sizeof(or_primary));
  S->n_staged = n;
  uint64_t g = 0;
  for (uint64_t i = 0; i < n; ++i)
    if (i == 0 || p[i].event != p[i - 1].event) g += 1;
  S->ev_first = (uint64_t *)calloc(g + 1, sizeof(uint64_t));
  S->ev_count = (uint64_t *)calloc(g + 1, sizeof(uint64_t));
  S->ev_energy = (double *)calloc(g + 1, sizeof(double));
  S->ev_id = (uint32_t *)calloc(g + 1, sizeof(uint32_t));
  S->ev_admit_iter = (uint64_t *)calloc(g + 1, sizeof(uint64_t));
  S->g_old = 0;
  for (int t = 0; t < 3; ++t) S->reserved[t] = 0.0;
  g = 0;
  for (uint64_t i = 0; i < n; ++i) {
    if (i == 0 || p[i].event != p[i - 1].event) {
      S->ev_first[g] = i;
      S->ev_id[g] = p[i].event;
      g += 1;
    }
    S->ev_count[g - 1] += 1;
    S->ev_energy[g - 1] = S->ev_energy[g - 1] + p[i].E; /* plain sum in input order */
  }
  S->n_groups = g;
  S->next_group = 0;
  return OR_OK;
}

/* Projected peak of an event group: ceil(kappa * E_event / 1000) tracks per type. */
static double need_of(const or_sim *S, uint64_t g, int t) { return ceil(S->kappa[t] * S->ev_energy[g] / 1000.0); }

/* Admission before an iteration: an admitted event keeps its projected peak
 * reserved for `hold` iterations (about the time its shower needs to peak).
 * Whole events are admitted in order while, for every type,
 * n + reserved + projected peak <= alpha * C; with no active track, the first
 * waiting event is always admitted. */
static int admit(or_sim *S) {
  if (!S->adm_on || S->next_group >= S->n_groups) return OR_OK;
  const uint64_t now = S->iter;
  while (S->g_old < S->next_group && S->ev_admit_iter[S->g_old] + S->hold <= now) {
    for (int t = 0; t < 3; ++t) S->reserved[t] = S->reserved[t] - need_of(S, S->g_old, t);
    S->g_old += 1;
  }
  double run[3];
  for (int t = 0; t < 3; ++t) run[t] = (double)S->n[t] + S->reserved[t];
  const int none_active = (S->n[0] + S->n[1] + S->n[2]) == 0;
  const double limit = S->alpha * (double)S->C;
  uint64_t g0 = S->next_group, g = g0;
  while (g < S->n_groups) {
    double need[3];
    int fits = 1;
    for (int t = 0; t < 3; ++t) {
      need[t] = need_of(S, g, t);
      if (!(run[t] + need[t] <= limit)) fits = 0;
    }
    if (!fits && !(none_active && g == g0)) break;
    for (int t = 0; t < 3; ++t) {
      run[t] = run[t] + need[t];
      S->reserved[t] = S->reserved[t] + need[t];
    }
    S->ev_admit_iter[g] = now;
    g += 1;
  }
  if (g == g0) return OR_OK;
  uint64_t first = S->ev_first[g0];
  uint64_t last = S->ev_first[g - 1] + S->ev_count[g - 1];
  S->next_group = g;
  return inject_range(S, S->staged + first, last - first);
}

int or_step(or_sim *S, uint64_t next_counts[3]) {
  if (S->status != OR_OK) return OR_E_STATE;
  int rc = admit(S);
  if (rc != OR_OK) return rc;
  const uint64_t t_iter = S->iter + 1;
  const int count_on = counting(S);
  S->n_out = 0;
  for (int t = 0; t < 3; ++t) {
    S->n_kills[t] = 0;
    if (S->n[t] > S->peak[t]) S->peak[t] = S->n[t];
  }
  /* pass 1: step every source in canonical order, collect outputs */
  for (int D = 0; D < 3; ++D) {
    const int b = S->scheme == OR_DENSE ? S->cur[D] : 0;
    uint64_t group[8] = {0, 0, 0, 0, 0, 0, 0, 0}; /* outcomes in the current group of 64 */
    for (uint64_t i = 0; i < S->n[D]; ++i) {
      const uint32_t slot = S->scheme == OR_DENSE ? (uint32_t)i : S->list_cur[D][i];
      or_track trk = S->buf[D][b][slot];
      if (count_on) count_source_reads(S, D, b, slot);
      creations cr;
      const int surv = step_track(S, D, &trk, &cr);
      S->steps[D] += 1;
      group[(surv ? 1 : 0) | (cr.n << 1)] += 1;
      if ((i & 63) == 63 || i + 1 == S->n[D]) {
        uint64_t all = 0, most = 0;
        for (int k = 0; k < 8; ++k) {
          all += group[k];
          if (group[k] > most) most = group[k];
          group[k] = 0;
        }
        S->led.off_mode += all - most;
      }
      if (surv) {
        S->led.survivors[D] += 1;
        if (count_on && S->scheme == OR_DENSE) count_leaf(S, D, b, slot, 9, 0);
        if (push_out(S, &trk, D, 1, slot) != OR_OK) return OR_E_NOMEM;
      } else if (S->scheme == OR_SPARSE) {
        if (push_kill(S, D, slot) != OR_OK) return OR_E_NOMEM;
      }
      for (int k = 0; k < cr.n; ++k)
        if (push_out(S, &cr.trk[k], cr.type[k], 0, 0) != OR_OK) return OR_E_NOMEM;
    }
  }
  /* pass 2: build the next iteration's buffers */
  uint64_t nn[3] = {0, 0, 0}, alloc[3] = {0, 0, 0};
  for (uint64_t i = 0; i < S->n_out; ++i) {
    nn[S->out[i].type] += 1;
    if (!S->out[i].survivor) alloc[S->out[i].type] += 1;
  }
  for (int t = 0; t < 3; ++t) {
    if (S->scheme == OR_DENSE ? (nn[t] > S->C) : (alloc[t] > S->count[t])) return fail_capacity(S, t_iter);
  }
  for (int t = 0; t < 3; ++t) S->led.outputs[t] += nn[t];
  if (S->scheme == OR_DENSE) {
    for (int t = 0; t < 3; ++t)
      if (dense_reserve(S, t, 1 - S->cur[t], nn[t]) != OR_OK) return OR_E_NOMEM;
    uint64_t j[3] = {0, 0, 0};
    for (uint64_t i = 0; i < S->n_out; ++i) {
      const outrec *o = &S->out[i];
      const int t = o->type, nb = 1 - S->cur[t];
      S->buf[t][nb][j[t]] = o->trk;
      if (count_on) count_full_write(S, t, nb, j[t]);
      if (j[t] + 1 > S->slots_hw[t]) S->slots_hw[t] = j[t] + 1;
      j[t] += 1;
    }
    for (int t = 0; t < 3; ++t) {
      S->cur[t] = 1 - S->cur[t];
      S->n[t] = nn[t];
    }
  } else {
    uint64_t j[3] = {0, 0, 0}, a[3] = {0, 0, 0};
    for (uint64_t i = 0; i < S->n_out; ++i) {
      const outrec *o = &S->out[i];
      const int t = o->type;
      uint32_t slot;
      if (o->survivor) {
        slot = o->slot;
        if (count_on) count_sparse_survivor(S, t, slot);
      } else {
        slot = S->ring[t][(S->head[t] + a[t]) % S->C];
        a[t] += 1;
        if (count_on) count_full_write(S, t, 0, slot);
        if (!S->touched[t][slot]) {
          S->touched[t][slot] = 1;
          S->slots_hw[t] += 1;
        }
      }
      S->buf[t][0][slot] = o->trk;
      S->list_next[t][j[t]++] = slot;
    }
    for (int t = 0; t < 3; ++t) {
      S->head[t] = (S->head[t] + alloc[t]) % S->C;
      S->count[t] -= alloc[t];
      for (uint64_t f = 0; f < S->n_kills[t]; ++f) S->ring[t][(S->head[t] + S->count[t] + f) % S->C] = S->kills[t][f];
      S->count[t] += S->n_kills[t];
      uint32_t *tmp = S->list_cur[t];
      S->list_cur[t] = S->list_next[t];
      S->list_next[t] = tmp;
      S->n[t] = nn[t];
    }
  }
  S->n_out = 0;
  S->iter = t_iter;
  if (next_counts)
    for (int t = 0; t < 3; ++t) next_counts[t] = S->n[t];
  return OR_OK;
}

int or_run(or_sim *S, uint64_t max_iter, uint64_t *iters_done) {
  uint64_t done = 0;
  int rc = OR_OK;
  while (done < max_iter) {
    const int staged_left = S->adm_on && S->next_group < S->n_groups;
    if (S->n[0] + S->n[1] + S->n[2] == 0 && !staged_left) break;
    rc = or_step(S, NULL);
    if (rc != OR_OK) break;
    done += 1;
  }
  if (iters_done) *iters_done = done;
  return rc;
}

int or_counts(const or_sim *S, uint64_t n[3]) {
  for (int t = 0; t < 3; ++t) n[t] = S->n[t];
  return OR_OK;
}

int or_tally(const or_sim *S, int kind, double *out, size_t n) {
  const uint64_t E = S->n_events;
  switch (kind) {
    case OR_T_DEP_CONT:
    case OR_T_DEP_CUT: {
      if (n != E * NVOL) return OR_E_INVALID;
      const nsum *src = kind == OR_T_DEP_CONT ? S->cont : S->cut;
      for (uint64_t i = 0; i < E * NVOL; ++i) out[i] = nval(&src[i]);
      return OR_OK;
    }
    case OR_T_LAYER: {
      if (n != E * NLAYER) return OR_E_INVALID;
      for (uint64_t e = 0; e < E; ++e)
        for (int l = 0; l < NLAYER; ++l) {
          nsum a = {0.0, 0.0};
          for (int k = 0; k < 2; ++k) {
            nadd(&a, nval(&S->cont[e * NVOL + 2 * l + k]));
            nadd(&a, nval(&S->cut[e * NVOL + 2 * l + k]));
          }
          out[e * NLAYER + l] = nval(&a);
        }
      return OR_OK;
    }
    case OR_T_ESCAPED:
    case OR_T_ROUND:
    case OR_T_EIN: {
      if (n != E) return OR_E_INVALID;
      const nsum *src = kind == OR_T_ESCAPED ? S->escaped : (kind == OR_T_ROUND ? S->round : S->ein);
      for (uint64_t e = 0; e < E; ++e) out[e] = nval(&src[e]);
      return OR_OK;
    }
    case OR_T_INFLIGHT: {
      if (n != E) return OR_E_INVALID;
      nsum *acc = (nsum *)calloc(E, sizeof(nsum));
      for (int t = 0; t < 3; ++t)
        for (uint64_t i = 0; i < S->n[t]; ++i) {
          const or_track *tr = S->scheme == OR_DENSE ? &S->buf[t][S->cur[t]][i] : &S->buf[t][0][S->list_cur[t][i]];
          nadd(&acc[tr->event], tr->E);
          if (t == OR_POSITRON) nadd(&acc[tr->event], rest2(S));
        }
      for (uint64_t e = 0; e < E; ++e) out[e] = nval(&acc[e]);
      free(acc);
      return OR_OK;
    }
    case OR_T_CELLS: {
      if (!S->cells || n != (uint64_t)NLAYER * S->nx * S->ny) return OR_E_INVALID;
      for (uint64_t i = 0; i < n; ++i) out[i] = nval(&S->cells[i]);
      return OR_OK;
    }
    default:
      return OR_E_INVALID;
  }
}

int or_stats_get(const or_sim *S, or_stats *o) {
  memset(o, 0, sizeof(*o));
  o->iterations = S->iter;
  for (int t = 0; t < 3; ++t) {
    o->track_steps[t] = S->steps[t];
    o->peak[t] = S->peak[t] > S->n[t] ? S->peak[t] : S->n[t];
    o->slots_touched[t] = S->slots_hw[t];
  }
  o->error_iter = S->error_iter;
  o->status = S->status;
  return OR_OK;
}

int or_ledger_get(const or_sim *S, or_ledger *o) {
  *o = S->led;
  return OR_OK;
}

int or_dump(const or_sim *S, int type, or_track *out, uint32_t *slots, uint64_t cap, uint64_t *n) {
  if (type < 0 || type > 2) return OR_E_INVALID;
  *n = S->n[type];
  if (cap < S->n[type]) return OR_E_INVALID;
  for (uint64_t i = 0; i < S->n[type]; ++i) {
    uint32_t slot = S->scheme == OR_DENSE ? (uint32_t)i : S->list_cur[type][i];
    out[i] = S->buf[type][S->scheme == OR_DENSE ? S->cur[type] : 0][slot];
    if (slots) slots[i] = slot;
  }
  return OR_OK;
}

/* Replace the current tracks of one type (for one-iteration checks from a
 * given state).  Sparse: slots[i] is the slot of trk[i] and the list order. */
int or_load(or_sim *S, int type, const or_track *trk, const uint32_t *slots, uint64_t n) {
  if (type < 0 || type > 2 || n > S->C) return OR_E_INVALID;
  if (S->scheme == OR_DENSE) {
    if (dense_reserve(S, type, S->cur[type], n) != OR_OK) return OR_E_NOMEM;
    for (uint64_t i = 0; i < n; ++i) S->buf[type][S->cur[type]][i] = trk[i];
  } else {
    for (uint64_t i = 0; i < n; ++i) {
      if (slots[i] >= S->C) return OR_E_INVALID;
      S->buf[type][0][slots[i]] = trk[i];
      S->list_cur[type][i] = slots[i];
    }
  }
  S->n[type] = n;
  return OR_OK;
}

int or_ring_get(const or_sim *S, int type, uint32_t *ring, uint64_t *head, uint64_t *count) {
  if (S->scheme != OR_SPARSE || type < 0 || type > 2) return OR_E_INVALID;
  memcpy(ring, S->ring[type], S->C * sizeof(uint32_t));
  *head = S->head[type];
  *count = S->count[type];
  return OR_OK;
}

int or_ring_set(or_sim *S, int type, const uint32_t *ring, uint64_t head, uint64_t count) {
  if (S->scheme != OR_SPARSE || type < 0 || type > 2 || head >= S->C || count > S->C) return OR_E_INVALID;
  memcpy(S->ring[type], ring, S->C * sizeof(uint32_t));
  S->head[type] = head;
  S->count[type] = count;
  return OR_OK;
}

/* Hand-over of a state: the iteration count, and (dense) which physical buffer,
 * A or B, holds the current tracks.  Tracks already loaded stay current: they
 * move with the label (the two buffers swap). */
int or_set_iteration(or_sim *S, uint64_t iter, int dense_current_b) {
  S->iter = iter;
  if (S->scheme == OR_DENSE)
    for (int t = 0; t < 3; ++t) {
      const int want = dense_current_b ? 1 : 0;
      if (S->cur[t] == want) continue;
      or_track *bp = S->buf[t][0];
      uint64_t cap = S->bufcap[t][0];
      S->buf[t][0] = S->buf[t][1];
      S->bufcap[t][0] = S->bufcap[t][1];
      S->buf[t][1] = bp;
      S->bufcap[t][1] = cap;
      S->cur[t] = want;
    }
  return OR_OK;
}

int or_access_totals(const or_sim *S, int type, int b, uint64_t reads[14], uint64_t writes[14]) {
  if (type < 0 || type > 2 || b < 0 || b > 1) return OR_E_INVALID;
  for (int l = 0; l < 14; ++l) {
    reads[l] = S->rw[type][b][l][0];
    writes[l] = S->rw[type][b][l][1];
  }
  return OR_OK;
}

int or_access_slotleaf(const or_sim *S, int type, int b, uint32_t *out, uint64_t n) {
  if (type < 0 || type > 2 || b < 0 || b > 1 || n != S->C * 14) return OR_E_INVALID;
  if (!S->slotleaf[type][b]) memset(out, 0, n * sizeof(uint32_t));
  else memcpy(out, S->slotleaf[type][b], n * sizeof(uint32_t));
  return OR_OK;
}

/* Heatmap of one physical buffer, one counter per 4-byte word: every access to
 * (slot, leaf) adds 1 to each word the leaf covers under the given mapping. */
int or_heat_words(const or_sim *S, int type, int b, int mapping, uint32_t N, uint32_t *out, uint64_t n_words) {
  if (type < 0 || type > 2 || b < 0 || b > 1) return OR_E_INVALID;
  if (mapping == OR_AOSOA && (N < 2 || (N & (N - 1)) || S->C % N)) return OR_E_INVALID;
  if (n_words * 4 != or_buffer_bytes(mapping, N, S->prec, S->C)) return OR_E_INVALID;
  memset(out, 0, n_words * sizeof(uint32_t));
  const uint32_t *sl = S->slotleaf[type][b];
  if (!sl) return OR_OK;
  for (uint64_t slot = 0; slot < S->C; ++slot)
    for (int l = 0; l < 14; ++l) {
      uint32_t c = sl[slot * 14 + (uint64_t)l];
      if (!c) continue;
      uint64_t addr = or_leaf_addr(mapping, N, S->prec, S->C, slot, l);
      for (uint32_t w = 0; w < or_leaf_size(S->prec, l) / 4; ++w) out[addr / 4 + w] += c;
    }
  return OR_OK;
}
