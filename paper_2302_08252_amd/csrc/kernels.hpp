// kernels.hpp -- HIP kernels of the transport iteration for gfx950 (wave64).
//
// One iteration (paper Sec. 2, both track data structures):
//   k_step   : a fixed grid of resident blocks takes tiles (one tile = one block
//              of 64..256 tracks) from an atomic ticket counter; tiles are laid
//              out electrons | positrons | photons, each in current order.  A
//              lane loads its track through the record layout, takes one step,
//              books its deposits in LDS, counts its outputs per particle type;
//              the block scans the counts with wavefront ballots/shuffles, and
//              the tile's global offsets come from a single-pass decoupled
//              look-back (Merrill & Garland 2016) over the tiles before it, so
//              the next buffers hold the outputs in exactly the canonical order
//              (every source in order, survivor first, then its creations).
//   k_epilogue (capi.hip): one wavefront turns the totals into the next counts,
//              advances the free-slot ring, swaps buffers by flipping the parity.
// Flags and values of the look-back share one 64-bit word read and written
// with relaxed device-scope atomics, which bypass the per-XCD L2 caches; no
// device-scope fences are needed.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/adept.h"
#include "layout.hpp"
#include "model.hpp"

namespace adept {

// Occupancy hint for the step kernel (minimum waves per SIMD; 0: none).
#ifndef ADEPT_WAVES_PER_EU
#define ADEPT_WAVES_PER_EU 0
#endif
#if ADEPT_WAVES_PER_EU > 0
#define ADEPT_STEP_ATTR __attribute__((amdgpu_waves_per_eu(ADEPT_WAVES_PER_EU)))
#else
#define ADEPT_STEP_ATTR
#endif

// Phase clocks of the step kernel (measurement only; 0 in normal builds): every
// wavefront adds the shader-clock cycles it spends in each phase of a tile to
// per-block LDS sums, which go to Ctrl::phase at the end of the launch.
#ifndef ADEPT_PHASE_CLOCKS
#define ADEPT_PHASE_CLOCKS 0
#endif
// Phases: 0 load + step, 1 block scan (with the wait for the block's slowest
// wavefront), 2 look-back (with its barrier), 3 writes, 4 end of tile (barriers
// and the next ticket), 5 before the first tile, 6 after the last tile.
constexpr int kPhases = 8;

// Blocks (= compaction tiles) of 64 to 1024 threads.  The step kernel exists in
// two register budgets: launch bounds 256 for tiles up to 256 tracks, and 1024
// (128 VGPRs, four waves per SIMD) for 512 and 1024: larger tiles spread the
// ticket and look-back latency over more tracks.
constexpr int kMaxBlock = 1024;
constexpr int kMaxWaves = kMaxBlock / 64;
constexpr unsigned kMaxGrid = 8192;          // largest grid of the step kernel
constexpr int kRowLen = 2 * 100 + 2;         // continuous[100], local[100], escaped, rounding
constexpr unsigned kXccRows = 16;            // tally rows per XCD id (the hardware XCC id has 4 bits)

// Device control block (one per context, in the arena).  Index p = parity
// selects the current iteration's counts / lists / dense buffers.
struct Ctrl {
  unsigned long long n[2][3];       // active counts per parity and type
  unsigned long long ticket[2];     // tile tickets of the step kernel per parity
  unsigned long long ntiles[2];     // tiles used by the step kernel of each parity
  unsigned long long tot[2][9];     // totals published by the last tile of a step
  unsigned long long head[3], count[3];  // sparse free rings
  unsigned long long iter;          // iterations done
  unsigned long long error_iter;
  unsigned long long steps[3], peak[3];
  unsigned long long waves, waves_div;
  unsigned long long off_mode;      // track-steps whose outcome differs from their wavefront's most common
  unsigned long long surv[3];       // surviving source tracks per type (all iterations)
  unsigned long long outputs[3];    // tracks written into next buffers per type
  unsigned long long inj_ticket[2], inj_ntiles[2], inj_tot[3];
  unsigned long long inj_begin, inj_end;
  unsigned long long next_group, n_groups;
  unsigned long long g_old;         // admission: first group whose reservation may still be held
  double reserved[3];               // admission: projected peaks of recently admitted groups
  unsigned int parity, inj_parity;
  int error;
  unsigned int had_staged;
  unsigned long long adm_for;       // admission: iterations done + 1 when the next one's admission is decided
  unsigned long long overflow;      // set by kernels that saw an index beyond capacity
  unsigned long long phase[kPhases];// wave-cycles per step-kernel phase (ADEPT_PHASE_CLOCKS builds)
};

// Mirror of the few values the host polls (pinned host memory).
struct HostMirror {
  unsigned long long iter;
  unsigned long long n[3];
  unsigned long long done;
  int error;
  int pad;
  unsigned long long error_iter;
};

struct EventGroup {
  unsigned long long first, count;
  double energy;
  unsigned long long admit_iter;  // iterations done when the group was admitted
};

// Everything a kernel needs, by value.
struct KArgs {
  Ctrl* ctrl;
  HostMirror* mirror;
  uint8_t* buf[3][2];          // dense: current/next by parity; sparse: [t][0]
  uint32_t* list[3][2];        // sparse slot lists by parity
  uint32_t* ring[3];           // sparse free rings
  unsigned long long* desc[2]; // look-back words of the step kernel by parity
  unsigned long long* idesc[2];// look-back words of the inject kernel by parity
  double* cont;                // [event][100]
  double* cut;                 // [event][100]
  double* esc;                 // [event]
  double* rnd;                 // [event]
  double* ein;                 // [event]
  double* cells;               // [50][nx][ny] or null
  double* rows;                // tally rows (row_len doubles each, n_rows rows): partial sums folded into
                               // the tallies when they are read.  A single event without cells: one row per
                               // block index; otherwise one row per XCD (hardware XCC id)
  unsigned long long row_len;  // 202 * events + cells: the flat tally index space
  unsigned n_rows;             // rows allocated (per block index, or kXccRows)
  unsigned pad_rows;
  uint32_t nx, ny;
  double pitch;
  double cell_hx, cell_hy;     // (0.5 * nx) * pitch, (0.5 * ny) * pitch
  double cell_xmax, cell_ymax; // nx - 1, ny - 1
  const adept_primary* staged; // primaries waiting for injection
  const EventGroup* groups;
  const uint32_t* seeds;
  uint32_t n_events;
  int scheme;
  unsigned long long C;
  MapArgs map;
  MapArgs tmap[3];             // per particle type (mapping MAP_TYPED)
  // instrumentation
  unsigned long long* rw[3][2];
  uint32_t* heat[3][2];
  unsigned long long instr_last;
  int instr_on;
  // admission
  int adm_on;
  double alpha;
  double kappa[3];
  unsigned long long hold;
  // epilogue behaviour: 1 = an iteration with nothing active still counts
  int count_empty;
  int off_mode_on;             // count Ctrl::off_mode (the lane-weighted divergence diagnostic)
};

__device__ __forceinline__ unsigned long long ld_agent(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(unsigned long long* p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Per-wavefront phase timer (lane 0 of every wavefront; compiled out unless
// ADEPT_PHASE_CLOCKS).
struct PhaseTimer {
#if ADEPT_PHASE_CLOCKS
  unsigned long long last;
  __device__ __forceinline__ void start() { last = __builtin_readcyclecounter(); }
  __device__ __forceinline__ void mark(unsigned long long* acc, int phase) {
    const unsigned long long now = __builtin_readcyclecounter();
    if (__lane_id() == 0) atomicAdd(&acc[phase], now - last);
    last = now;
  }
#else
  __device__ __forceinline__ void start() {}
  __device__ __forceinline__ void mark(unsigned long long*, int) {}
#endif
};

// Cross-lane sums with DPP row shifts (no LDS permute, no per-lane addresses):
// row_shr<K>(x) is x of lane (l - K) when that lane lies in l's row of 16, else 0.
template <int K>
__device__ __forceinline__ uint32_t row_shr(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x110 + K, 0xf, 0xf, false);
}
template <int K>
__device__ __forceinline__ unsigned long long row_shr(unsigned long long x) {
  const uint32_t lo = row_shr<K>((uint32_t)x), hi = row_shr<K>((uint32_t)(x >> 32));
  return ((unsigned long long)hi << 32) | lo;
}
template <class T>
__device__ __forceinline__ T row_scan(T x) {  // inclusive, within each row of 16 lanes
  x += row_shr<1>(x);
  x += row_shr<2>(x);
  x += row_shr<4>(x);
  x += row_shr<8>(x);
  return x;
}
__device__ __forceinline__ uint32_t lane_value(uint32_t x, int l) { return __builtin_amdgcn_readlane(x, l); }
// (readlane yields a signed int: both halves are zero-extended before they are joined)
__device__ __forceinline__ unsigned long long lane_value(unsigned long long x, int l) {
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), l);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, l);
  return ((unsigned long long)hi << 32) | lo;
}
__device__ __forceinline__ double row_shr_f64(double x, int k) {
  const unsigned long long u = __double_as_longlong(x);
  unsigned long long r = 0;
  switch (k) {
    case 1: r = row_shr<1>(u); break;
    case 2: r = row_shr<2>(u); break;
    case 4: r = row_shr<4>(u); break;
    default: r = row_shr<8>(u); break;
  }
  return __longlong_as_double((long long)r);
}
// Sum of a double over the 64 lanes of a wavefront (every lane active; fixed
// order); uniform result.
__device__ __forceinline__ double wave_sum_f64(double v) {
  v += row_shr_f64(v, 1);
  v += row_shr_f64(v, 2);
  v += row_shr_f64(v, 4);
  v += row_shr_f64(v, 8);
  const unsigned long long u = __double_as_longlong(v);
  return ((__longlong_as_double((long long)lane_value(u, 15)) + __longlong_as_double((long long)lane_value(u, 31))) +
          __longlong_as_double((long long)lane_value(u, 47))) +
         __longlong_as_double((long long)lane_value(u, 63));
}

// Inclusive scan over the 64 lanes of a wavefront (every lane active): row scans,
// then the GFX9 row broadcasts (row_bcast:15 adds lane 15 of each row to rows 1
// and 3, row_bcast:31 adds lane 31 to rows 2 and 3), with no lane reads.
__device__ __forceinline__ uint32_t wave_scan(uint32_t x) {
  x = row_scan(x);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);
  return x;
}
// Sum over the 64 lanes of a wavefront (every lane active); uniform result.
__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
  v = row_scan(v);
  return lane_value(v, 15) + lane_value(v, 31) + lane_value(v, 47) + lane_value(v, 63);
}

// ---------------------------------------------------------------------------
// Ordered compaction: block scan of NV small counts per lane (each < 4, packed
// as 16-bit fields, four per 64-bit word) and decoupled look-back for the
// tile's exclusive prefix.  Values are saturated at 2^31 - 1 (capacities are at
// most 2^30, so a saturated total always reads as an overflow).
// ---------------------------------------------------------------------------
constexpr unsigned long long kSat = (1ull << 31) - 1;
constexpr unsigned long long kStA = 1ull << 62, kStP = 2ull << 62;

// LDS state of the ordered compaction: NS values scanned per lane (NV values
// per track times the tracks a lane holds), NV values per tile.
template <int NS, int NV = NS>
struct Scan {
  static constexpr int W = (NS + 2) / 3;  // 32-bit words of three 10-bit fields
  uint32_t wave_tot[kMaxWaves][W];
  unsigned long long tile_excl[NV];
  unsigned long long tile_agg[NV];
  unsigned long long ticket;
};

__device__ __forceinline__ unsigned long long sat_add(unsigned long long a, unsigned long long b) {
  const unsigned long long s = a + b;
  return s > kSat ? kSat : s;
}

// Three 10-bit fields to three 16-bit fields of a 64-bit word.
__device__ __forceinline__ unsigned long long widen3(uint32_t t) {
  return (unsigned long long)(t & 0x3FFu) | ((unsigned long long)(t & 0xFFC00u) << 6) |
         ((unsigned long long)(t & 0x3FF00000u) << 12);
}

// Block-exclusive prefix per lane (lex) and the block aggregates of all NV
// values, packed three per 64-bit word in 16-bit fields (aggw; the same in every
// lane).  Per-lane counts are below 5 and a wavefront's totals below 2^10, so a
// wavefront scans three counts per 32-bit word; sums over wavefronts (below
// 2^13) use 16-bit fields.  One barrier: the wave totals in LDS.
template <int NV, class S>
__device__ __forceinline__ void block_scan(const uint32_t cnt[NV], uint32_t lex[NV],
                                           unsigned long long aggw[(NV + 2) / 3], S& sh) {
  constexpr int W = (NV + 2) / 3;
  const int lane = __lane_id(), wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  uint32_t x[W], inc[W];
#pragma unroll
  for (int w = 0; w < W; ++w) {
    x[w] = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k)
      if (3 * w + k < NV) x[w] |= cnt[3 * w + k] << (10 * k);
    inc[w] = wave_scan(x[w]);
    if (lane == 63) sh.wave_tot[wave][w] = inc[w];
  }
  __syncthreads();
#pragma unroll
  for (int w = 0; w < W; ++w) {
    // lane j < nw takes wave j's totals, widened to 16-bit fields (fields 0 and 1
    // in one word, field 2 in another: sums stay below 2^13, so no carries cross
    // fields); an inclusive scan over the first row of 16 lanes then holds every
    // prefix of the wave totals, read out for this wavefront and for the block
    const uint32_t tw = lane < nw ? sh.wave_tot[lane][w] : 0u;
    const uint32_t lo = row_scan((tw & 0x3FFu) | ((tw & 0xFFC00u) << 6));
    const uint32_t hi = row_scan((tw & 0x3FF00000u) >> 20);
    const unsigned long long sc = ((unsigned long long)hi << 32) | lo;
    const unsigned long long before = wave > 0 ? lane_value(sc, wave - 1) : 0ull;
    const unsigned long long all = lane_value(sc, nw - 1);
    const unsigned long long ex = before + widen3(inc[w] - x[w]);
#pragma unroll
    for (int k = 0; k < 3; ++k)
      if (3 * w + k < NV) lex[3 * w + k] = (uint32_t)((ex >> (16 * k)) & 0xFFFF);
    aggw[w] = all;
  }
}

// Value v of packed block aggregates.
template <int NV>
__device__ __forceinline__ uint32_t agg_value(const unsigned long long aggw[(NV + 2) / 3], int v) {
  return (uint32_t)((aggw[v / 3] >> (16 * (v % 3))) & 0xFFFF);
}

// Decoupled look-back by wavefront 0: publishes the tile aggregate, gathers
// the exclusive prefix from its predecessors, publishes the inclusive prefix.
// Word layout: [status 2][inclusive 31][aggregate 31].
// The wait for predecessors is bounded: after kSpinLimit polls the kernel
// latches an error flag (bit 1 of Ctrl::overflow) and gives up, so every wave
// always reaches its exit.
constexpr unsigned kSpinLimit = 1u << 24;

template <int NV, class S>
__device__ __forceinline__ void lookback(unsigned long long* desc, unsigned long long tile, unsigned long long agg,
                                         S& sh, unsigned long long* err) {
  if (threadIdx.x >= 64) return;
  const int lane = __lane_id();
  if (lane < NV) sh.tile_agg[lane] = agg;
  if (tile == 0) {
    if (lane < NV) {
      st_agent(&desc[lane], kStP | (agg << 31) | agg);
      sh.tile_excl[lane] = 0;
    }
    return;
  }
  if (lane < NV) st_agent(&desc[tile * NV + lane], kStA | agg);
  unsigned long long acc[NV];
  long long base[NV];
  bool done[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    acc[v] = 0;
    base[v] = (long long)tile - 1;
    done[v] = false;
  }
  for (unsigned polls = 0;; ++polls) {
    if (polls >= kSpinLimit) {
      if (lane == 0) atomicOr(err, 2ull);
      break;
    }
    bool all_done = true;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      if (done[v]) continue;
      const long long j = base[v] - lane;
      const unsigned long long w = j >= 0 ? ld_agent(&desc[(unsigned long long)j * NV + v]) : kStP;
      const unsigned long long st = w >> 62;
      const unsigned long long pm = __ballot(st == 2);
      const unsigned long long xm = __ballot(st == 0);
      const int fp = pm ? __ffsll((long long)pm) - 1 : 64;
      const unsigned long long need = fp >= 63 ? ~0ull : ((2ull << fp) - 1);
      if (xm & need) {
        all_done = false;
        continue;  // a tile we depend on has not published yet: read again
      }
      unsigned long long val = 0;
      if (lane < fp) val = w & kSat;                       // aggregates
      else if (lane == fp) val = (w >> 31) & kSat;         // inclusive prefix
      const unsigned long long s = wave_sum(val);
      acc[v] = sat_add(acc[v], s);
      if (fp < 64) done[v] = true;
      else {
        base[v] -= 64;
        all_done = false;
      }
    }
    if (all_done) break;
  }
  if (lane < NV) {
    unsigned long long ex = 0;
#pragma unroll
    for (int v = 0; v < NV; ++v)
      if (v == lane) ex = acc[v];
    st_agent(&desc[tile * NV + lane], kStP | (sat_add(ex, agg) << 31) | agg);
    sh.tile_excl[lane] = ex;
  }
}

// ---------------------------------------------------------------------------
// Tallies: deposits staged in LDS per block (single-event runs), flushed with
// device-scope FP64 atomics at the end of the kernel.
// ---------------------------------------------------------------------------
struct TallyLDS {
  double cont[kNumVol];
  double cut[kNumVol];
  double esc, rnd;
};

// Per-block statistics, flushed with one atomic per counter at the end.
struct StatLDS {
  unsigned long long waves, waves_div, off_mode, surv[3];
};

// Batched runs (several events) and cell scoring: deposits go through a
// direct-mapped LDS cache keyed by the flat tally index
//   [0, 100E) continuous, [100E, 200E) local, [200E, 201E) escaped,
//   [201E, 202E) rounding, then the cells;
// a lane whose slot holds another key adds to HBM directly; occupied slots are
// added to HBM once per block at the end of the kernel.
constexpr uint32_t kCacheEmpty = 0xFFFFFFFFu;
template <int BITS>
struct TallyCache {
  static constexpr int bits = BITS, slots = 1 << BITS;
  uint32_t key[slots];
  double val[slots];
};

__device__ __forceinline__ double* tally_ptr(const KArgs& a, uint32_t key) {
  const uint32_t E = a.n_events;
  if (key < 100u * E) return a.cont + key;
  if (key < 200u * E) return a.cut + (key - 100u * E);
  if (key < 201u * E) return a.esc + (key - 200u * E);
  if (key < 202u * E) return a.rnd + (key - 201u * E);
  return a.cells + (key - 202u * E);
}

// The XCD (accelerator complex die, one L2 cache) the calling workgroup runs on.
__device__ __forceinline__ uint32_t xcc_id() {
  uint32_t x;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID, 0, 4)" : "=s"(x));
  return x;
}

// Where a block's deposits go past its LDS cache: the row of its XCD.  Every
// block that adds to a row runs on that row's XCD, so the row's lines stay in
// one L2 (827 KB for 512 events, against 4 MB of L2 per XCD), where the atomics
// are performed; the rows reach memory when the launch ends.
__device__ __forceinline__ void spill_add(const KArgs& a, uint32_t key, double v) {
  __hip_atomic_fetch_add(a.rows + (unsigned long long)xcc_id() * a.row_len + key, v, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
}

template <class TC>
__device__ __forceinline__ void cache_add(const KArgs& a, TC& tc, uint32_t key, double v) {
  const uint32_t h = (key * 2654435761u) >> (32 - TC::bits);
  uint32_t cur = tc.key[h];
  if (cur == kCacheEmpty) cur = atomicCAS(&tc.key[h], kCacheEmpty, key) == kCacheEmpty ? key : tc.key[h];
  if (cur == key) {
    __hip_atomic_fetch_add(&tc.val[h], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  } else {
    spill_add(a, key, v);
  }
}

template <class TC>
__device__ __forceinline__ void cache_init(TC& tc) {
  for (int i = threadIdx.x; i < TC::slots; i += blockDim.x) {
    tc.key[i] = kCacheEmpty;
    tc.val[i] = 0.0;
  }
}

template <class TC>
__device__ __forceinline__ void cache_flush(const KArgs& a, TC& tc) {
  __syncthreads();
  for (int i = threadIdx.x; i < TC::slots; i += blockDim.x)
    if (tc.key[i] != kCacheEmpty && tc.val[i] != 0.0) spill_add(a, tc.key[i], tc.val[i]);
}

__device__ __forceinline__ void gadd(double* p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// base[key] += v over the lanes of a wavefront (every lane calls it, inactive
// ones with v = 0): one device atomic per distinct key per wavefront instead of
// one per lane on the same address.
__device__ __forceinline__ void wave_gadd_keyed(double* base, uint32_t key, double v) {
  const int lane = __lane_id();
  unsigned long long pending = __ballot(v != 0.0);
  while (pending) {
    const int leader = __ffsll((long long)pending) - 1;
    const uint32_t k = __builtin_amdgcn_readlane(key, leader);
    const unsigned long long m = __ballot(((pending >> lane) & 1ull) && key == k);
    const double s = wave_sum_f64(((m >> lane) & 1ull) ? v : 0.0);
    if (lane == leader) gadd(base + k, s);
    pending &= ~m;
  }
}
__device__ __forceinline__ void ladd(double* p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Flat index of the cell of (x, y) in the layer of volume v.
__device__ __forceinline__ uint32_t cell_index(const KArgs& a, int v, double x, double y) {
  const double fx = floor((x + a.cell_hx) / a.pitch), fy = floor((y + a.cell_hy) / a.pitch);
  const uint32_t ix = fx < 0.0 ? 0u : (fx > a.cell_xmax ? a.nx - 1 : (uint32_t)fx);
  const uint32_t iy = fy < 0.0 ? 0u : (fy > a.cell_ymax ? a.ny - 1 : (uint32_t)fy);
  return ((uint32_t)(v >> 1) * a.nx + ix) * a.ny + iy;
}

// Book one lane's deposits: pre-step volume v, event ev.  tl: single-event
// LDS arrays; tc: LDS cache; neither: direct device atomics.
template <class TC>
__device__ __forceinline__ void book(const KArgs& a, TallyLDS* tl, TC* tc, uint32_t ev, int v,
                                     const Deposits& d, const double pos[3]) {
  if (tl) {
    if (d.cont != 0.0) ladd(&tl->cont[v], d.cont);
    if (d.cut != 0.0) ladd(&tl->cut[v], d.cut);
    if (d.escaped != 0.0) ladd(&tl->esc, d.escaped);
    if (d.round != 0.0) ladd(&tl->rnd, d.round);
    return;
  }
  const uint32_t E = a.n_events;
  const uint32_t kc = ev * kNumVol + (uint32_t)v, ku = 100u * E + kc, ke = 200u * E + ev, kr = 201u * E + ev;
  if (tc) {
    if (d.cont != 0.0) cache_add(a, *tc, kc, d.cont);
    if (d.cut != 0.0) cache_add(a, *tc, ku, d.cut);
    if (d.escaped != 0.0) cache_add(a, *tc, ke, d.escaped);
    if (d.round != 0.0) cache_add(a, *tc, kr, d.round);
    if (a.cells) {
      if (d.cont != 0.0) cache_add(a, *tc, 202u * E + cell_index(a, v, d.mid[0], d.mid[1]), d.cont);
      if (d.cut != 0.0) cache_add(a, *tc, 202u * E + cell_index(a, v, pos[0], pos[1]), d.cut);
    }
    return;
  }
  if (d.cont != 0.0) gadd(tally_ptr(a, kc), d.cont);
  if (d.cut != 0.0) gadd(tally_ptr(a, ku), d.cut);
  if (d.escaped != 0.0) gadd(tally_ptr(a, ke), d.escaped);
  if (d.round != 0.0) gadd(tally_ptr(a, kr), d.round);
  if (a.cells) {
    if (d.cont != 0.0) gadd(a.cells + cell_index(a, v, d.mid[0], d.mid[1]), d.cont);
    if (d.cut != 0.0) gadd(a.cells + cell_index(a, v, pos[0], pos[1]), d.cut);
  }
}

// The block's partial sums go to its own row (plain read-modify-write: no other
// block writes this row during the launch); rows are folded into the event
// tallies in a fixed order when the tallies are read.
__device__ __forceinline__ void flush(const KArgs& a, TallyLDS& tl) {
  __syncthreads();
  double* row = a.rows + (unsigned long long)blockIdx.x * a.row_len;
  for (int i = threadIdx.x; i < kRowLen; i += blockDim.x) {
    double v;
    if (i < kNumVol) v = tl.cont[i];
    else if (i < 2 * kNumVol) v = tl.cut[i - kNumVol];
    else if (i == 2 * kNumVol) v = tl.esc;
    else v = tl.rnd;
    if (v != 0.0) row[i] += v;
  }
}

__device__ __forceinline__ void tally_init(TallyLDS& tl) {
  for (int i = threadIdx.x; i < kNumVol; i += blockDim.x) {
    tl.cont[i] = 0.0;
    tl.cut[i] = 0.0;
  }
  if (threadIdx.x == 0) tl.esc = tl.rnd = 0.0;
}

// Divergence diagnostics of one wavefront step (outcome code = survived? | buffered
// creations << 1, at most 7): whether any lanes disagree, and how many lanes
// differ from the wavefront's most common outcome; also the survivor count.
// Counts of one wavefront over the tracks it steps in a tile (wave-uniform
// values, added to the block's LDS statistics once per tile).
struct DivCount {
  uint32_t waves, waves_div, off_mode, surv;
};
__device__ __forceinline__ void div_count(DivCount& k, bool valid, bool surv, int code, bool off_on) {
  const unsigned long long vm = __ballot(valid);
  if (!vm) return;
  const int first = __ffsll((long long)vm) - 1;
  const int ref = __builtin_amdgcn_readlane(code, first);
  const unsigned long long dm = __ballot(valid && code != ref);
  const unsigned long long sm = __ballot(valid && surv);
  k.waves += 1u;
  k.surv += (uint32_t)__popcll(sm);
  if (dm) {
    k.waves_div += 1u;
    if (off_on) {  // lane masks of the eight codes from the three bit planes (scalar work)
      const unsigned long long b0 = __ballot(code & 1), b1 = __ballot(code & 2), b2 = __ballot(code & 4);
      int most = 0;
#pragma unroll
      for (int c8 = 0; c8 < 8; ++c8) {
        const unsigned long long m = vm & ((c8 & 1) ? b0 : ~b0) & ((c8 & 2) ? b1 : ~b1) & ((c8 & 4) ? b2 : ~b2);
        const int c = __popcll(m);
        most = c > most ? c : most;
      }
      k.off_mode += (uint32_t)(__popcll(vm) - most);
    }
  }
}
__device__ __forceinline__ void div_flush(StatLDS& ss, const DivCount& k, int D) {
  if (__lane_id() == 0 && k.waves) {
    atomicAdd(&ss.waves, (unsigned long long)k.waves);
    if (k.waves_div) atomicAdd(&ss.waves_div, (unsigned long long)k.waves_div);
    if (k.off_mode) atomicAdd(&ss.off_mode, (unsigned long long)k.off_mode);
    if (k.surv) atomicAdd(&ss.surv[D], (unsigned long long)k.surv);
  }
}

__device__ __forceinline__ void div_stats(StatLDS& ss, int D, bool valid, bool surv, int code, bool off_on) {
  const unsigned long long vm = __ballot(valid);
  if (!vm) return;
  const int lane = __lane_id();
  const int first = __ffsll((long long)vm) - 1;
  const int ref = __builtin_amdgcn_readlane(code, first);
  const unsigned long long dm = __ballot(valid && code != ref);
  const unsigned long long sm = __ballot(valid && surv);
  int most = 0;
  if (dm && off_on) {  // lane masks of the eight codes from the three bit planes (scalar work)
    const unsigned long long b0 = __ballot(code & 1), b1 = __ballot(code & 2), b2 = __ballot(code & 4);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const unsigned long long m = vm & ((k & 1) ? b0 : ~b0) & ((k & 2) ? b1 : ~b1) & ((k & 4) ? b2 : ~b2);
      const int c = __popcll(m);
      most = c > most ? c : most;
    }
  } else {
    most = __popcll(vm);
  }
  if (lane == first) {
    atomicAdd(&ss.waves, 1ull);
    if (dm) {
      atomicAdd(&ss.waves_div, 1ull);
      if (off_on) atomicAdd(&ss.off_mode, (unsigned long long)(__popcll(vm) - most));
    }
    if (sm) atomicAdd(&ss.surv[D], (unsigned long long)__popcll(sm));
  }
}

// Creations of each particle type: the type fields of the three slots sit at bits
// 8s and 8s + 1 of the metadata, and a slot not pushed reads as type 0, so type 0
// is what remains of the count after types 1 and 2 (two bit planes, two popcounts).
template <class R>
__device__ __forceinline__ void creation_counts(const Creations<R>& cr, uint32_t c[3]) {
  const uint32_t lo = cr.meta & 0x010101u, hi = (cr.meta >> 1) & 0x010101u;
  c[1] = (uint32_t)__popc(lo & ~hi);
  c[2] = (uint32_t)__popc(hi & ~lo);
  c[0] = (uint32_t)cr.n - c[1] - c[2];
}

// ---------------------------------------------------------------------------
// Track load / store through the accessor.
// ---------------------------------------------------------------------------
template <int MAP, class P, bool INSTR>
__device__ __forceinline__ void load_track(const Acc<MAP, P::mixed, INSTR>& A, uint64_t s, Track<typename P::R>& t) {
  using R = typename P::R;
#pragma unroll
  for (int i = 0; i < 3; ++i) t.pos[i] = A.template ld<double>(s, i);
#pragma unroll
  for (int i = 0; i < 3; ++i) t.dir[i] = A.template ld<R>(s, 3 + i);
  t.E = A.template ld<R>(s, 6);
  t.nl = A.template ld<R>(s, 7);
  t.id = A.template ld<uint64_t>(s, 8);
  t.seed = A.template ld<uint32_t>(s, 10);
  t.ctr = A.template ld<uint32_t>(s, 11);
  t.vol = A.template ld<int32_t>(s, 12);
  t.event = A.template ld<uint32_t>(s, 13);
}

template <int MAP, class P, bool INSTR>
__device__ __forceinline__ void store_full(const Acc<MAP, P::mixed, INSTR>& A, uint64_t s, const double pos[3],
                                           const typename P::R dir[3], typename P::R E, typename P::R nl, uint64_t id,
                                           uint64_t parent, uint32_t seed, uint32_t ctr, int32_t vol, uint32_t ev) {
  using R = typename P::R;
#pragma unroll
  for (int i = 0; i < 3; ++i) A.template st<double>(s, i, pos[i]);
#pragma unroll
  for (int i = 0; i < 3; ++i) A.template st<R>(s, 3 + i, dir[i]);
  A.template st<R>(s, 6, E);
  A.template st<R>(s, 7, nl);
  A.template st<uint64_t>(s, 8, id);
  A.template st<uint64_t>(s, 9, parent);
  A.template st<uint32_t>(s, 10, seed);
  A.template st<uint32_t>(s, 11, ctr);
  A.template st<int32_t>(s, 12, vol);
  A.template st<uint32_t>(s, 13, ev);
}

// Sparse survivor, in place: pos, (dir for e+-), E, numIALeft, rngCtr, volume.
template <int MAP, class P, bool INSTR>
__device__ __forceinline__ void store_inplace(const Acc<MAP, P::mixed, INSTR>& A, uint64_t s,
                                              const Track<typename P::R>& t, bool charged) {
  using R = typename P::R;
#pragma unroll
  for (int i = 0; i < 3; ++i) A.template st<double>(s, i, t.pos[i]);
  if (charged) {
#pragma unroll
    for (int i = 0; i < 3; ++i) A.template st<R>(s, 3 + i, t.dir[i]);
  }
  A.template st<R>(s, 6, t.E);
  A.template st<R>(s, 7, t.nl);
  A.template st<uint32_t>(s, 11, t.ctr);
  A.template st<int32_t>(s, 12, t.vol);
}

template <int MAP, class P, bool INSTR>
__device__ __forceinline__ Acc<MAP, P::mixed, INSTR> make_acc(const KArgs& a, int type, int b, bool on) {
  Acc<MAP, P::mixed, INSTR> A;
  A.base = a.buf[type][b];
  if constexpr (MAP == MAP_TYPED) A.m = a.tmap[type];
  else A.m = a.map;
  A.in.rw = a.rw[type][b];
  A.in.heat = a.heat[type][b];
  A.on = on;
  return A;
}

__device__ __forceinline__ unsigned long long ceil_div(unsigned long long x, unsigned long long y) {
  return (x + y - 1) / y;
}

// Value of creation slot i (a runtime index) without indexing a register array.
template <class T>
__device__ __forceinline__ T sel3(int i, T x0, T x1, T x2) {
  return i == 0 ? x0 : (i == 1 ? x1 : x2);
}

// Write creation slot i (full record) of type d at slot s of physical buffer b;
// n is the counter of the step that made it.
template <int MAP, class P, bool INSTR>
__device__ __forceinline__ void write_creation(const KArgs& a, int d, int b, uint64_t s, bool on,
                                               const Track<typename P::R>& t, const Creations<typename P::R>& cr,
                                               int i, uint32_t n) {
  using R = typename P::R;
  const auto A = make_acc<MAP, P, INSTR>(a, d, b, on);
  const int ds = cr.dsel(i);
  R dir[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) dir[k] = ds == 0 ? t.dir[k] : (ds == 1 ? cr.d[k] : -cr.d[k]);
  const uint64_t parent = creation_parent<P::philox_unroll>(cr, i, t.seed, t.id, n);
  store_full<MAP, P, INSTR>(A, s, t.pos, dir, sel3(i, cr.E[0], cr.E[1], cr.E[2]), (R)-1,
                            creation_id<P::philox_unroll>(cr, i, t.seed, parent, n), parent, t.seed, 0u, t.vol, t.event);
}

// ---------------------------------------------------------------------------
// Outputs of a stepped track kept in LDS while the lane steps its next track
// (field-major: consecutive lanes touch consecutive words).  `aux` holds the
// parent id of a dense survivor or the slot of a sparse source.
// ---------------------------------------------------------------------------
template <class R, bool ON>
struct Park {};
template <class R>
struct Park<R, true> {
  double pos[3][kMaxBlock];
  uint64_t id[kMaxBlock], aux[kMaxBlock];
  R dir[3][kMaxBlock], E[kMaxBlock], nl[kMaxBlock];
  R cE[3][kMaxBlock], cd[3][kMaxBlock];
  uint32_t seed[kMaxBlock], ctr[kMaxBlock], vol[kMaxBlock], event[kMaxBlock];
  uint32_t meta[kMaxBlock];  // creation metadata (bits 0-25), creations (26-27), survived (28), valid (29)
};

template <class R>
__device__ __forceinline__ void park(Park<R, true>& k, int i, const Track<R>& t, const Creations<R>& cr, bool surv,
                                     bool valid, uint64_t aux) {
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    k.pos[j][i] = t.pos[j];
    k.dir[j][i] = t.dir[j];
    k.cE[j][i] = cr.E[j];
    k.cd[j][i] = cr.d[j];
  }
  k.E[i] = t.E;
  k.nl[i] = t.nl;
  k.id[i] = t.id;
  k.aux[i] = aux;
  k.seed[i] = t.seed;
  k.ctr[i] = t.ctr;
  k.vol[i] = (uint32_t)t.vol;
  k.event[i] = t.event;
  k.meta[i] = cr.meta | ((uint32_t)cr.n << 26) | (surv ? 1u << 28 : 0u) | (valid ? 1u << 29 : 0u);
}

template <class R>
__device__ __forceinline__ void unpark(const Park<R, true>& k, int i, Track<R>& t, Creations<R>& cr, bool& surv,
                                       bool& valid, uint64_t& aux) {
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    t.pos[j] = k.pos[j][i];
    t.dir[j] = k.dir[j][i];
    cr.E[j] = k.cE[j][i];
    cr.d[j] = k.cd[j][i];
  }
  t.E = k.E[i];
  t.nl = k.nl[i];
  t.id = k.id[i];
  aux = k.aux[i];
  t.seed = k.seed[i];
  t.ctr = k.ctr[i];
  t.vol = (int32_t)k.vol[i];
  t.event = k.event[i];
  const uint32_t m = k.meta[i];
  cr.meta = m & ((1u << 26) - 1);
  cr.n = (int)((m >> 26) & 3u);
  surv = ((m >> 28) & 1u) != 0;
  valid = ((m >> 29) & 1u) != 0;
}

// ---------------------------------------------------------------------------
// The fused step kernel.  A tile is TPT * blockDim.x consecutive tracks of one
// type; lane l steps tracks l, l + blockDim.x, ...  The outputs of all but the
// last are parked in LDS, so the scan, the look-back and the barriers of a tile
// are paid once for TPT tracks per lane.  Canonical order within a tile: the
// sources in index order, i.e. the first track of every lane, then the second.
// ---------------------------------------------------------------------------
template <int SCHEME, int MAP, class P, bool INSTR, int LB>
__global__ void __launch_bounds__(LB) ADEPT_STEP_ATTR k_step(const KArgs a) {
  using R = typename P::R;
  constexpr int NV = SCHEME == DENSE ? 3 : 9;  // next[3] (+ new[3], kill[3])
  constexpr int TPT = P::tracks_per_lane(LB);
  constexpr int NS = NV * TPT;
  __shared__ Scan<NS, NV> sh;
  __shared__ Park<R, (TPT > 1)> pk;
  __shared__ TallyLDS tl;
  __shared__ TallyCache<P::tally_cache_bits> tc;
  __shared__ StatLDS ss;
  __shared__ unsigned long long ph_acc[kPhases];
  PhaseTimer pt;
  pt.start();
  Ctrl* c = a.ctrl;
  const uint32_t p = c->parity;
  const unsigned long long n0 = c->n[p][0], n1 = c->n[p][1], n2 = c->n[p][2];
  const unsigned long long T = blockDim.x, TT = T * TPT;
  const unsigned long long t0 = ceil_div(n0, TT), t1 = ceil_div(n1, TT), t2 = ceil_div(n2, TT);
  const unsigned long long total = t0 + t1 + t2;
  const bool counting = INSTR && a.instr_on && c->iter < a.instr_last;
  const bool lds_tally = a.n_events == 1 && !a.cells;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    c->ticket[1 - p] = 0;
    c->ntiles[p] = total;
  }
  {  // clear the look-back words of the previous iteration
    const unsigned long long prev = c->ntiles[1 - p] * NV;
    unsigned long long* d = a.desc[1 - p];
    for (unsigned long long i = (unsigned long long)blockIdx.x * T + threadIdx.x; i < prev;
         i += (unsigned long long)gridDim.x * T)
      d[i] = 0;
  }
  if (blockIdx.x >= total) return;
  if (lds_tally) tally_init(tl);
  else cache_init(tc);
  if (threadIdx.x == 0) ss.waves = ss.waves_div = ss.off_mode = ss.surv[0] = ss.surv[1] = ss.surv[2] = 0;
  if (ADEPT_PHASE_CLOCKS && threadIdx.x < kPhases) ph_acc[threadIdx.x] = 0;
  __syncthreads();
  const int lane = __lane_id();
  // Tiles are claimed in ticket order when a block is ready to start one, so
  // that a tile's predecessors are as far along as it is.
  if (threadIdx.x == 0)
    sh.ticket = __hip_atomic_fetch_add(&c->ticket[p], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  pt.mark(ph_acc, 5);
  for (;;) {
    const unsigned long long tile = sh.ticket;
    if (tile >= total) break;
    int D;
    unsigned long long lt, nD;
    if (tile < t0) { D = ELECTRON; lt = tile; nD = n0; }
    else if (tile < t0 + t1) { D = POSITRON; lt = tile - t0; nD = n1; }
    else { D = GAMMA; lt = tile - t0 - t1; nD = n2; }
    const int bcur = SCHEME == DENSE ? (int)p : 0;
    const auto Acur = make_acc<MAP, P, INSTR>(a, D, bcur, counting);
    uint32_t cnt[NS];
#pragma unroll
    for (int v = 0; v < NS; ++v) cnt[v] = 0;
    DivCount dk{0u, 0u, 0u, 0u};
    // state of the lane's last track of the tile (the earlier ones are parked)
    Track<R> t;
    Creations<R> cr;
    bool surv = false, valid = false;
    uint64_t aux = 0;  // dense: parent id of a survivor; sparse: slot
#pragma unroll
    for (int u = 0; u < TPT; ++u) {
      const unsigned long long idx = lt * TT + (unsigned long long)u * T + threadIdx.x;
      valid = idx < nD;
      cr.n = 0;
      cr.meta = 0;
      surv = false;
      aux = 0;
      Deposits dep{0.0, 0.0, 0.0, 0.0, {0.0, 0.0}};
      int lim_code = 0;
      uint32_t slot = 0;
      if (valid) {
        slot = SCHEME == DENSE ? (uint32_t)idx : a.list[D][p][idx];
        load_track<MAP, P, INSTR>(Acur, slot, t);
        const int v0 = t.vol;
        surv = D == GAMMA ? step_photon<P>(t, cr, dep) : step_charged<P>(t, D, cr, dep);
        lim_code = (surv ? 1 : 0) | (cr.n << 1);
        book(a, lds_tally ? &tl : nullptr, lds_tally ? nullptr : &tc, t.event, v0, dep, t.pos);
      }
      div_count(dk, valid, surv, lim_code, a.off_mode_on != 0);
      // output counts of this track (constant indices only: the arrays stay in registers)
      if (valid) {
        uint32_t cc[3];
        creation_counts(cr, cc);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const uint32_t c_new = cc[d];
          cnt[u * NV + d] = c_new + ((surv && D == d) ? 1u : 0u);
          if (SCHEME == SPARSE) {
            cnt[u * NV + 3 + d] = c_new;
            cnt[u * NV + 6 + d] = (!surv && D == d) ? 1u : 0u;
          }
        }
      }
      // a dense survivor's record is copied whole: its parent id is read here so
      // that the load overlaps the rest of the tile's work
      if (SCHEME == DENSE) {
        if (valid && surv) aux = Acur.template ld<uint64_t>(slot, 9);
      } else {
        aux = slot;
      }
      if constexpr (TPT > 1) {
        if (u < TPT - 1) park(pk, threadIdx.x, t, cr, surv, valid, aux);
      }
    }
    div_flush(ss, dk, D);
    pt.mark(ph_acc, 0);
    uint32_t lex[NS];
    unsigned long long aggw[(NS + 2) / 3];
    block_scan<NS>(cnt, lex, aggw, sh);
    pt.mark(ph_acc, 1);
    unsigned long long agg = 0;  // lane v < NV: the tile aggregate of value v
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      unsigned long long sum = 0;
#pragma unroll
      for (int u = 0; u < TPT; ++u) sum += agg_value<NS>(aggw, u * NV + v);
      if (lane == v) agg = sum;
    }
    lookback<NV>(a.desc[p], tile, agg, sh, &c->overflow);
    __syncthreads();
    pt.mark(ph_acc, 2);
    if (tile == total - 1 && threadIdx.x < NV)
      c->tot[p][threadIdx.x] = sat_add(sh.tile_excl[threadIdx.x], sh.tile_agg[threadIdx.x]);

    // Writes of one track u of this lane: survivor, kill, creations.
    auto emit = [&](int u, const Track<R>& t, const Creations<R>& cr, bool surv, uint64_t aux) {
      // tile-local exclusive prefix of value v for this track: the outputs of the
      // lane's earlier tracks' sub-tiles come first
      auto base = [&](int v) -> uint32_t {
        uint32_t b = 0;
#pragma unroll
        for (int w = 0; w < TPT; ++w)
          if (w < u) b += agg_value<NS>(aggw, w * NV + v);
        return b + lex[u * NV + v];
      };
      const uint32_t n_step = t.ctr - (surv ? 1u : 0u);  // a survivor leaves with the next counter
      const int ncr = cr.n;
      // running position of this track's next output of each type (next list / dense index)
      uint32_t k0 = base(0), k1 = base(1), k2 = base(2);
      auto next_pos = [&](int d) -> unsigned long long {
        const uint32_t r = d == 0 ? k0 : (d == 1 ? k1 : k2);
        k0 += d == 0 ? 1u : 0u;
        k1 += d == 1 ? 1u : 0u;
        k2 += d == 2 ? 1u : 0u;
        return sh.tile_excl[d] + r;
      };
      if (SCHEME == DENSE) {
        const int bn = 1 - (int)p;
        if (surv) {
          const unsigned long long pos = next_pos(D);
          if (pos < a.C) {
            const auto An = make_acc<MAP, P, INSTR>(a, D, bn, counting);
            store_full<MAP, P, INSTR>(An, pos, t.pos, t.dir, t.E, t.nl, t.id, aux, t.seed, t.ctr, t.vol, t.event);
          } else {
            atomicOr(&c->overflow, 1ull);
          }
        }
#pragma unroll 1
        for (int i = 0; i < ncr; ++i) {  // one copy of the record store for every creation
          const int d = cr.type(i);
          const unsigned long long pos = next_pos(d);
          if (pos < a.C) write_creation<MAP, P, INSTR>(a, d, bn, pos, counting, t, cr, i, n_step);
          else atomicOr(&c->overflow, 1ull);
        }
      } else {
        const uint32_t slot = (uint32_t)aux;
        uint32_t m0 = base(SCHEME == SPARSE ? 3 : 0), m1 = base(SCHEME == SPARSE ? 4 : 1),
                 m2 = base(SCHEME == SPARSE ? 5 : 2);
        if (surv) {
          const unsigned long long pos = next_pos(D);
          store_inplace<MAP, P, INSTR>(Acur, slot, t, D != GAMMA);
          if (pos < a.C) a.list[D][1 - p][pos] = slot;
        } else {
          const uint32_t lk = D == 0 ? base(SCHEME == SPARSE ? 6 : 0)
                                     : (D == 1 ? base(SCHEME == SPARSE ? 7 : 0) : base(SCHEME == SPARSE ? 8 : 0));
          const unsigned long long f = sh.tile_excl[6 % NV + (SCHEME == SPARSE ? D : 0)] + lk;
          a.ring[D][(c->head[D] + c->count[D] + f) % a.C] = slot;
        }
#pragma unroll 1
        for (int i = 0; i < ncr; ++i) {
          const int d = cr.type(i);
          const unsigned long long pos = next_pos(d);
          const uint32_t r = d == 0 ? m0 : (d == 1 ? m1 : m2);
          m0 += d == 0 ? 1u : 0u;
          m1 += d == 1 ? 1u : 0u;
          m2 += d == 2 ? 1u : 0u;
          const unsigned long long j = sh.tile_excl[(SCHEME == SPARSE ? 3 : 0) + d] + r;
          if (j < c->count[d] && pos < a.C) {
            const uint32_t s = a.ring[d][(c->head[d] + j) % a.C];
            write_creation<MAP, P, INSTR>(a, d, 0, s, counting, t, cr, i, n_step);
            a.list[d][1 - p][pos] = s;
          } else {
            atomicOr(&c->overflow, 1ull);
          }
        }
      }
    };
    if (valid) emit(TPT - 1, t, cr, surv, aux);
    if constexpr (TPT > 1) {
#pragma unroll
      for (int u = 0; u < TPT - 1; ++u) {
        unpark(pk, threadIdx.x, t, cr, surv, valid, aux);
        if (valid) emit(u, t, cr, surv, aux);
      }
    }
    pt.mark(ph_acc, 3);
    // Every read of this tile's LDS state is done.  The next ticket is taken only
    // now, when the block can start on it at once: a tile claimed while its block
    // is still writing holds up the look-back of every later tile.
    __syncthreads();
    if (threadIdx.x == 0)
      sh.ticket = __hip_atomic_fetch_add(&c->ticket[p], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    pt.mark(ph_acc, 4);
  }
  if (lds_tally) flush(a, tl);
  else cache_flush(a, tc);
  __syncthreads();
  pt.mark(ph_acc, 6);
  if (ADEPT_PHASE_CLOCKS) {
    __syncthreads();
    if (threadIdx.x < kPhases && ph_acc[threadIdx.x]) atomicAdd(&c->phase[threadIdx.x], ph_acc[threadIdx.x]);
  }
  if (threadIdx.x == 0) {
    atomicAdd(&c->waves, ss.waves);
    if (ss.waves_div) atomicAdd(&c->waves_div, ss.waves_div);
    if (ss.off_mode) atomicAdd(&c->off_mode, ss.off_mode);
    for (int d = 0; d < 3; ++d)
      if (ss.surv[d]) atomicAdd(&c->surv[d], ss.surv[d]);
  }
}

// ---------------------------------------------------------------------------
// Wavefront tiles: the same iteration with one compaction tile per wavefront
// (TPT * 64 consecutive tracks of one type) instead of one per block.  A
// wavefront claims its tile from the ticket counter, steps it, scans its output
// counts with DPP, resolves the tile's global offsets by its own decoupled
// look-back, and writes; it never waits for the other wavefronts of its block,
// so a wavefront that polls its predecessors (asleep between polls) leaves the
// CU's issue slots to the block's other wavefronts, which go on stepping.
// The canonical order, and hence every slot, is the one of the block tiles.
// ---------------------------------------------------------------------------

// Decoupled look-back of one wavefront: lane v < NV holds the tile aggregate of
// value v on entry and receives its exclusive prefix.  Same descriptor words and
// spin bound as `lookback`; polls are spaced by s_sleep.
template <int NV>
__device__ __forceinline__ unsigned long long lookback_wave(unsigned long long* desc, unsigned long long tile,
                                                            unsigned long long agg, unsigned long long* err) {
  const int lane = __lane_id();
  if (tile == 0) {
    if (lane < NV) st_agent(&desc[lane], kStP | (agg << 31) | agg);
    return 0;
  }
  if (lane < NV) st_agent(&desc[tile * NV + lane], kStA | agg);
  unsigned long long acc[NV];
  long long base[NV];
  bool done[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    acc[v] = 0;
    base[v] = (long long)tile - 1;
    done[v] = false;
  }
  for (unsigned polls = 0;; ++polls) {
    if (polls >= kSpinLimit) {
      if (lane == 0) atomicOr(err, 2ull);
      break;
    }
    bool all_done = true, waiting = false;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      if (done[v]) continue;
      const long long j = base[v] - lane;
      const unsigned long long w = j >= 0 ? ld_agent(&desc[(unsigned long long)j * NV + v]) : kStP;
      const unsigned long long st = w >> 62;
      const unsigned long long pm = __ballot(st == 2);
      const unsigned long long xm = __ballot(st == 0);
      const int fp = pm ? __ffsll((long long)pm) - 1 : 64;
      const unsigned long long need = fp >= 63 ? ~0ull : ((2ull << fp) - 1);
      if (xm & need) {
        all_done = false;
        waiting = true;
        continue;
      }
      unsigned long long val = 0;
      if (lane < fp) val = w & kSat;
      else if (lane == fp) val = (w >> 31) & kSat;
      acc[v] = sat_add(acc[v], wave_sum(val));
      if (fp < 64) done[v] = true;
      else {
        base[v] -= 64;
        all_done = false;
      }
    }
    if (all_done) break;
    if (waiting) __builtin_amdgcn_s_sleep(2);
  }
  unsigned long long ex = 0;
#pragma unroll
  for (int v = 0; v < NV; ++v)
    if (v == lane) ex = acc[v];
  if (lane < NV) st_agent(&desc[tile * NV + lane], kStP | (sat_add(ex, agg) << 31) | agg);
  return ex;
}

// 64-bit value of lane 0, uniform.
__device__ __forceinline__ unsigned long long first_lane_u64(unsigned long long x) {
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
  return ((unsigned long long)hi << 32) | lo;
}

// Tile tickets of the wavefront-tile kernel.  A device-scope atomic on one
// address completes only some tens of millions of times per second, fewer than
// the wavefront tiles a launch gets through, so the block claims kBatch
// consecutive tiles per atomic and hands them to its wavefronts in claim order
// through LDS.  The wavefront that opens batch j (claim index kBatch j) takes it from
// the device counter; the others wait for its base in ring entry j mod kRing.
// An entry is reused only after every claim of the batch it held was served.
#ifndef ADEPT_WAVE_BATCH
#define ADEPT_WAVE_BATCH 16
#endif
constexpr unsigned kBatch = ADEPT_WAVE_BATCH, kRing = 4;
struct WaveTickets {
  unsigned int claims;
  unsigned int gen[kRing];      // batch number + 1 of the base the entry holds
  unsigned int served[kRing];   // claims of that batch that have read it
  unsigned long long base[kRing];
};

__device__ __forceinline__ void tickets_init(WaveTickets& wt) {
  if (threadIdx.x == 0) {
    wt.claims = 0;
    for (unsigned e = 0; e < kRing; ++e) {
      wt.gen[e] = 0;
      wt.served[e] = 0;
      wt.base[e] = 0;
    }
  }
}

__device__ __forceinline__ unsigned long long claim_wave_tile(WaveTickets& wt, unsigned long long* ticket) {
  const int lane = __lane_id();
  unsigned k = 0;
  if (lane == 0) k = atomicAdd(&wt.claims, 1u);
  k = (unsigned)__builtin_amdgcn_readfirstlane((int)k);
  const unsigned j = k / kBatch, slot = k % kBatch, e = j % kRing;
  if (slot == 0) {
    if (j >= kRing)
      while (__hip_atomic_load(&wt.served[e], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < kBatch)
        __builtin_amdgcn_s_sleep(1);
    unsigned long long b = 0;
    if (lane == 0) b = __hip_atomic_fetch_add(ticket, (unsigned long long)kBatch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    b = first_lane_u64(b);
    if (lane == 0) {
      wt.base[e] = b;
      wt.served[e] = 0;
      __hip_atomic_store(&wt.gen[e], j + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
  } else {
    while (__hip_atomic_load(&wt.gen[e], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) != j + 1)
      __builtin_amdgcn_s_sleep(1);
  }
  const unsigned long long b = first_lane_u64(wt.base[e]);
  if (lane == 0) __hip_atomic_fetch_add(&wt.served[e], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
  return b + slot;
}

// Writes of one stepped track: the survivor (dense: the whole record into the
// next buffer; sparse: in place, its slot into the next list, or the freed slot
// into the ring) and its creations.  pos(v) gives the global position of the
// track's next output of value v and advances it (v < 3: next array / next list
// of type v; sparse 3 + d: ring allocations of type d; 6 + d: slots freed).
template <int SCHEME, int MAP, class P, bool INSTR, class Pos>
__device__ __forceinline__ void emit_track(const KArgs& a, Ctrl* c, uint32_t p, int D,
                                           const Acc<MAP, P::mixed, INSTR>& Acur, bool counting,
                                           const Track<typename P::R>& t, const Creations<typename P::R>& cr,
                                           bool surv, uint64_t aux, Pos&& pos) {
  const uint32_t n_step = t.ctr - (surv ? 1u : 0u);  // a survivor leaves with the next counter
  const int ncr = cr.n;
  if constexpr (SCHEME == DENSE) {
    const int bn = 1 - (int)p;
    if (surv) {
      const unsigned long long q = pos(D);
      if (q < a.C) {
        const auto An = make_acc<MAP, P, INSTR>(a, D, bn, counting);
        store_full<MAP, P, INSTR>(An, q, t.pos, t.dir, t.E, t.nl, t.id, aux, t.seed, t.ctr, t.vol, t.event);
      } else {
        atomicOr(&c->overflow, 1ull);
      }
    }
#pragma unroll 1
    for (int i = 0; i < ncr; ++i) {
      const int d = cr.type(i);
      const unsigned long long q = pos(d);
      if (q < a.C) write_creation<MAP, P, INSTR>(a, d, bn, q, counting, t, cr, i, n_step);
      else atomicOr(&c->overflow, 1ull);
    }
  } else {
    const uint32_t slot = (uint32_t)aux;
    if (surv) {
      const unsigned long long q = pos(D);
      store_inplace<MAP, P, INSTR>(Acur, slot, t, D != GAMMA);
      if (q < a.C) a.list[D][1 - p][q] = slot;
    } else {
      const unsigned long long f = pos(6 + D);
      a.ring[D][(c->head[D] + c->count[D] + f) % a.C] = slot;
    }
#pragma unroll 1
    for (int i = 0; i < ncr; ++i) {
      const int d = cr.type(i);
      const unsigned long long q = pos(d);
      const unsigned long long j = pos(3 + d);
      if (j < c->count[d] && q < a.C) {
        const uint32_t s = a.ring[d][(c->head[d] + j) % a.C];
        write_creation<MAP, P, INSTR>(a, d, 0, s, counting, t, cr, i, n_step);
        a.list[d][1 - p][q] = s;
      } else {
        atomicOr(&c->overflow, 1ull);
      }
    }
  }
}

template <int SCHEME, int MAP, class P, bool INSTR, int LB>
__global__ void __launch_bounds__(LB) ADEPT_STEP_ATTR k_step_wave(const KArgs a) {
  using R = typename P::R;
  constexpr int NV = SCHEME == DENSE ? 3 : 9;
  constexpr int TPT = P::tracks_per_lane(LB);
  constexpr int NS = NV * TPT;
  constexpr int W = (NS + 2) / 3;  // 32-bit words of three 10-bit counts
  __shared__ Park<R, (TPT > 1)> pk;
  __shared__ TallyLDS tl;
  __shared__ TallyCache<P::tally_cache_bits> tc;
  __shared__ StatLDS ss;
  __shared__ WaveTickets wt;
  __shared__ unsigned long long ph_acc[kPhases];
  PhaseTimer pt;
  pt.start();
  Ctrl* c = a.ctrl;
  const uint32_t p = c->parity;
  const unsigned long long n0 = c->n[p][0], n1 = c->n[p][1], n2 = c->n[p][2];
  constexpr unsigned long long TT = 64ull * TPT;
  const unsigned long long t0 = ceil_div(n0, TT), t1 = ceil_div(n1, TT), t2 = ceil_div(n2, TT);
  const unsigned long long total = t0 + t1 + t2;
  const unsigned long long T = blockDim.x;
  const bool counting = INSTR && a.instr_on && c->iter < a.instr_last;
  const bool lds_tally = a.n_events == 1 && !a.cells;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    c->ticket[1 - p] = 0;
    c->ntiles[p] = total;
  }
  {  // clear the look-back words of the previous iteration
    const unsigned long long prev = c->ntiles[1 - p] * NV;
    unsigned long long* d = a.desc[1 - p];
    for (unsigned long long i = (unsigned long long)blockIdx.x * T + threadIdx.x; i < prev;
         i += (unsigned long long)gridDim.x * T)
      d[i] = 0;
  }
  if ((unsigned long long)blockIdx.x * (T / 64) >= total) return;
  if (lds_tally) tally_init(tl);
  else cache_init(tc);
  if (threadIdx.x == 0) ss.waves = ss.waves_div = ss.off_mode = ss.surv[0] = ss.surv[1] = ss.surv[2] = 0;
  tickets_init(wt);
  if (ADEPT_PHASE_CLOCKS && threadIdx.x < kPhases) ph_acc[threadIdx.x] = 0;
  __syncthreads();
  const int lane = __lane_id();
  unsigned long long tile = claim_wave_tile(wt, &c->ticket[p]);
  pt.mark(ph_acc, 5);
  while (tile < total) {
    int D;
    unsigned long long lt, nD;
    if (tile < t0) { D = ELECTRON; lt = tile; nD = n0; }
    else if (tile < t0 + t1) { D = POSITRON; lt = tile - t0; nD = n1; }
    else { D = GAMMA; lt = tile - t0 - t1; nD = n2; }
    const int bcur = SCHEME == DENSE ? (int)p : 0;
    const auto Acur = make_acc<MAP, P, INSTR>(a, D, bcur, counting);
    uint32_t cnt[NS];
#pragma unroll
    for (int v = 0; v < NS; ++v) cnt[v] = 0;
    Track<R> t;
    Creations<R> cr;
    bool surv = false, valid = false;
    uint64_t aux = 0;
#pragma unroll
    for (int u = 0; u < TPT; ++u) {
      const unsigned long long idx = lt * TT + (unsigned long long)u * 64 + lane;
      valid = idx < nD;
      cr.n = 0;
      cr.meta = 0;
      surv = false;
      aux = 0;
      Deposits dep{0.0, 0.0, 0.0, 0.0, {0.0, 0.0}};
      int lim_code = 0;
      uint32_t slot = 0;
      if (valid) {
        slot = SCHEME == DENSE ? (uint32_t)idx : a.list[D][p][idx];
        load_track<MAP, P, INSTR>(Acur, slot, t);
        const int v0 = t.vol;
        surv = D == GAMMA ? step_photon<P>(t, cr, dep) : step_charged<P>(t, D, cr, dep);
        lim_code = (surv ? 1 : 0) | (cr.n << 1);
        book(a, lds_tally ? &tl : nullptr, lds_tally ? nullptr : &tc, t.event, v0, dep, t.pos);
      }
      div_stats(ss, D, valid, surv, lim_code, a.off_mode_on != 0);
      if (valid) {
        uint32_t cc[3];
        creation_counts(cr, cc);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const uint32_t c_new = cc[d];
          cnt[u * NV + d] = c_new + ((surv && D == d) ? 1u : 0u);
          if (SCHEME == SPARSE) {
            cnt[u * NV + 3 + d] = c_new;
            cnt[u * NV + 6 + d] = (!surv && D == d) ? 1u : 0u;
          }
        }
      }
      if (SCHEME == DENSE) {
        if (valid && surv) aux = Acur.template ld<uint64_t>(slot, 9);
      } else {
        aux = slot;
      }
      if constexpr (TPT > 1) {
        if (u < TPT - 1) park(pk, threadIdx.x, t, cr, surv, valid, aux);
      }
    }
    pt.mark(ph_acc, 0);
    // wavefront scan of the counts, three 10-bit fields per word (a wavefront's
    // totals stay below 2^10)
    uint32_t lexw[W], totw[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
      uint32_t x = 0;
#pragma unroll
      for (int k = 0; k < 3; ++k)
        if (3 * w + k < NS) x |= cnt[3 * w + k] << (10 * k);
      const uint32_t inc = wave_scan(x);
      lexw[w] = inc - x;
      totw[w] = (uint32_t)__builtin_amdgcn_readlane((int)inc, 63);
    }
    auto field = [&](const uint32_t* words, int s) -> uint32_t { return (words[s / 3] >> (10 * (s % 3))) & 0x3FFu; };
    unsigned long long agg = 0;  // lane v < NV: the tile aggregate of value v
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      uint32_t sum = 0;
#pragma unroll
      for (int u = 0; u < TPT; ++u) sum += field(totw, u * NV + v);
      if (lane == v) agg = sum;
    }
    pt.mark(ph_acc, 1);
    const unsigned long long exl = lookback_wave<NV>(a.desc[p], tile, agg, &c->overflow);
    unsigned long long excl[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) excl[v] = lane_value(exl, v);
    if (tile == total - 1 && lane < NV) c->tot[p][lane] = sat_add(exl, agg);
    pt.mark(ph_acc, 2);
    auto emit_u = [&](int u, const Track<R>& t, const Creations<R>& cr, bool surv,
                      uint64_t aux) __attribute__((always_inline)) {
      // running tile-local position of this track's next output of each value:
      // the lane's earlier tracks' sub-tiles come first
      uint32_t k[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        uint32_t b = 0;
#pragma unroll
        for (int w = 0; w < TPT; ++w)
          if (w < u) b += field(totw, w * NV + v);
        k[v] = b + field(lexw, u * NV + v);
      }
      auto pos = [&](int v) __attribute__((always_inline)) -> unsigned long long {
        unsigned long long r = 0;
#pragma unroll
        for (int x = 0; x < NV; ++x) {
          if (x == v) {
            r = excl[x] + k[x];
            k[x] += 1;
          }
        }
        return r;
      };
      emit_track<SCHEME, MAP, P, INSTR>(a, c, p, D, Acur, counting, t, cr, surv, aux, pos);
    };
    if (valid) emit_u(TPT - 1, t, cr, surv, aux);
    if constexpr (TPT > 1) {
#pragma unroll
      for (int u = 0; u < TPT - 1; ++u) {
        unpark(pk, threadIdx.x, t, cr, surv, valid, aux);
        if (valid) emit_u(u, t, cr, surv, aux);
      }
    }
    pt.mark(ph_acc, 3);
    tile = claim_wave_tile(wt, &c->ticket[p]);
    pt.mark(ph_acc, 4);
  }
  if (lds_tally) flush(a, tl);
  else cache_flush(a, tc);
  __syncthreads();
  pt.mark(ph_acc, 6);
  if (ADEPT_PHASE_CLOCKS) {
    __syncthreads();
    if (threadIdx.x < kPhases && ph_acc[threadIdx.x]) atomicAdd(&c->phase[threadIdx.x], ph_acc[threadIdx.x]);
  }
  if (threadIdx.x == 0) {
    atomicAdd(&c->waves, ss.waves);
    if (ss.waves_div) atomicAdd(&c->waves_div, ss.waves_div);
    if (ss.off_mode) atomicAdd(&c->off_mode, ss.off_mode);
    for (int d = 0; d < 3; ++d)
      if (ss.surv[d]) atomicAdd(&c->surv[d], ss.surv[d]);
  }
}

// ---------------------------------------------------------------------------
// Injection: primaries [inj_begin, inj_end) of the staged array pass through the
// creation path in input order and are appended after the current tracks.
// ---------------------------------------------------------------------------
template <int SCHEME, int MAP, class P, bool INSTR>
__global__ void __launch_bounds__(kMaxBlock) k_inject(const KArgs a) {
  using R = typename P::R;
  constexpr int NV = 3;
  __shared__ Scan<NV> sh;
  Ctrl* c = a.ctrl;
  const uint32_t p = c->parity, q = c->inj_parity;
  const unsigned long long begin = c->inj_begin, end = c->inj_end;
  const unsigned long long T = blockDim.x;
  const unsigned long long total = ceil_div(end - begin, T);
  const bool counting = INSTR && a.instr_on && c->iter < a.instr_last;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    c->inj_ticket[1 - q] = 0;
    c->inj_ntiles[q] = total;
  }
  {
    const unsigned long long prev = c->inj_ntiles[1 - q] * NV;
    unsigned long long* d = a.idesc[1 - q];
    for (unsigned long long i = (unsigned long long)blockIdx.x * T + threadIdx.x; i < prev;
         i += (unsigned long long)gridDim.x * T)
      d[i] = 0;
  }
  if (blockIdx.x >= total) return;
  for (;;) {
    if (threadIdx.x == 0)
      sh.ticket = __hip_atomic_fetch_add(&c->inj_ticket[q], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const unsigned long long tile = sh.ticket;
    if (tile >= total) break;
    const unsigned long long idx = begin + tile * T + threadIdx.x;
    const bool valid = idx < end;
    Track<R> t;
    Creations<R> cr;
    cr.n = 0;
    cr.meta = 0;
    Deposits dep{0.0, 0.0, 0.0, 0.0, {0.0, 0.0}};
    int type = 0;
    bool keep = false;
    double ein = 0.0, ein2 = 0.0, rnd = 0.0;  // input energy, positron rest mass, rounding residual
    uint32_t evk = 0;
    if (valid) {
      const adept_primary q0 = a.staged[idx];
      type = q0.type;
      const uint32_t ev = q0.event;
      evk = ev;
      t.pos[0] = q0.pos[0];
      t.pos[1] = q0.pos[1];
      t.pos[2] = q0.pos[2];
#pragma unroll
      for (int k = 0; k < 3; ++k) t.dir[k] = (R)q0.dir[k];
      t.E = (R)q0.E;
      t.nl = (R)q0.numIALeft;
      t.id = q0.trackId;
      t.parent = ~0ull;
      t.seed = a.seeds[ev];
      t.ctr = 0;
      t.vol = locate(q0.pos[2]);
      t.event = ev;
      ein = q0.E;
      if (type == POSITRON) ein2 = 2.0 * (double)Consts<R>::me;
      if (P::mixed) rnd = q0.E - (double)t.E;
      const bool subcut = type == GAMMA ? (t.E < Consts<R>::cut_g) : (t.E < Consts<R>::cut_e);
      if (subcut) {
        dep.cut = (double)t.E;
        if (type == POSITRON) {
          const Creator<P> X{t.seed, t.id, 0u, 0};
          int kidx = 0;
          annihilate<P>(track_block<P::philox_unroll>(X.seed, X.id, X.n, 1u), X, &kidx, 0, cr);
        }
        book<TallyCache<P::tally_cache_bits>>(a, nullptr, nullptr, ev, t.vol, dep, t.pos);
      } else {
        keep = true;
      }
    }
    // energy ledger of the event, reduced per wavefront (every lane is active here)
    wave_gadd_keyed(a.ein, evk, ein);
    wave_gadd_keyed(a.ein, evk, ein2);
    if (P::mixed) wave_gadd_keyed(a.rnd, evk, rnd);
    uint32_t cnt[NV] = {0, 0, 0};
    if (valid) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        uint32_t c_ = (keep && type == d) ? 1u : 0u;
#pragma unroll
        for (int i = 0; i < 3; ++i) c_ += (i < cr.n && cr.type(i) == d) ? 1u : 0u;
        cnt[d] = c_;
      }
    }
    uint32_t lex[NV];
    unsigned long long aggw[1];
    block_scan<NV>(cnt, lex, aggw, sh);
    unsigned long long agg = 0;
#pragma unroll
    for (int v = 0; v < NV; ++v)
      if (__lane_id() == v) agg = agg_value<NV>(aggw, v);
    lookback<NV>(a.idesc[q], tile, agg, sh, &c->overflow);
    __syncthreads();
    if (tile == total - 1 && threadIdx.x < NV)
      c->inj_tot[threadIdx.x] = sat_add(sh.tile_excl[threadIdx.x], sh.tile_agg[threadIdx.x]);
    if (valid) {
      uint32_t k0 = lex[0], k1 = lex[1], k2 = lex[2];
      const int b = SCHEME == DENSE ? (int)p : 0;
      const int nout = (keep ? 1 : 0) + cr.n;
#pragma unroll
      for (int o = 0; o < 3; ++o) {
        if (o >= nout) continue;
        const int d = keep ? type : cr.type(o);
        const uint32_t r = d == 0 ? k0 : (d == 1 ? k1 : k2);
        k0 += d == 0 ? 1u : 0u;
        k1 += d == 1 ? 1u : 0u;
        k2 += d == 2 ? 1u : 0u;
        const unsigned long long j = sh.tile_excl[d] + r;
        unsigned long long s;
        bool ok;
        if (SCHEME == DENSE) {
          s = c->n[p][d] + j;
          ok = s < a.C;
        } else {
          ok = j < c->count[d] && c->n[p][d] + j < a.C;
          s = ok ? a.ring[d][(c->head[d] + j) % a.C] : 0;
          if (ok) a.list[d][p][c->n[p][d] + j] = (uint32_t)s;
        }
        if (!ok) {
          atomicOr(&c->overflow, 1ull);
          continue;
        }
        if (keep) {
          const auto A = make_acc<MAP, P, INSTR>(a, d, b, counting);
          store_full<MAP, P, INSTR>(A, s, t.pos, t.dir, t.E, t.nl, t.id, ~0ull, t.seed, 0u, t.vol, t.event);
        } else {
          write_creation<MAP, P, INSTR>(a, d, b, s, counting, t, cr, o, 0u);
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Debug / parity: gather the current tracks of one type into host-format records.
// ---------------------------------------------------------------------------
template <int SCHEME, int MAP, class P>
__global__ void k_dump(const KArgs a, int type, adept_track_host* out, uint32_t* slots, unsigned long long n) {
  const unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t p = a.ctrl->parity;
  const uint32_t s = SCHEME == DENSE ? (uint32_t)i : a.list[type][p][i];
  const auto A = make_acc<MAP, P, false>(a, type, SCHEME == DENSE ? (int)p : 0, false);
  using R = typename P::R;
  adept_track_host h;
  for (int k = 0; k < 3; ++k) h.pos[k] = A.template ld<double>(s, k);
  for (int k = 0; k < 3; ++k) h.dir[k] = (double)A.template ld<R>(s, 3 + k);
  h.E = (double)A.template ld<R>(s, 6);
  h.numIALeft = (double)A.template ld<R>(s, 7);
  h.trackId = A.template ld<uint64_t>(s, 8);
  h.parentId = A.template ld<uint64_t>(s, 9);
  h.rngSeed = A.template ld<uint32_t>(s, 10);
  h.rngCtr = A.template ld<uint32_t>(s, 11);
  h.volume = A.template ld<int32_t>(s, 12);
  h.event = A.template ld<uint32_t>(s, 13);
  out[i] = h;
  if (slots) slots[i] = s;
}

// Energy of the buffered tracks per event (+ 2 m_e per positron).
template <int SCHEME, int MAP, class P>
__global__ void k_inflight(const KArgs a, double* out) {
  const uint32_t p = a.ctrl->parity;
  using R = typename P::R;
  for (int type = 0; type < 3; ++type) {
    const unsigned long long n = a.ctrl->n[p][type];
    const auto A = make_acc<MAP, P, false>(a, type, SCHEME == DENSE ? (int)p : 0, false);
    for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (unsigned long long)gridDim.x * blockDim.x) {
      const uint32_t s = SCHEME == DENSE ? (uint32_t)i : a.list[type][p][i];
      const uint32_t ev = A.template ld<uint32_t>(s, 13);
      gadd(&out[ev], (double)A.template ld<R>(s, 6));
      if (type == POSITRON) gadd(&out[ev], 2.0 * (double)Consts<R>::me);
    }
  }
}

// Host-side table of the launchers of one (scheme, mapping, precision, instr) variant.
struct Ops {
  // wave: one compaction tile per wavefront (k_step_wave) instead of per block
  void (*step)(const KArgs&, unsigned grid, unsigned block, int wave, hipStream_t);
  void (*inject)(const KArgs&, unsigned grid, unsigned block, hipStream_t);
  void (*dump)(const KArgs&, int type, adept_track_host*, uint32_t*, unsigned long long n, hipStream_t);
  void (*inflight)(const KArgs&, double*, hipStream_t);
};

template <int SCHEME, int MAP, class P, bool INSTR>
struct Variant {
  static void step(const KArgs& a, unsigned grid, unsigned block, int wave, hipStream_t s) {
    if (wave) {
      if (block <= 256)
        hipLaunchKernelGGL((k_step_wave<SCHEME, MAP, P, INSTR, 256>), dim3(grid), dim3(block), 0, s, a);
      else
        hipLaunchKernelGGL((k_step_wave<SCHEME, MAP, P, INSTR, 1024>), dim3(grid), dim3(block), 0, s, a);
    } else if (block <= 256) {
      hipLaunchKernelGGL((k_step<SCHEME, MAP, P, INSTR, 256>), dim3(grid), dim3(block), 0, s, a);
    } else {
      hipLaunchKernelGGL((k_step<SCHEME, MAP, P, INSTR, 1024>), dim3(grid), dim3(block), 0, s, a);
    }
  }
  static void inject(const KArgs& a, unsigned grid, unsigned block, hipStream_t s) {
    hipLaunchKernelGGL((k_inject<SCHEME, MAP, P, INSTR>), dim3(grid), dim3(block), 0, s, a);
  }
  static void dump(const KArgs& a, int type, adept_track_host* out, uint32_t* slots, unsigned long long n,
                   hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL((k_dump<SCHEME, MAP, P>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, type, out,
                       slots, n);
  }
  static void inflight(const KArgs& a, double* out, hipStream_t s) {
    hipLaunchKernelGGL((k_inflight<SCHEME, MAP, P>), dim3(1024), dim3(256), 0, s, a, out);
  }
  static Ops ops() { return Ops{&step, &inject, &dump, &inflight}; }
};

// ops_<scheme>_<precision>(table[map][instr]) are defined one per translation unit.
void ops_sparse_f64(Ops t[4][2]);
void ops_sparse_mixed(Ops t[4][2]);
void ops_dense_f64(Ops t[4][2]);
void ops_dense_mixed(Ops t[4][2]);
void ops_typed(Ops t[2][2][4][2]);  // the per-type mapping of both schemes and precisions

}  // namespace adept
