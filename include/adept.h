/*
 * adept.h -- C ABI of the MI355X (gfx950) track-transport library.
 *
 * The library runs the per-iteration transport step of the paper "Challenges
 * and opportunities integrating LLAMA into AdePT" (arXiv 2302.08252) on one
 * GPU: every active electron, positron and photon track is loaded through a
 * switchable record layout (Sec. 3-4: AoS, SoA, AoSoA-N) from one of the two
 * track data structures of Sec. 2 (the sparse single buffer with slot lists,
 * or the dense double buffer), stepped once through a seeded toy
 * electromagnetic shower in a 50-layer absorber/gap calorimeter, and written
 * with its secondaries into the next iteration's buffer by ordered stream
 * compaction.  An instrumented mode counts field reads and writes and builds
 * per-byte heatmaps of the track buffers (Sec. 5).
 *
 * Conventions
 *  - Every function returns adept_status: 0 on success, a negative code on error.
 *  - Host arrays belong to the caller; inputs are copied in before return,
 *    outputs are copied out into caller buffers.  Out-parameters are written
 *    only on success.
 *  - Device memory: either the caller hands in an arena (adept_bind, a device
 *    pointer and size, kept alive by the caller) or the library allocates one
 *    at the first call that needs it.  Either way all work is enqueued on one
 *    HIP stream (the caller's, if bound).  A context is not thread-safe.
 *  - After ADEPT_E_CAPACITY or ADEPT_E_DEVICE the context is failed: only
 *    adept_tally, adept_stats, adept_dump_tracks, adept_last_error and
 *    adept_destroy remain valid.
 *  - Units: mm and MeV.
 */
#ifndef ADEPT_H
#define ADEPT_H
#include <stddef.h>
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t adept_status;
enum {
  ADEPT_OK = 0,
  ADEPT_E_INVALID = -1,     /* bad argument (range, NaN, unknown enum, wrong size)   */
  ADEPT_E_CAPACITY = -2,    /* a buffer overflowed; the iteration is in adept_stats   */
  ADEPT_E_DEVICE = -3,      /* a HIP call failed; see adept_last_error                */
  ADEPT_E_STATE = -4,       /* call not allowed in the context's current state        */
  ADEPT_E_NOMEM = -5,       /* allocation failed or the bound arena is too small      */
  ADEPT_E_UNSUPPORTED = -6  /* option not available in this build                     */
};

typedef struct adept_ctx adept_ctx; /* opaque, owned by the library */

/* Sec. 2: sparse single buffer (slot array + current/next slot lists, free
 * slots recycled through a FIFO ring) or dense double buffer (two dense
 * arrays per particle type, swapped every iteration). */
typedef enum { ADEPT_SPARSE_SINGLE = 0, ADEPT_DENSE_DOUBLE = 1 } adept_scheme;
/* Sec. 3-4: record layouts. */
typedef enum { ADEPT_MAP_AOS = 0, ADEPT_MAP_SOA = 1, ADEPT_MAP_AOSOA = 2 } adept_mapping;
typedef struct {
  int32_t scheme;       /* adept_scheme                                  */
  int32_t mapping;      /* adept_mapping                                 */
  uint32_t aosoa_lanes; /* AoSoA lanes N: a power of two in [2, 256]     */
} adept_layout;

/* FP64: all track arithmetic in binary64.  MIXED: direction, energy and
 * interaction length stored and stepped in binary32; position, boundary
 * distance and energy tallies stay binary64. */
typedef enum { ADEPT_FP64 = 0, ADEPT_MIXED = 1 } adept_precision;
typedef enum { ADEPT_ELECTRON = 0, ADEPT_POSITRON = 1, ADEPT_GAMMA = 2 } adept_particle;

typedef enum {
  ADEPT_T_DEP_CONT = 0, /* [event][volume 0..99] continuous-loss deposits            */
  ADEPT_T_DEP_CUT = 1,  /* [event][volume 0..99] local (below-cut) deposits          */
  ADEPT_T_LAYER = 2,    /* [event][layer 0..49] = continuous + local, both volumes    */
  ADEPT_T_ESCAPED = 3,  /* [event] energy leaving the calorimeter (+ 2 m_e per e+)   */
  ADEPT_T_ROUND = 4,    /* [event] exact rounding residuals of the energy ledger     */
  ADEPT_T_INFLIGHT = 5, /* [event] energy of buffered tracks (+ 2 m_e per e+)        */
  ADEPT_T_CELLS = 6,    /* [layer][ix][iy] deposits summed over events (scoring on)  */
  ADEPT_T_EIN = 7       /* [event] primary energy injected (+ 2 m_e per e+)          */
} adept_tally_kind;

/* A primary (80 bytes).  event indexes the table of adept_set_events (0 if none
 * was set); type is an adept_particle; E finite and > 0; pos inside the
 * calorimeter (0 <= z < 400, |x|, |y| <= 200); dir used as given; numIALeft < 0
 * means "sample at the first step", >= 0 forces it; trackId < 2^63, unique in
 * its event. */
typedef struct {
  uint32_t event;
  int32_t type;
  double E;
  double pos[3];
  double dir[3];
  double numIALeft;
  uint64_t trackId;
} adept_primary;

/* A track as returned by adept_dump_tracks (96 bytes, values widened to double). */
typedef struct {
  double pos[3];
  double dir[3];
  double E;
  double numIALeft;
  uint64_t trackId;
  uint64_t parentId;
  uint32_t rngSeed;
  uint32_t rngCtr;
  int32_t volume;
  uint32_t event;
} adept_track_host;

typedef struct {
  uint64_t iterations;       /* iterations done                                      */
  uint64_t track_steps[3];   /* step-function executions per source type            */
  uint64_t peak[3];          /* largest active count per type at an iteration start */
  uint64_t counts[3];        /* current active counts                                */
  uint64_t error_iter;       /* iteration at which a capacity overflow latched (0)  */
  uint64_t survivors[3];     /* source tracks that survived their step, per type     */
  uint64_t outputs[3];       /* tracks written into next buffers (survivors +
                                buffered creations), per type                        */
  double step_kernel_ms;     /* summed step-kernel time of timed runs (adept_set_timing) */
  uint64_t step_launches;    /* step-kernel launches those milliseconds cover        */
  uint64_t waves;            /* wavefronts that stepped tracks                       */
  uint64_t waves_divergent;  /* ... whose lanes disagreed on the step limiter or the
                                interaction outcome (divergence diagnostic)          */
  uint64_t off_mode;         /* divergence diagnostic: track-steps whose outcome (survived?,
                                buffered creations) differs from the most common outcome
                                of their wavefront (64 consecutive sources of one type)  */
  int32_t status;            /* ADEPT_OK or the latched error                        */
  int32_t pad;
} adept_stats;

/* Launch configuration (autotuner output; also settable by hand). */
typedef struct {
  uint32_t block;       /* threads per block: power of 2, 64-1024 (default 1024)  */
  uint32_t grid;        /* resident blocks (0: library default)                  */
  uint32_t graph_iters; /* iterations captured per hipGraph replay (1..256)      */
  uint32_t wave_tiles;  /* compaction granularity of the step: 0 = one tile per
                           block (block scan, one look-back per block), 1 = one
                           tile per wavefront (each wavefront scans and looks
                           back on its own; no block barrier in the tile loop).
                           Same results either way.                            */
} adept_launch;

/* Create a context (paper Sec. 2: the track data structure, one of its two
 * buffer schemes; Sec. 3-4: the record layout its buffers use).  capacity =
 * slots per particle type and per buffer, in [1, 2^30]; for AoSoA a multiple
 * of aosoa_lanes.  The layout, precision and capacity are fixed for the
 * context's lifetime.  The context owns its host state; device memory comes at
 * the first call that needs it (or from adept_bind).  Errors: ADEPT_E_INVALID
 * (nothing is created, *out untouched), ADEPT_E_DEVICE. */
adept_status adept_create(adept_layout layout, adept_precision precision, uint64_t capacity, adept_ctx** out);

/* Create a context whose particle types keep their tracks in different record
 * layouts (the per-particle-type layouts proposed in Sec. 6): layouts[t] is the
 * mapping of type t's buffers (electron, positron, photon), each validated as
 * by adept_create; the three must name the same scheme.  Every access goes
 * through one general form of the three mappings, so results equal those of
 * adept_create for any choice.  Errors: ADEPT_E_INVALID. */
adept_status adept_create_typed(const adept_layout layouts[3], adept_precision precision, uint64_t capacity,
                                adept_ctx** out);

/* Device bytes the context needs with its current settings (events, scoring,
 * instrumentation).  Valid before adept_bind. */
adept_status adept_arena_bytes(const adept_ctx* ctx, size_t* bytes);

/* Hand in a caller-owned device arena (256-byte aligned, >= adept_arena_bytes)
 * and the HIP stream (hipStream_t, may be NULL for the null stream) on which
 * all work is enqueued.  Must come before the first inject.  The caller keeps
 * both alive until adept_destroy.  Errors: ADEPT_E_NOMEM (too small),
 * ADEPT_E_STATE (already bound or allocated). */
adept_status adept_bind(adept_ctx* ctx, void* dev_arena, size_t bytes, void* hip_stream);

/* Per-event seeds (copied); default is one event with seed 1.  Before bind. */
adept_status adept_set_events(adept_ctx* ctx, uint32_t n_events, const uint32_t* seeds);

/* Per-cell deposit tally: each layer split into nx x ny cells of pitch mm,
 * centred on the beam axis.  Before bind. */
adept_status adept_set_scoring(adept_ctx* ctx, uint32_t nx, uint32_t ny, double pitch_mm);

/* Event admission before each iteration, a capacity guard for batched runs of
 * uneven events (Sec. 4 transports primaries in batches; the rule itself is
 * this library's).  An event's projected peak is ceil(kappa_type * E_event /
 * 1000) tracks of each type (kappa in tracks per GeV, E in MeV); an admitted
 * event keeps it reserved for hold_iters iterations, about the time a shower
 * needs to reach its peak.  Whole events are admitted in order while
 * n_type + reserved_type + projected peak <= alpha * capacity for every type;
 * the first waiting event is always admitted when no track is active.  The
 * rule is a heuristic: a shower that outgrows its projection can still
 * overflow, which adept_step / adept_run report as ADEPT_E_CAPACITY.
 * When on, adept_inject stages primaries instead of injecting them.  Before
 * bind. */
adept_status adept_set_admission(adept_ctx* ctx, int on, double alpha, const double kappa[3],
                                 uint64_t hold_iters);

/* Instrumented mode (Sec. 5): count field reads/writes and per-word accesses
 * of every operation that starts while fewer than last_iter iterations are
 * done.  Before bind. */
adept_status adept_set_instrumented(adept_ctx* ctx, int on, uint64_t last_iter);

/* Launch configuration; invalidates the captured graph. */
adept_status adept_set_launch(adept_ctx* ctx, const adept_launch* launch);
adept_status adept_get_launch(const adept_ctx* ctx, adept_launch* launch);

/* Primaries (copied; paper Sec. 2: new tracks enter the list of active tracks
 * of their particle type, Sec. 4: the benchmark feeds primaries in batches).
 * Without admission they pass through the creation path
 * at once, in input order, appended after the current tracks of their type;
 * with admission they must be grouped by non-decreasing event and wait to be
 * admitted (staging is only allowed before the first iteration).  Errors: ADEPT_E_INVALID (bad primary; nothing is injected),
 * ADEPT_E_CAPACITY. */
adept_status adept_inject(adept_ctx* ctx, const adept_primary* p, uint64_t n);

/* As adept_inject, for primaries already in device memory (80-byte records
 * at dev_p, owned by the caller, read before return).  They are checked on the
 * device; any invalid primary fails the call with nothing injected.  Not
 * available with admission (ADEPT_E_UNSUPPORTED). */
adept_status adept_inject_device(adept_ctx* ctx, const adept_primary* dev_p, uint64_t n);

/* Exactly one iteration (paper Sec. 2: every active track of the current
 * buffer is stepped once and survivors plus secondaries are written to the
 * next buffer / slot list): admission, then one step of every active track;
 * synchronous; next_counts (nullable, 3 host words owned by the caller)
 * receives the active counts per type.  Errors: ADEPT_E_CAPACITY (a next
 * buffer or the free ring overflowed: the context is failed),
 * ADEPT_E_DEVICE, ADEPT_E_STATE. */
adept_status adept_step(adept_ctx* ctx, uint64_t next_counts[3]);

/* Iterate (paper Sec. 2 iterations, Sec. 4: a benchmark run transports every
 * primary to the end of its shower) until no track is active and nothing is
 * staged, or max_iter iterations; iterations replay a captured hipGraph of
 * graph_iters iterations.  iters_done (nullable, caller-owned) receives the
 * iterations done by this call.  Errors as adept_step; on an error the
 * iterations before it stay done. */
adept_status adept_run(adept_ctx* ctx, uint64_t max_iter, uint64_t* iters_done);

/* Copy a tally out (paper Sec. 4: the energy deposited in the layers of the
 * sampling calorimeter; the per-event, per-volume and per-cell forms here):
 * out is a caller-owned host array of n doubles; n must equal the kind's size
 * (see adept_tally_kind), else ADEPT_E_INVALID and out is untouched.  Valid on
 * a failed context too (the state at the failure). */
adept_status adept_tally(adept_ctx* ctx, adept_tally_kind kind, double* out, size_t n);

/* Access counts of one physical buffer (paper Sec. 5: field access counts of
 * the Trace instrumentation and the per-byte Heatmap; buffer 0, or 1 = second
 * dense array): reads/writes per field (14 host words each, nullable) and, if
 * heat_words is not NULL, the per-4-byte-word access counters (a caller-owned
 * host array; n_words must equal the buffer size / 4; every field is a
 * multiple of 4 bytes and 4-aligned, so a word's count is each of its bytes'
 * count).  Zero unless the context is instrumented.  Errors: ADEPT_E_INVALID,
 * ADEPT_E_STATE (no device state yet). */
adept_status adept_access_counts(adept_ctx* ctx, adept_particle t, uint32_t buffer, uint64_t reads[14],
                                 uint64_t writes[14], uint32_t* heat_words, size_t n_words);

/* Access counts of one physical buffer at the granularity the memory system
 * moves (the heatmaps of Sec. 5, per cache line): out[i] is the sum of the
 * per-4-byte-word counters of bytes [i * line_bytes, (i + 1) * line_bytes).
 * line_bytes is 64 or 128; n_lines must equal ceil(buffer bytes / line_bytes).
 * Needs an instrumented context (ADEPT_E_STATE otherwise).  Synchronous;
 * allocates device memory for the reduction. */
adept_status adept_line_heat(adept_ctx* ctx, adept_particle t, uint32_t buffer, uint32_t line_bytes, uint64_t* out,
                             size_t n_lines);

/* The record layouts of Sec. 3 as a byte picture: for bytes [first_byte,
 * first_byte + n) of one track buffer of the given layout, precision and
 * capacity (validated as by adept_create), the field stored there (0-13, in
 * the order of adept_track_host: pos x y z, dir x y z, E, numIALeft, trackId,
 * parentId, rngSeed, rngCtr, volume, event) or -1 for padding or bytes past
 * the buffer's end.  If total_bytes is not NULL it receives the buffer's byte
 * size (what adept_buffer_bytes reports for such a context).  leaf_out may be
 * NULL when n is 0.  Host-only; no context, no device, nothing allocated. */
adept_status adept_layout_map(adept_layout layout, adept_precision precision, uint64_t capacity, uint64_t first_byte,
                              uint64_t n, int8_t* leaf_out, uint64_t* total_bytes);

/* Byte size of one physical track buffer of this context (ADEPT_E_INVALID for
 * a context made by adept_create_typed: use adept_type_buffer_bytes). */
adept_status adept_buffer_bytes(const adept_ctx* ctx, size_t* bytes);

/* Byte size of one physical track buffer of particle type t. */
adept_status adept_type_buffer_bytes(const adept_ctx* ctx, adept_particle t, size_t* bytes);

adept_status adept_stats_get(adept_ctx* ctx, adept_stats* out);

/* The current tracks of one type in current order (dense: array order; sparse:
 * slot-list order) with their slot numbers (slots nullable).  Debug/parity. */
adept_status adept_dump_tracks(adept_ctx* ctx, adept_particle t, adept_track_host* out, uint32_t* slots,
                               uint64_t cap, uint64_t* n);

/* Bytes of the fixed device array that adept_dump_tracks_noalloc stages
 * through (one array per GPU, held until the process ends). */
#define ADEPT_NOALLOC_BYTES (16u << 20)

/* adept_dump_tracks for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same result, staged through the library's fixed per-GPU array of
 * ADEPT_NOALLOC_BYTES instead of buffers allocated per call.  n tracks need
 * ceil(96 n / 256) * 256 bytes, plus 4 n when slots is not NULL; a dump that
 * needs more fails with ADEPT_E_INVALID (and *n = the track count), nothing
 * copied.  Allocates nothing on the device and calls no allocating routine.
 * Every call on one GPU shares that GPU's array: calls that overlap on one GPU
 * (from several host threads or contexts) race and must be serialised by the
 * caller.  Synchronous. */
adept_status adept_dump_tracks_noalloc(adept_ctx* ctx, adept_particle t, adept_track_host* out, uint32_t* slots,
                                       uint64_t cap, uint64_t* n);

/* Sparse scheme: the free-slot ring of one type, its head and free count. */
adept_status adept_dump_ring(adept_ctx* ctx, adept_particle t, uint32_t* ring, uint64_t cap, uint64_t* head,
                             uint64_t* count);

/* Reset to the state right after creation+bind (tracks, ring, tallies,
 * counters, staged primaries) without reallocating. */
adept_status adept_reset(adept_ctx* ctx);

/* Pick the launch configuration (block size, graph iterations and the
 * compaction granularity: block tiles of 64-1024 threads, or wavefront tiles
 * in blocks of 1024) for this context by timing runs of the given primaries on
 * scratch state; the context is reset afterwards.  Candidates are tried block tiles first, smaller blocks first; a
 * later candidate wins only if it is 2% faster.  result (nullable) receives
 * the choice. */
adept_status adept_autotune(adept_ctx* ctx, const adept_primary* p, uint64_t n, adept_launch* result);

/* The lane-weighted divergence diagnostic (adept_stats.off_mode), on by default;
 * counting it costs about 1% of the step kernel, so timed runs may switch it
 * off.  Takes effect from the next iteration. */
adept_status adept_set_divergence_count(adept_ctx* ctx, int on);

/* Timed mode for measurements: adept_run launches iterations one by one with
 * HIP events around every step kernel and accumulates their durations into
 * adept_stats (step_kernel_ms, step_launches); resets the accumulators. */
adept_status adept_set_timing(adept_ctx* ctx, int on);

/* Cycle breakdown of the step kernel (a diagnostic): the shader-clock cycles
 * every wavefront spent in each phase of its tiles, summed over all step launches
 * since the last reset: out[0] loading and stepping the tracks, [1] the block
 * scan with the wait for the block's slowest wavefront, [2] the decoupled
 * look-back for the tile's offsets with its barrier, [3] writing the next
 * buffers, [4] the end of a tile (barriers, next ticket), [5] before the first
 * tile, [6] after the last one, [7] unused.  All zero unless the library was
 * built with ADEPT_PHASE_CLOCKS=1 (build.py --define ADEPT_PHASE_CLOCKS=1);
 * out is 8 host words owned by the caller.  Errors: ADEPT_E_INVALID,
 * ADEPT_E_DEVICE. */
adept_status adept_phase_clocks(adept_ctx* ctx, uint64_t out[8]);

/* Layout autotuner: for every candidate layout, a scratch context (library-
 * owned memory, the given precision, capacity and event seeds) is tuned with
 * adept_autotune on the given primaries and the tuned configuration is timed on
 * one more run; the fastest layout wins (an earlier candidate wins unless a
 * later one is more than 2% faster).  Results never depend on the choice. */
adept_status adept_autotune_layout(adept_precision precision, uint64_t capacity, const adept_layout* candidates,
                                   uint32_t n_candidates, uint32_t n_events, const uint32_t* seeds,
                                   const adept_primary* p, uint64_t n, adept_layout* best_layout,
                                   adept_launch* best_launch, double* best_ms);

/* Per-type layout autotuner (Sec. 6): the candidates (one scheme) are first
 * timed as a layout shared by all types, each with its tuned launch, as in
 * adept_autotune_layout; then, in the order electron, positron, photon, each
 * type moves to another candidate when that makes the whole run more than 2%
 * faster (with the launch of the best shared layout).  Contexts made with
 * adept_create_typed; best[t] receives the layout of type t.  Results never
 * depend on the choice. */
adept_status adept_autotune_type_layouts(adept_precision precision, uint64_t capacity, const adept_layout* candidates,
                                         uint32_t n_candidates, uint32_t n_events, const uint32_t* seeds,
                                         const adept_primary* p, uint64_t n, adept_layout best[3],
                                         adept_launch* best_launch, double* best_ms);

/* Last error message of this context (valid until the next call on it). */
const char* adept_last_error(const adept_ctx* ctx);

/* Destroy the context (accepts NULL); frees library-owned memory only. */
void adept_destroy(adept_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
