/*
 * oracle.h -- plain CPU reference of the per-iteration track-transport step.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that tests, the smoke
 * check and the CPU-baseline leg of the benchmark can check the HIP library
 * against an independent, slow, obviously-correct implementation.  No
 * product code path may load it.  It shares no code, header, table or
 * constant with the HIP library; the two only read the same primaries
 * (80-byte records produced by the ``workloads`` package).
 *
 * What it computes (paper: "Challenges and opportunities integrating LLAMA
 * into AdePT", Sec. 2-5):
 *   - the track buffers of Sec. 2: the sparse single buffer (one slot array
 *     per particle type plus a current and a next slot list) and the dense
 *     double buffer (a current and a next dense array per type);
 *   - one transport iteration over every active track of a seeded toy
 *     electromagnetic shower in a 50-layer absorber/gap slab calorimeter
 *     (the stand-in for the Geant4 physics of Sec. 4);
 *   - the record layouts of Sec. 3-4 (AoS, SoA, AoSoA-N) as byte maps;
 *   - the field access counts and per-byte heatmaps of Sec. 5.
 * Every rule it follows is written next to the code that implements it.
 */
#ifndef ADEPT_ORACLE_H
#define ADEPT_ORACLE_H
#include <stddef.h>
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

enum { OR_OK = 0, OR_E_INVALID = -1, OR_E_CAPACITY = -2, OR_E_STATE = -4, OR_E_NOMEM = -5 };
enum { OR_SPARSE = 0, OR_DENSE = 1 };
enum { OR_FP64 = 0, OR_MIXED = 1 };
enum { OR_AOS = 0, OR_SOA = 1, OR_AOSOA = 2 };
enum { OR_ELECTRON = 0, OR_POSITRON = 1, OR_GAMMA = 2 };
enum { OR_T_DEP_CONT = 0, OR_T_DEP_CUT = 1, OR_T_LAYER = 2, OR_T_ESCAPED = 3, OR_T_ROUND = 4,
       OR_T_INFLIGHT = 5, OR_T_CELLS = 6, OR_T_EIN = 7 };

/* A primary as handed in by the caller (80 bytes). */
typedef struct {
  uint32_t event;
  int32_t type;
  double E;
  double pos[3];
  double dir[3];
  double numIALeft;
  uint64_t trackId;
} or_primary;

/* One track record, in value form (96 bytes).  Under the mixed policy the
 * fields dir, E and numIALeft always hold values exactly representable as
 * binary32. */
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
} or_track;

typedef struct {
  uint64_t iterations;
  uint64_t track_steps[3];
  uint64_t peak[3];         /* largest active count of each type seen at an iteration start */
  uint64_t slots_touched[3];/* distinct slots ever written (sparse) / largest dense index + 1 */
  uint64_t error_iter;      /* iteration at which a capacity overflow latched (0: none) */
  int32_t status;
  int32_t pad;
} or_stats;

/* Particle ledger (integers, exact), kept for the invariant pins: every track
 * that enters a type's list (primary or creation, sub-cut ones included) ends
 * in exactly one of escaped / cut / annihilated (positrons) / absorbed by pair
 * production (photons), or is still in flight.  Interactions are counted where
 * each process branch is taken, creations where the creation path runs, deaths
 * where the track dies, so the relations between them check that each process
 * makes the particles it should. */
typedef struct {
  uint64_t primaries[3];  /* injected primaries per type                              */
  uint64_t created[3];    /* tracks made by the creation path per type                */
  uint64_t escaped[3];    /* left the calorimeter                                     */
  uint64_t cut[3];        /* stopped below the cut (electrons, photons)               */
  uint64_t annihilated;   /* positrons that annihilated at rest                       */
  uint64_t absorbed;      /* photons absorbed by pair production                      */
  uint64_t n_brem, n_pair, n_compton, n_annihilation;  /* interactions                */
  uint64_t survivors[3];  /* source tracks that survived their step (all iterations)  */
  uint64_t outputs[3];    /* tracks written into the next buffers (all iterations)    */
  uint64_t off_mode;      /* divergence diagnostic: sources whose outcome (survived?,
                             buffered creations) differs from the most common outcome
                             of their group of 64 consecutive sources of one type in
                             current order (the tracks one wavefront steps together) */
} or_ledger;

typedef struct or_sim or_sim;

or_sim *or_create(int scheme, int precision, uint64_t capacity, uint32_t n_events, const uint32_t *seeds);
void or_destroy(or_sim *s);
int or_set_scoring(or_sim *s, uint32_t nx, uint32_t ny, double pitch);
int or_set_instrumented(or_sim *s, int on, uint64_t last_iter);
int or_set_admission(or_sim *s, int on, double alpha, const double kappa[3], uint64_t hold_iters);
int or_inject(or_sim *s, const or_primary *p, uint64_t n);
int or_stage(or_sim *s, const or_primary *p, uint64_t n);
int or_step(or_sim *s, uint64_t next_counts[3]);
int or_run(or_sim *s, uint64_t max_iter, uint64_t *iters_done);
int or_counts(const or_sim *s, uint64_t n[3]);
int or_tally(const or_sim *s, int kind, double *out, size_t n);
int or_stats_get(const or_sim *s, or_stats *out);
int or_ledger_get(const or_sim *s, or_ledger *out);
int or_dump(const or_sim *s, int type, or_track *out, uint32_t *slots, uint64_t cap, uint64_t *n);
int or_load(or_sim *s, int type, const or_track *trk, const uint32_t *slots, uint64_t n);
int or_ring_get(const or_sim *s, int type, uint32_t *ring, uint64_t *head, uint64_t *count);
int or_ring_set(or_sim *s, int type, const uint32_t *ring, uint64_t head, uint64_t count);
int or_set_iteration(or_sim *s, uint64_t iter, int dense_current_b);
int or_access_totals(const or_sim *s, int type, int buffer, uint64_t reads[14], uint64_t writes[14]);
int or_access_slotleaf(const or_sim *s, int type, int buffer, uint32_t *out, uint64_t n);
int or_heat_words(const or_sim *s, int type, int buffer, int mapping, uint32_t lanes, uint32_t *out, uint64_t n_words);

/* Building blocks, exported for the unit pins. */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double or_u01(uint32_t r);
float or_u01f(uint32_t r);
double or_log(double x);
double or_exp(double x);
void or_sincos(double x, double *s, double *c);
float or_logf(float x);
float or_expf(float x);
void or_sincosf(float x, float *s, float *c);
void or_constants(double *d, float *f);
uint64_t or_leaf_addr(int mapping, uint32_t lanes, int precision, uint64_t capacity, uint64_t slot, int leaf);
uint64_t or_buffer_bytes(int mapping, uint32_t lanes, int precision, uint64_t capacity);
uint32_t or_leaf_size(int precision, int leaf);
uint64_t or_child_id(uint32_t seed, uint64_t parent_id, uint32_t ctr, uint32_t k);
int or_locate(const double pos[3], int32_t *volume);
double or_distance(const double pos[3], const double dir[3], int32_t volume, int32_t *axis);

#ifdef __cplusplus
}
#endif
#endif
