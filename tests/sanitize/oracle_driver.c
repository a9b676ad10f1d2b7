/* Drives every entry point of the oracle (dense and sparse buffers, both
 * precision policies, admission of staged events, cell scoring,
 * instrumentation, state hand-over, a capacity overflow) so that a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer checks its memory handling:
 * the growing output and kill arrays, the dense buffers reallocated on demand,
 * the free-slot ring indices and the per-(slot, field) counters. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define CHECK(x)                                                   \
  do {                                                             \
    if (!(x)) {                                                    \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #x); \
      return 1;                                                    \
    }                                                              \
  } while (0)

static void prim(or_primary *p, uint32_t ev, int type, double E, uint64_t id) {
  memset(p, 0, sizeof(*p));
  p->event = ev;
  p->type = type;
  p->E = E;
  p->dir[2] = 1.0;
  p->numIALeft = -1.0;
  p->trackId = id;
}

static int shower(int scheme, int prec, uint64_t C, int cells, int instr) {
  const uint32_t seeds[3] = {1, 2, 3};
  or_sim *s = or_create(scheme, prec, C, 3, seeds);
  CHECK(s);
  if (cells) CHECK(or_set_scoring(s, 10, 10, 40.0) == OR_OK);
  if (instr) CHECK(or_set_instrumented(s, 1, 8) == OR_OK);
  or_primary p[12];
  for (int i = 0; i < 12; ++i) prim(&p[i], (uint32_t)(i / 4), i % 3, i % 4 == 3 ? 0.05 : 300.0 + 50.0 * i, (uint64_t)i);
  CHECK(or_inject(s, p, 12) == OR_OK);
  uint64_t it = 0;
  CHECK(or_run(s, 1u << 20, &it) == OR_OK);
  CHECK(it > 0);
  double lay[150], cell[5000];
  CHECK(or_tally(s, OR_T_LAYER, lay, 150) == OR_OK);
  if (cells) CHECK(or_tally(s, OR_T_CELLS, cell, 5000) == OR_OK);
  if (instr) {
    uint64_t r[14], w[14];
    for (int t = 0; t < 3; ++t)
      for (int b = 0; b < (scheme == OR_DENSE ? 2 : 1); ++b) {
        CHECK(or_access_totals(s, t, b, r, w) == OR_OK);
        uint64_t nw = or_buffer_bytes(OR_AOSOA, 8, prec, C) / 4;
        uint32_t *h = (uint32_t *)calloc(nw, 4);
        CHECK(or_heat_words(s, t, b, OR_AOSOA, 8, h, nw) == OR_OK);
        free(h);
      }
  }
  or_stats st;
  or_ledger lg;
  CHECK(or_stats_get(s, &st) == OR_OK && or_ledger_get(s, &lg) == OR_OK);
  or_destroy(s);
  return 0;
}

static int admission(int scheme, int prec) {
  const uint32_t seeds[4] = {5, 6, 7, 8};
  or_sim *s = or_create(scheme, prec, 1u << 12, 4, seeds);
  CHECK(s);
  const double kappa[3] = {3.0, 2.0, 25.0};
  CHECK(or_set_admission(s, 1, 0.8, kappa, 16) == OR_OK);
  or_primary p[16];
  for (int i = 0; i < 16; ++i) prim(&p[i], (uint32_t)(i / 4), i % 3, 200.0 + 10.0 * i, (uint64_t)(i % 4));
  CHECK(or_stage(s, p, 16) == OR_OK);
  uint64_t it = 0;
  CHECK(or_run(s, 1u << 20, &it) == OR_OK);
  or_destroy(s);
  return 0;
}

static int overflow_and_handover(int scheme) {
  const uint32_t seed = 1;
  or_sim *s = or_create(scheme, OR_FP64, 64, 1, &seed);
  CHECK(s);
  or_primary p[3];
  for (int i = 0; i < 3; ++i) prim(&p[i], 0, 0, 1000.0, (uint64_t)i);
  CHECK(or_inject(s, p, 3) == OR_OK);
  uint64_t it = 0;
  CHECK(or_run(s, 1u << 20, &it) == OR_E_CAPACITY);
  or_destroy(s);
  /* hand a state to a second context (ring included) and take one step */
  or_sim *a = or_create(scheme, OR_MIXED, 1024, 1, &seed);
  or_sim *b = or_create(scheme, OR_MIXED, 1024, 1, &seed);
  CHECK(a && b);
  CHECK(or_inject(a, p, 3) == OR_OK);
  CHECK(or_run(a, 5, &it) == OR_OK);
  for (int t = 0; t < 3; ++t) {
    uint64_t n[3];
    or_counts(a, n);
    or_track *trk = (or_track *)malloc(sizeof(or_track) * (n[t] + 1));
    uint32_t *sl = (uint32_t *)malloc(4 * (n[t] + 1));
    uint64_t m = 0;
    CHECK(or_dump(a, t, trk, sl, n[t] + 1, &m) == OR_OK && m == n[t]);
    CHECK(or_load(b, t, trk, sl, m) == OR_OK);
    if (scheme == OR_SPARSE) {
      uint32_t *ring = (uint32_t *)malloc(4 * 1024);
      uint64_t head, count;
      CHECK(or_ring_get(a, t, ring, &head, &count) == OR_OK);
      CHECK(or_ring_set(b, t, ring, head, count) == OR_OK);
      free(ring);
    }
    free(trk);
    free(sl);
  }
  CHECK(or_set_iteration(b, 5, 1) == OR_OK);
  uint64_t na[3], nb[3];
  CHECK(or_step(a, na) == OR_OK && or_step(b, nb) == OR_OK);
  CHECK(memcmp(na, nb, sizeof(na)) == 0);
  or_destroy(a);
  or_destroy(b);
  return 0;
}

int main(void) {
  for (int scheme = 0; scheme < 2; ++scheme)
    for (int prec = 0; prec < 2; ++prec) {
      /* sparse: 512 slots, so the free-slot rings wrap around several times */
      if (shower(scheme, prec, scheme == OR_SPARSE ? 512u : 1u << 14, prec, 1 - prec)) return 1;
      if (admission(scheme, prec)) return 1;
    }
  for (int scheme = 0; scheme < 2; ++scheme)
    if (overflow_and_handover(scheme)) return 1;
  printf("oracle driver ok\n");
  return 0;
}
