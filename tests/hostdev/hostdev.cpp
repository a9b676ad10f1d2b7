// Host build of the library's device-side model (model.hpp, layout.hpp) for
// CPU-side checks against the oracle: the HIP path's physics, random numbers,
// elementary functions and layouts compiled for x86 with the same flags
// (-ffp-contract=off), exposed through a C interface for ctypes.
#include <cstring>

#include "../../paper_2302_08252_amd/csrc/layout.hpp"
#include "../../paper_2302_08252_amd/csrc/model.hpp"

using namespace adept;

struct TrackIO {  // the 96-byte dump record
  double pos[3], dir[3], E, nl;
  uint64_t id, parent;
  uint32_t seed, ctr;
  int32_t vol;
  uint32_t event;
};

template <class P>
static int step_one(int type, const TrackIO* in, int* surv, TrackIO out[4], int out_type[4], double dep[5]) {
  using R = typename P::R;
  Track<R> t;
  for (int i = 0; i < 3; ++i) {
    t.pos[i] = in->pos[i];
    t.dir[i] = (R)in->dir[i];
  }
  t.E = (R)in->E;
  t.nl = (R)in->nl;
  t.id = in->id;
  t.parent = in->parent;
  t.seed = in->seed;
  t.ctr = in->ctr;
  t.vol = in->vol;
  t.event = in->event;
  Creations<R> cr;
  cr.n = 0;
  cr.meta = 0;
  Deposits d{0.0, 0.0, 0.0, 0.0, {0.0, 0.0}};
  const bool s = type == GAMMA ? step_photon<P>(t, cr, d) : step_charged<P>(t, type, cr, d);
  int k = 0;
  if (s) {
    TrackIO& o = out[k];
    for (int i = 0; i < 3; ++i) {
      o.pos[i] = t.pos[i];
      o.dir[i] = (double)t.dir[i];
    }
    o.E = (double)t.E;
    o.nl = (double)t.nl;
    o.id = t.id;
    o.parent = in->parent;
    o.seed = t.seed;
    o.ctr = t.ctr;
    o.vol = t.vol;
    o.event = t.event;
    out_type[k++] = type;
  }
  for (int i = 0; i < cr.n; ++i) {
    TrackIO& o = out[k];
    for (int j = 0; j < 3; ++j) {
      o.pos[j] = t.pos[j];
      const R dd = cr.dsel(i) == 0 ? t.dir[j] : (cr.dsel(i) == 1 ? cr.d[j] : -cr.d[j]);
      o.dir[j] = (double)dd;
    }
    o.E = (double)cr.E[i];
    o.nl = -1.0;
    o.parent = creation_parent(cr, i, t.seed, t.id, in->ctr);
    o.id = creation_id(cr, i, t.seed, o.parent, in->ctr);
    o.seed = t.seed;
    o.ctr = 0;
    o.vol = t.vol;
    o.event = t.event;
    out_type[k++] = cr.type(i);
  }
  *surv = s ? 1 : 0;
  dep[0] = d.cont;
  dep[1] = d.cut;
  dep[2] = d.escaped;
  dep[3] = d.round;
  dep[4] = 0.0;
  return k;
}

extern "C" {
void hd_philox(const uint32_t c[4], const uint32_t k[2], uint32_t o[4]) {
  const U4 r = philox(U4{c[0], c[1], c[2], c[3]}, k[0], k[1]);
  o[0] = r.x; o[1] = r.y; o[2] = r.z; o[3] = r.w;
}
double hd_log(double x) { return plog<double>(x); }
double hd_exp(double x) { return pexp<double>(x); }
void hd_sincos(double x, double* s, double* c) { psincos<double>(x, s, c); }
float hd_logf(float x) { return plog<float>(x); }
float hd_expf(float x) { return pexp<float>(x); }
void hd_sincosf(float x, float* s, float* c) { psincos<float>(x, s, c); }
uint64_t hd_child_id(uint32_t seed, uint64_t id, uint32_t n, uint32_t k) { return child_id(seed, id, n, k); }
int hd_step(int mixed, int type, const TrackIO* in, int* surv, TrackIO out[4], int out_type[4], double dep[5]) {
  return mixed ? step_one<PolicyMixed>(type, in, surv, out, out_type, dep)
               : step_one<PolicyF64>(type, in, surv, out, out_type, dep);
}
uint64_t hd_leaf_addr(int map, int mixed, uint32_t lanes, uint64_t C, uint64_t slot, int leaf) {
  if (mixed) {
    const MapArgs m = make_map_args<true>(map, lanes, C);
    if (map == MAP_AOS) return leaf_addr<MAP_AOS, true>(m, slot, leaf);
    if (map == MAP_SOA) return leaf_addr<MAP_SOA, true>(m, slot, leaf);
    return leaf_addr<MAP_AOSOA, true>(m, slot, leaf);
  }
  const MapArgs m = make_map_args<false>(map, lanes, C);
  if (map == MAP_AOS) return leaf_addr<MAP_AOS, false>(m, slot, leaf);
  if (map == MAP_SOA) return leaf_addr<MAP_SOA, false>(m, slot, leaf);
  return leaf_addr<MAP_AOSOA, false>(m, slot, leaf);
}
double hd_distance(const double p[3], const double d[3], int v, int* axis) { return distance(p, d, v, axis); }
uint64_t hd_buffer_bytes(int map, int mixed, uint32_t lanes, uint64_t C) {
  return mixed ? buffer_bytes<true>(map, lanes, C) : buffer_bytes<false>(map, lanes, C);
}
}
