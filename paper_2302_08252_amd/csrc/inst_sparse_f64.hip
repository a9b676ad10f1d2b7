// Kernel instantiations: sparse scheme, f64 precision, every record layout,
// with and without instrumentation.
#include "kernels.hpp"

namespace adept {
void ops_sparse_f64(Ops t[4][2]) {
  t[MAP_AOS][0] = Variant<SPARSE, MAP_AOS, PolicyF64, false>::ops();
  t[MAP_AOS][1] = Variant<SPARSE, MAP_AOS, PolicyF64, true>::ops();
  t[MAP_SOA][0] = Variant<SPARSE, MAP_SOA, PolicyF64, false>::ops();
  t[MAP_SOA][1] = Variant<SPARSE, MAP_SOA, PolicyF64, true>::ops();
  t[MAP_AOSOA][0] = Variant<SPARSE, MAP_AOSOA, PolicyF64, false>::ops();
  t[MAP_AOSOA][1] = Variant<SPARSE, MAP_AOSOA, PolicyF64, true>::ops();
}
}  // namespace adept
