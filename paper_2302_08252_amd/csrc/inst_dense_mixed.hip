// Kernel instantiations: dense scheme, mixed precision, every record layout,
// with and without instrumentation.
#include "kernels.hpp"

namespace adept {
void ops_dense_mixed(Ops t[4][2]) {
  t[MAP_AOS][0] = Variant<DENSE, MAP_AOS, PolicyMixed, false>::ops();
  t[MAP_AOS][1] = Variant<DENSE, MAP_AOS, PolicyMixed, true>::ops();
  t[MAP_SOA][0] = Variant<DENSE, MAP_SOA, PolicyMixed, false>::ops();
  t[MAP_SOA][1] = Variant<DENSE, MAP_SOA, PolicyMixed, true>::ops();
  t[MAP_AOSOA][0] = Variant<DENSE, MAP_AOSOA, PolicyMixed, false>::ops();
  t[MAP_AOSOA][1] = Variant<DENSE, MAP_AOSOA, PolicyMixed, true>::ops();
}
}  // namespace adept
