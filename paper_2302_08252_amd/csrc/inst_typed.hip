// Kernel instantiations: the per-particle-type mapping, both schemes and
// precisions, with and without instrumentation.
#include "kernels.hpp"

namespace adept {
void ops_typed(Ops t[2][2][4][2]) {
  t[SPARSE][0][MAP_TYPED][0] = Variant<SPARSE, MAP_TYPED, PolicyF64, false>::ops();
  t[SPARSE][0][MAP_TYPED][1] = Variant<SPARSE, MAP_TYPED, PolicyF64, true>::ops();
  t[SPARSE][1][MAP_TYPED][0] = Variant<SPARSE, MAP_TYPED, PolicyMixed, false>::ops();
  t[SPARSE][1][MAP_TYPED][1] = Variant<SPARSE, MAP_TYPED, PolicyMixed, true>::ops();
  t[DENSE][0][MAP_TYPED][0] = Variant<DENSE, MAP_TYPED, PolicyF64, false>::ops();
  t[DENSE][0][MAP_TYPED][1] = Variant<DENSE, MAP_TYPED, PolicyF64, true>::ops();
  t[DENSE][1][MAP_TYPED][0] = Variant<DENSE, MAP_TYPED, PolicyMixed, false>::ops();
  t[DENSE][1][MAP_TYPED][1] = Variant<DENSE, MAP_TYPED, PolicyMixed, true>::ops();
}
}  // namespace adept
