// Reverse derivative of the force evaluation (placeholder until the adjoint
// kernels land).
#include "common.h"

namespace hot {
void adjoint(hot_ctx*, hot_tree*, const double*, const double*, double, int, const double*,
             double*, double*) {
  throw Error{HOT_E_STATE, "adjoint not available in this build"};
}
}  // namespace hot
