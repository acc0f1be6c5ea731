// Instantiations: general linear model padded to nx = 5, float storage.
#include "runner_impl.h"
namespace ms {
MS_INSTANTIATE_LARGE(float, ModelLinearPadded<5>)
}  // namespace ms
