// Instantiations: general linear model padded to nx = 7, float storage.
#include "runner_impl.h"
namespace ms {
MS_INSTANTIATE_LARGE(float, ModelLinearPadded<7>)
}  // namespace ms
