// Instantiations: general linear model padded to nx = 6, float storage.
#include "runner_impl.h"
namespace ms {
MS_INSTANTIATE_LARGE(float, ModelLinearPadded<6>)
}  // namespace ms
