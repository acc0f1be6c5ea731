// Instantiations: general linear model padded to nx = 8, float storage.
#include "runner_impl.h"
namespace ms {
MS_INSTANTIATE_LARGE(float, ModelLinearPadded<8>)
}  // namespace ms
