// Instantiations: general linear model padded to nx = 6, double storage.
#include "runner_impl.h"
namespace ms {
MS_INSTANTIATE_LARGE(double, ModelLinearPadded<6>)
}  // namespace ms
