// Instantiations: general linear model padded to nx = 7, double storage.
#include "runner_impl.h"
namespace ms {
MS_INSTANTIATE_LARGE(double, ModelLinearPadded<7>)
}  // namespace ms
