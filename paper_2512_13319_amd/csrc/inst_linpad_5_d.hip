// Instantiations: general linear model padded to nx = 5, double storage.
#include "runner_impl.h"
namespace ms {
MS_INSTANTIATE_LARGE(double, ModelLinearPadded<5>)
}  // namespace ms
