// Instantiations: general linear model padded to nx = 8, double storage.
#include "runner_impl.h"
namespace ms {
MS_INSTANTIATE_LARGE(double, ModelLinearPadded<8>)
}  // namespace ms
