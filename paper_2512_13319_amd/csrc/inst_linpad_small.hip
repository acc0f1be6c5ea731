// Instantiations: general linear model with ny, nw padded to nx, nx <= 4.
#include "runner_impl.h"
namespace ms {
MS_INSTANTIATE(ModelLinearPadded<1>)
MS_INSTANTIATE(ModelLinearPadded<2>)
MS_INSTANTIATE(ModelLinearPadded<3>)
MS_INSTANTIATE(ModelLinearPadded<4>)
}  // namespace ms
