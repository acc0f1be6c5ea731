// Instantiations: general linear model (nx, ny, nw) = (2, 1, 1).
#include "runner_impl.h"
namespace ms {
MS_INSTANTIATE(ModelLinear<2 MS_COMMA 1 MS_COMMA 1>)
}  // namespace ms
