// Instantiations: general linear model (nx, ny, nw) = (2, 2, 2).
#include "runner_impl.h"
namespace ms {
MS_INSTANTIATE(ModelLinear<2 MS_COMMA 2 MS_COMMA 2>)
}  // namespace ms
