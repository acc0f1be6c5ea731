// Instantiations: general linear model (nx, ny, nw) = (3, 3, 3).
#include "runner_impl.h"
namespace ms {
MS_INSTANTIATE(ModelLinear<3 MS_COMMA 3 MS_COMMA 3>)
}  // namespace ms
