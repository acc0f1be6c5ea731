// Instantiations: general linear model (nx, ny, nw) = (4, 2, 4).
#include "runner_impl.h"
namespace ms {
MS_INSTANTIATE(ModelLinear<4 MS_COMMA 2 MS_COMMA 4>)
}  // namespace ms
