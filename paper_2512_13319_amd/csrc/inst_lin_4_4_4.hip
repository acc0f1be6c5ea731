// Instantiations: general linear model (nx, ny, nw) = (4, 4, 4).
#include "runner_impl.h"
namespace ms {
MS_INSTANTIATE(ModelLinear<4 MS_COMMA 4 MS_COMMA 4>)
}  // namespace ms
