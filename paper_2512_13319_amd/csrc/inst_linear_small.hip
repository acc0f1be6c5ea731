// Instantiations: general linear model, nx <= 3.
#include "runner_impl.h"
namespace ms {
MS_INSTANTIATE(ModelLinear<1 MS_COMMA 1 MS_COMMA 1>)
MS_INSTANTIATE(ModelLinear<2 MS_COMMA 1 MS_COMMA 1>)
MS_INSTANTIATE(ModelLinear<2 MS_COMMA 1 MS_COMMA 2>)
MS_INSTANTIATE(ModelLinear<2 MS_COMMA 2 MS_COMMA 2>)
MS_INSTANTIATE(ModelLinear<3 MS_COMMA 2 MS_COMMA 2>)
MS_INSTANTIATE(ModelLinear<3 MS_COMMA 2 MS_COMMA 3>)
MS_INSTANTIATE(ModelLinear<3 MS_COMMA 3 MS_COMMA 3>)
}  // namespace ms
