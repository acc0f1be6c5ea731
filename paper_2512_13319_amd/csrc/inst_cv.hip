// Instantiations: constant-velocity / Wiener velocity models.
#include "runner_impl.h"
namespace ms {
MS_INSTANTIATE(ModelCV<1>)
MS_INSTANTIATE(ModelCV<2>)
MS_INSTANTIATE(ModelCV<3>)
}  // namespace ms
