// Instantiations: Wiener velocity model, one axis (nx = 2).
#include "runner_impl.h"
namespace ms {
MS_INSTANTIATE(ModelCV<1>)
}  // namespace ms
