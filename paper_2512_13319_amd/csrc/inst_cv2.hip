// Instantiations: constant-velocity model, two axes (nx = 4).
#include "runner_impl.h"
namespace ms {
MS_INSTANTIATE(ModelCV<2>)
}  // namespace ms
