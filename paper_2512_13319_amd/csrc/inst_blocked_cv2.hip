// Instantiations: sub-stepped blocks of the constant-velocity model (nx = 4).
#include "runner_impl.h"
namespace ms {
MS_INSTANTIATE_BLOCKED(ModelCV<2>)
}  // namespace ms
