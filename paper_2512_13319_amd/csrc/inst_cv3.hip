// Instantiations: constant-velocity model, three axes (nx = 6).
#include "runner_impl.h"
namespace ms {
MS_INSTANTIATE(ModelCV<3>)
}  // namespace ms
