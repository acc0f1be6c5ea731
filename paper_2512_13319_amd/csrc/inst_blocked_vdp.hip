// Instantiations: sub-stepped blocks of the Van der Pol model.
#include "runner_impl.h"
namespace ms {
MS_INSTANTIATE_BLOCKED(ModelVdP)
}  // namespace ms
