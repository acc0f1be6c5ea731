// Instantiations: Van der Pol model.
#include "runner_impl.h"
namespace ms {
MS_INSTANTIATE(ModelVdP)
}  // namespace ms
