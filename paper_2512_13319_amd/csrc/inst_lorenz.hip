// Instantiations: Lorenz-63 model.
#include "runner_impl.h"
namespace ms {
MS_INSTANTIATE(ModelLorenz63)
}  // namespace ms
