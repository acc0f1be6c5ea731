// Instantiations: nonlinear models (Van der Pol, Lorenz-63).
#include "runner_impl.h"
namespace ms {
MS_INSTANTIATE(ModelVdP)
MS_INSTANTIATE(ModelLorenz63)
}  // namespace ms
