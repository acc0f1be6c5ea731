// Instantiations: coordinated-turn model (nx = 5).
#include "runner_impl.h"
namespace ms {
MS_INSTANTIATE(ModelCT)
}  // namespace ms
