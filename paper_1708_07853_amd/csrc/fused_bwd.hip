// Pair kernels (two levels per pass) of the adjoint (float32).
#include "fused.h"

namespace dwt2 {
DWT2_INSTANTIATE_PAIR(kBwd)
}  // namespace dwt2
