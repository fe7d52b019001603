// Per-level strip kernels of the adjoint (float32).
#include "strip_kernels.h"

namespace dwt2 {
DWT2_INSTANTIATE_LEVEL(kBwd)
}  // namespace dwt2
