// Persistent job and level-synchronous table kernels of the adjoint (float32).
#include "strip_kernels.h"

namespace dwt2 {
DWT2_INSTANTIATE_JOB(kBwd)
}  // namespace dwt2
