// Persistent job and level-synchronous table kernels of the inverse (float32 and int32).
#include "strip_kernels.h"

namespace dwt2 {
DWT2_INSTANTIATE_JOB(kInv)
}  // namespace dwt2
