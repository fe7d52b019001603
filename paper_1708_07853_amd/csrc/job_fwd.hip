// Persistent job and level-synchronous table kernels of the forward (float32 and int32).
#include "strip_kernels.h"

namespace dwt2 {
DWT2_INSTANTIATE_JOB(kFwd)
}  // namespace dwt2
