// Pair kernels (two levels per pass) of the inverse (float32 and int32).
#include "fused.h"

namespace dwt2 {
DWT2_INSTANTIATE_PAIR(kInv)
}  // namespace dwt2
