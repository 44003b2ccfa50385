// Inverse-map kernels: 14 momentum slots, 8 invariants, FP64.
#include "chain_launch.h"

namespace msx {
MSX_INSTANTIATE_INVERSE(14, 8)
}  // namespace msx
