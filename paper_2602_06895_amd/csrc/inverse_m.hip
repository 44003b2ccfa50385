// Inverse-map kernels: 10 momentum slots, 8 invariants, FP64.
#include "chain_launch.h"

namespace msx {
MSX_INSTANTIATE_INVERSE(10, 8)
}  // namespace msx
