// Inverse-map kernels: 6 momentum slots, 4 invariants, FP64.
#include "chain_launch.h"

namespace msx {
MSX_INSTANTIATE_INVERSE(6, 4)
}  // namespace msx
