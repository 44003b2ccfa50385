// Mapping-chain kernels: 14 momentum slots, 8 invariants, FP64.
#include "chain_launch.h"

namespace msx {
MSX_INSTANTIATE_CHAIN(14, 8, false)
}  // namespace msx
