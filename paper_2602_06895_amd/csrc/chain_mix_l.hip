// Mapping-chain kernels: 14 momentum slots, 8 invariants, mixed precision.
#include "chain_launch.h"

namespace msx {
MSX_INSTANTIATE_CHAIN(14, 8, true)
}  // namespace msx
