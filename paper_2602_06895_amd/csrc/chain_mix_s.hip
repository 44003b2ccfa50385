// Mapping-chain kernels: 6 momentum slots, 4 invariants, mixed precision.
#include "chain_launch.h"

namespace msx {
MSX_INSTANTIATE_CHAIN(6, 4, true)
}  // namespace msx
