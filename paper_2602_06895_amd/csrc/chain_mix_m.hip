// Mapping-chain kernels: 10 momentum slots, 8 invariants, mixed precision.
#include "chain_launch.h"

namespace msx {
MSX_INSTANTIATE_CHAIN(10, 8, true)
}  // namespace msx
