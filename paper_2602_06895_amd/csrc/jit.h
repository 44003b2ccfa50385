// Run-time specialisation of the fused multichannel sample (jit.cpp).
#pragma once

#include <string>

#include "compiler.h"
#include "launch.h"

namespace msx {

// Compiles (HIP run-time compiler, for `device`'s architecture) and loads
// fused-sample kernels for the channels of `comp` (groups of consecutive
// channels, one kernel each), with every channel and process table a
// compile-time constant.  On failure returns false with the reason (the
// compiler's log) in err and leaves out untouched; spills is set when a
// single channel's kernel compiled but uses scratch.
bool jit_build_sample(const Compiled& comp, int mixed, int device, JitSampleSet& out, std::string& err,
                      bool& spills);
// Unloads the kernels' modules.
void jit_release(JitSampleSet& s);

}  // namespace msx
