// Run-time specialisation of the fused multichannel sample (jit.cpp).
#pragma once

#include <string>

#include "compiler.h"
#include "launch.h"

namespace msx {

// Compiles (HIP run-time compiler, for `device`'s architecture) and loads a
// fused-sample kernel for the channels of `comp`, with every channel and
// process table a compile-time constant.  On failure returns false with the
// reason (the compiler's log) in err and leaves out untouched; spills is set
// when the kernel compiled but uses scratch (it is then not kept).
bool jit_build_sample(const Compiled& comp, int mixed, int device, JitSample& out, std::string& err,
                      bool& spills);
// Unloads the kernel's module.
void jit_release(JitSample& j);

}  // namespace msx
