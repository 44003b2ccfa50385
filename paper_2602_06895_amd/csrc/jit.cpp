// Run-time specialisation of the fused multichannel sample.
//
// The kernel is the source of k_sample (sample_loop and sample_tile in
// chain_kernels.h), compiled with the HIP run-time compiler for one
// context's channels: every channel's and process's table becomes a
// constexpr object (bit-cast from its bytes), so the compiler folds the
// table reads, the map-kind and operation-count branches and the slot
// indices of the chain into constants, unrolls each channel's operations
// and keeps only the momentum slots that are still live.  The arithmetic is
// the same source and the forward chain is compiled without floating-point
// contraction, so the results are bit-identical to the class kernel's; only
// the code is smaller (no AGPR spilling, fewer registers, more waves per
// SIMD) and runs fewer instructions.  The headers come from jit_sources.cpp, which the build
// generates from the kernel headers.
#include "jit.h"

#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <algorithm>
#include <cstdio>
#include <vector>

#include "tables.h"

namespace msx {
namespace jit_src {
extern const int kHeaderCount;
extern const char* const kHeaderNames[];
extern const char* const kHeaderTexts[];
}  // namespace jit_src

namespace {

// (NS, NI) register class of a channel, as the class kernels pick it
void reg_class_of(const ChannelTab& t, int& ns, int& ni) {
    if (t.n_slots <= 6 && t.n_inv <= 4) {
        ns = 6;
        ni = 4;
    } else if (t.n_slots <= 10 && t.n_inv <= 8) {
        ns = 10;
        ni = 8;
    } else {
        ns = 14;
        ni = 8;
    }
}

// constexpr <type> <name><index> = the table whose bytes are p[0 .. n)
// (bit-cast from a byte image, so the compiler sees every field's value)
void emit_table(std::string& s, const char* type, const char* name, int index, const void* p, size_t n) {
    char head[128];
    std::snprintf(head, sizeof head, "constexpr %s %s%d = __builtin_bit_cast(%s, Image<%zu>{{", type, name, index,
                  type, n);
    s += head;
    const unsigned char* b = (const unsigned char*)p;
    for (size_t i = 0; i < n; ++i) {
        char v[8];
        std::snprintf(v, sizeof v, i ? ",%u" : "%u", (unsigned)b[i]);
        s += v;
    }
    s += "}});\n";
}

// waves > 0: ask the compiler for at least that many waves per SIMD (it
// then limits the registers to 512 / waves)
std::string sample_source(const Compiled& comp, int mixed, int waves, int c0, int c1, int& rows) {
    std::string s =
        "using __hip_internal::int32_t;\nusing __hip_internal::uint32_t;\nusing __hip_internal::int64_t;\n"
        "using __hip_internal::uint64_t;\nusing __hip_internal::uint8_t;\n#include \"chain_kernels.h\"\n"
        "namespace msx {\nnamespace spec {\ntemplate <unsigned long N>\nstruct Image {\n    unsigned char b[N];\n};\n";
    rows = kMaxUniq + 1;
    std::vector<int> procs;
    for (int c = c0; c < c1; ++c) {
        emit_table(s, "ChannelTab", "chan", c, &comp.chans[c], sizeof(ChannelTab));
        int ns, ni;
        reg_class_of(comp.chans[c], ns, ni);
        rows = std::max(rows, ns + ni + 1);
        if (std::find(procs.begin(), procs.end(), comp.chans[c].process) == procs.end())
            procs.push_back(comp.chans[c].process);
    }
    for (int q : procs) emit_table(s, "ProcessTab", "proc", q, &comp.procs[q], sizeof(ProcessTab));
    s += "}  // namespace spec\n}  // namespace msx\n";
    s += "extern \"C\" __global__ __launch_bounds__(msx::kBlock) ";
    if (waves > 0) s += "__attribute__((amdgpu_waves_per_eu(" + std::to_string(waves) + "))) ";
    s += "void MSX_JIT_NAME(\n"
         "    const msx::ChannelTab* __restrict__ cts, const msx::ProcessTab* __restrict__ pts,\n"
         "    const double* __restrict__ grids, const int64_t* __restrict__ grid_off,\n"
         "    const int32_t* __restrict__ chan_nb, const msx::SampleCall* __restrict__ call, uint64_t seed,\n"
         "    uint64_t sid, const uint64_t* __restrict__ ctr_dev, uint64_t ctr_off, int np, int64_t ld,\n"
         "    double* __restrict__ p, double* __restrict__ x1x2, double* __restrict__ w,\n"
         "    int32_t* __restrict__ chan_out, double* __restrict__ tile_stats, int grid_doubles,\n"
         "    double* __restrict__ vpart, int vstride) {\n"
         "    using namespace msx;\n";
    s += "    sample_loop<" + std::to_string(rows) +
         ">(cts, grids, grid_off, chan_nb, call, seed, sid, ctr_dev, ctr_off, np, ld, p, x1x2, w, chan_out,\n"
         "        tile_stats, grid_doubles, vpart, vstride, [&](auto& run) {\n";
    for (int c = c0; c < c1; ++c) {
        int ns, ni;
        reg_class_of(comp.chans[c], ns, ni);
        const std::string cs = std::to_string(c);
        s += "        run(" + cs + ", [&](const TileArgs& t, TileAcc& acc) { sample_tile<" + std::to_string(ns) + ", " +
             std::to_string(ni) + ", " + std::to_string(comp.chans[c].kinds) + ", " + (mixed ? "true" : "false") +
             ">(&spec::chan" + cs + ", &spec::proc" + std::to_string(comp.chans[c].process) + ", " + cs +
             ", t, acc); });\n";
    }
    s += "    });\n}\n";
    return s;
}

// The kernel's name: msx_jit_sample_ and a 64-bit FNV-1a hash of its source
// (so that the kernels of different contexts are told apart in traces).
std::string kernel_name(const std::string& src) {
    uint64_t h = 0xcbf29ce484222325ull;
    for (unsigned char ch : src) {
        h ^= ch;
        h *= 0x100000001b3ull;
    }
    char buf[40];
    std::snprintf(buf, sizeof buf, "msx_jit_sample_%016llx", (unsigned long long)h);
    return buf;
}

// Compiles `body` and loads its kernel; *scratch gets its scratch bytes per
// lane.
bool compile_load(const std::string& body, const std::string& arch, JitSample& j, int* scratch, std::string& err) {
    const std::string name = kernel_name(body);
    const std::string src = "#define MSX_JIT_NAME " + name + "\n" + body;
    // the library's own flags for the FP64 path (no contraction, no packed
    // FP32); no machine-level loop-invariant hoisting, which in this kernel
    // only lengthens the live ranges of constants and table values
    const char* opts[] = {arch.c_str(), "-O3", "-std=c++17", "-ffp-contract=off", "-Xclang", "-target-feature",
                          "-Xclang", "-packed-fp32-ops", "-mllvm", "-disable-machine-licm"};
    hiprtcProgram prog;
    hiprtcResult r = hiprtcCreateProgram(&prog, src.c_str(), "msx_jit_sample.hip", jit_src::kHeaderCount,
                                         jit_src::kHeaderTexts, jit_src::kHeaderNames);
    if (r != HIPRTC_SUCCESS) {
        err = std::string("hiprtcCreateProgram: ") + hiprtcGetErrorString(r);
        return false;
    }
    r = hiprtcCompileProgram(prog, (int)(sizeof opts / sizeof opts[0]), opts);
    if (r != HIPRTC_SUCCESS) {
        size_t n = 0;
        std::string log;
        if (hiprtcGetProgramLogSize(prog, &n) == HIPRTC_SUCCESS && n > 1) {
            log.resize(n);
            (void)hiprtcGetProgramLog(prog, &log[0]);
        }
        (void)hiprtcDestroyProgram(&prog);
        err = std::string("hiprtcCompileProgram: ") + hiprtcGetErrorString(r) + "\n" + log.substr(0, 4000);
        return false;
    }
    size_t code_size = 0;
    std::vector<char> code;
    if ((r = hiprtcGetCodeSize(prog, &code_size)) == HIPRTC_SUCCESS) {
        code.resize(code_size);
        r = hiprtcGetCode(prog, code.data());
    }
    (void)hiprtcDestroyProgram(&prog);
    if (r != HIPRTC_SUCCESS) {
        err = std::string("hiprtcGetCode: ") + hiprtcGetErrorString(r);
        return false;
    }
    hipError_t he;
    if ((he = hipModuleLoadData(&j.module, code.data())) != hipSuccess) {
        err = std::string("hipModuleLoadData: ") + hipGetErrorString(he);
        return false;
    }
    if ((he = hipModuleGetFunction(&j.fn, j.module, name.c_str())) != hipSuccess ||
        (he = hipFuncGetAttribute(scratch, HIP_FUNC_ATTRIBUTE_LOCAL_SIZE_BYTES, j.fn)) != hipSuccess) {
        err = std::string("hipModuleGetFunction: ") + hipGetErrorString(he);
        (void)hipModuleUnload(j.module);
        j = JitSample{};
        return false;
    }
    return true;
}

// One kernel for channels [c0, c1): first at three waves per SIMD (168
// registers), which is faster than two waves where it needs little or no
// scratch (t tbar: 12 B/lane, 5% faster); a three-wave build with more
// scratch than kMaxScratch is dropped for the compiler's default occupancy
// (the eight pp -> 4 jets channels at three waves need 120 B/lane, which
// costs 100 B/event of HBM traffic).  Returns 0 with the kernel in j, 1 when
// the kernel spills even at the default occupancy (not kept), -1 on error.
int build_group(const Compiled& comp, int mixed, const std::string& arch, int c0, int c1, JitSample& j,
                int* scratch_out, std::string& err) {
    constexpr int kMaxScratch = 32;
    for (int waves : {3, 0}) {
        int rows = 0;
        const std::string src = sample_source(comp, mixed, waves, c0, c1, rows);
        JitSample k;
        int scratch = 0;
        if (!compile_load(src, arch, k, &scratch, err)) return -1;
        if ((waves > 0 && scratch > kMaxScratch) || (waves == 0 && scratch > 0)) {
            (void)hipModuleUnload(k.module);
            if (waves > 0) continue;
            *scratch_out = scratch;
            return 1;
        }
        k.rows = rows;
        k.waves = waves;
        k.scratch = scratch;
        k.c0 = c0;
        k.c1 = c1;
        j = k;
        return 0;
    }
    return -1;
}

}  // namespace

bool jit_build_sample(const Compiled& comp, int mixed, int device, JitSampleSet& out, std::string& err, bool& spills) {
    spills = false;
    hipDeviceProp_t prop;
    hipError_t he = hipGetDeviceProperties(&prop, device);
    if (he != hipSuccess) {
        err = std::string("hipGetDeviceProperties: ") + hipGetErrorString(he);
        return false;
    }
    const std::string arch = std::string("--offload-arch=") + prop.gcnArchName;
    // Channels go into kernels of at most kGroup consecutive channels, one
    // launch each: the register file of one kernel is the largest any of its
    // channel loops needs plus what the compiler keeps live across them, and
    // grows with the channel count (24 channels in one kernel: 342 VGPRs and
    // 412 B/lane of scratch).  A group whose kernel spills is split in
    // halves; a single channel whose kernel spills makes the whole call fail
    // (the class kernel is kept).
    constexpr int kGroup = 8;
    const int C = (int)comp.chans.size();
    std::vector<std::pair<int, int>> todo;
    for (int c = 0; c < C; c += kGroup) todo.push_back({c, std::min(C, c + kGroup)});
    JitSampleSet set;
    auto release = [&]() {
        for (int g = 0; g < set.n; ++g) (void)hipModuleUnload(set.k[g].module);
    };
    for (size_t i = 0; i < todo.size(); ++i) {
        const int c0 = todo[i].first, c1 = todo[i].second;
        JitSample k;
        int scratch = 0;
        const int r = build_group(comp, mixed, arch, c0, c1, k, &scratch, err);
        if (r < 0) {
            release();
            return false;
        }
        if (r == 1) {
            if (c1 - c0 == 1) {
                err = "the kernel compiled for channel " + std::to_string(c0) + " spills registers (" +
                      std::to_string(scratch) + " B of scratch per lane); the class kernel is kept";
                spills = true;
                release();
                return false;
            }
            const int mid = (c0 + c1) / 2;
            todo.insert(todo.begin() + (std::ptrdiff_t)i + 1, {{c0, mid}, {mid, c1}});
            continue;
        }
        if (set.n == kMaxJitGroups) {
            err = "too many specialised kernels";
            (void)hipModuleUnload(k.module);
            release();
            return false;
        }
        set.k[set.n++] = k;
    }
    out = set;
    return true;
}

void jit_release(JitSampleSet& s) {
    for (int g = 0; g < s.n; ++g)
        if (s.k[g].module) (void)hipModuleUnload(s.k[g].module);
    s = JitSampleSet{};
}

}  // namespace msx
