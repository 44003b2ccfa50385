// Host launcher of the mapping-chain kernels of one register class (NS, NI)
// and precision; each chain_*.hip unit includes this header and
// instantiates it.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "chain_kernels.h"
#include "launch.h"

namespace msx {

// Kind classes: `kc` picks the compiled map kinds (0: integer-root power
// laws, 1: plus Breit-Wigner, 2: all tree kinds; 3: those of class 1 with
// Chili channels, 4: those of class 1 with 1 -> 3 decays, 5: everything,
// (s~, t) blocks included).  Chili and 1 -> 3 decays have classes of their
// own because compiled together they overflow the register file.
template <class Go>
void with_kind_class(int kc, Go&& go) {
    constexpr int K0 = KIND_POW_INT, K1 = KIND_POW_INT | KIND_BW, K2 = KINDS_ALL;
    constexpr int K3 = K1 | KIND_CHILI, K4 = K1 | KIND_DEC3, K5 = KINDS_ALL | KIND_CHILI | KIND_DEC3 | KIND_ST;
    if (kc == 0) go(std::integral_constant<int, K0>{});
    else if (kc <= 1) go(std::integral_constant<int, K1>{});
    else if (kc == 2) go(std::integral_constant<int, K2>{});
    else if (kc == 3) go(std::integral_constant<int, K3>{});
    else if (kc == 4) go(std::integral_constant<int, K4>{});
    else go(std::integral_constant<int, K5>{});
}

// Map or fused-sample launch of one register class and precision.
template <int NS, int NI, bool MIX>
hipError_t launch_chain_class(int kc, const ChainLaunch& a) {
    hipError_t err = hipSuccess;
    with_kind_class(kc, [&](auto kt) {
        constexpr int K = decltype(kt)::value;
        const size_t lds = a.lds + (a.sample ? sizeof(double) * stage_rows<NS, NI>() * kBlock : kQBytes) +
                           (a.vpart ? vegas_acc_lds(a.vstride) : 0);
        if (lds > 65536) {
            // beyond the default 64 KiB per workgroup (gfx950 has 160 KiB per CU)
            const void* fn = a.sample ? (const void*)k_sample<NS, NI, K, MIX> : (const void*)k_map<NS, NI, K, MIX>;
            err = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (err != hipSuccess) return;
        }
        if (a.sample)
            k_sample<NS, NI, K, MIX><<<a.grid, kBlock, lds, a.stream>>>(
                a.cts, a.pts, a.grids, a.grid_off, a.chan_nb, a.call, a.seed, a.sid, a.ctr_dev, a.ctr_off, a.np, a.n,
                a.p, a.x1x2, a.w, a.chan, a.tile_stats, (int)(a.lds / sizeof(double)), a.vpart, a.vstride);
        else
            k_map<NS, NI, K, MIX><<<a.grid, kBlock, lds, a.stream>>>(a.cts, a.pts, a.grids, a.nb, a.s_lab, a.np, a.n,
                                                                         a.y, a.p, a.x1x2, a.jac, a.w);
    });
    if (err != hipSuccess) return err;
    return hipGetLastError();
}

// Inverse-map launch of one register class (FP64).  Its units keep the
// compiler's default floating-point contraction (the forward units turn it
// off so that the specialised sample is bit-identical to the class kernel).
template <int NS, int NI>
hipError_t launch_inverse_class(int kc, const ChainLaunch& a) {
    hipError_t err = hipSuccess;
    with_kind_class(kc, [&](auto kt) {
        constexpr int K = decltype(kt)::value;
        const size_t li = a.lds + sizeof(double) * stage_rows<NS, NI>() * kBlock;
        if (li > 65536) {
            err = hipFuncSetAttribute((const void*)k_inverse<NS, NI, K>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)li);
            if (err != hipSuccess) return;
        }
        k_inverse<NS, NI, K><<<a.grid, kBlock, li, a.stream>>>(a.cts, a.grids, a.nb, a.s_lab, a.np, a.n, a.p_in,
                                                              a.x1x2_in, a.y_out);
    });
    if (err != hipSuccess) return err;
    return hipGetLastError();
}

#define MSX_INSTANTIATE_CHAIN(NS, NI, MIX) \
    template hipError_t launch_chain_class<NS, NI, MIX>(int kc, const ChainLaunch& a);
#define MSX_INSTANTIATE_INVERSE(NS, NI) template hipError_t launch_inverse_class<NS, NI>(int kc, const ChainLaunch& a);

}  // namespace msx
