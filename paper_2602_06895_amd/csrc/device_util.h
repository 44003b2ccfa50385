// Small device helpers shared by the kernels: launch shape, the VEGAS lookup
// and deterministic wave reductions.
#pragma once

#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#include <stdint.h>
#endif

#include "tables.h"

namespace msx {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

// VEGAS map of one uniform through a grid row in LDS: bin i = floor(y nb),
// linear inside the bin, Jacobian nb (e_{i+1} - e_i).
__device__ __forceinline__ double vegas_map(double y, const double* __restrict__ g, int nb, double& jv) {
    double t = y * nb;
    int i = (int)t;
    i = i < 0 ? 0 : (i > nb - 1 ? nb - 1 : i);
    double e0 = g[i], e1 = g[i + 1];
    double wd = e1 - e0;
    jv *= nb * wd;
    return e0 + wd * (t - i);
}

// vegas_map for caller-supplied y, which may lie outside [0, 1] or be NaN
// (the inverse map marks events outside a channel's image with NaN): the bin
// index is formed without converting a NaN or an out-of-range value to int;
// a NaN y stays NaN, so the chain cuts the event.
__device__ __forceinline__ double vegas_map_checked(double y, const double* __restrict__ g, int nb, double& jv) {
    const double t = y * nb;
    const int i = t >= 1.0 ? (t < nb - 1 ? (int)t : nb - 1) : 0;
    const double e0 = g[i], e1 = g[i + 1];
    const double wd = e1 - e0;
    jv *= nb * wd;
    return e0 + wd * (t - i);
}

// Recovered uniforms farther than this outside [0, 1] mark an event that is
// not in a channel's image (its density there is 0).
constexpr double kSupportMargin = 1e-6;

// VEGAS bin of a uniform y in (0, 1): floor(y nb), clamped (vegas_map's bin).
__device__ __forceinline__ int vegas_bin(double y, int nb) {
    int i = (int)(y * nb);
    return i < 0 ? 0 : (i > nb - 1 ? nb - 1 : i);
}

// Bytes of dynamic LDS that VEGAS histogram accumulation adds to the fused
// sample kernel: one [vstride] FP64 histogram per wave, then the events' bin
// numbers as bytes [kMaxDims][kBlock].
constexpr size_t vegas_acc_lds(int vstride) {
    return sizeof(double) * (size_t)kWaves * (size_t)vstride + (size_t)kMaxDims * kBlock;
}

// Adds w^2 of this wave's events to the wave's private histogram hw [dims][nb]
// (VEGAS: sum of w^2 per bin of every dimension).  bins points at this
// thread's bin bytes, row k at bins[k kBlock].  Lane b owns bins b and b + 64
// (nb <= 128): for every dimension it collects, in lane order, the squared
// weights of the wave's events with w != 0 that fall in its bins, read from
// the event's lane; no two lanes write the same entry, and the order of the
// sums is fixed, so the result is deterministic.  Called by every lane of the
// wave (live: the lane holds an event).
__device__ __forceinline__ void vegas_wave_accumulate(double* __restrict__ hw, const uint8_t* __restrict__ bins,
                                                      int dims, int nb, int lane, bool live, double wv) {
    const uint64_t nz = __ballot(live && wv != 0.0);
    if (nz == 0) return;
    const double w2 = wv * wv;
    const int lo = __double2loint(w2), hi = __double2hiint(w2);
    for (int k = 0; k < dims; ++k) {
        const int mb = bins[k * kBlock];
        double a0 = 0.0, a1 = 0.0;
        uint64_t m = nz;
        if (nb <= 64) {
            while (m) {
                const int j = __builtin_ctzll(m);
                m &= m - 1;
                const int bj = __builtin_amdgcn_readlane(mb, j);
                const double wj = __hiloint2double(__builtin_amdgcn_readlane(hi, j), __builtin_amdgcn_readlane(lo, j));
                a0 += bj == lane ? wj : 0.0;
            }
        } else {
            while (m) {
                const int j = __builtin_ctzll(m);
                m &= m - 1;
                const int bj = __builtin_amdgcn_readlane(mb, j);
                const double wj = __hiloint2double(__builtin_amdgcn_readlane(hi, j), __builtin_amdgcn_readlane(lo, j));
                a0 += bj == lane ? wj : 0.0;
                a1 += bj == lane + 64 ? wj : 0.0;
            }
        }
        if (lane < nb) hw[k * nb + lane] += a0;
        if (lane + 64 < nb) hw[k * nb + lane + 64] += a1;
    }
}

// Deterministic wave-level reductions (fixed butterfly order).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

}  // namespace msx
