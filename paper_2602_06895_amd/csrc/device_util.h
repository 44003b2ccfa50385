// Small device helpers shared by the kernels: launch shape, the VEGAS lookup
// and deterministic wave reductions.
#pragma once

#include <hip/hip_runtime.h>

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
