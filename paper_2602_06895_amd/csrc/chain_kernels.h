// The mapping-chain kernels (single-channel map and fused multichannel
// sample) as templates over the register class (NS momentum slots, NI
// invariants), the compiled map kinds and the precision.  Each instantiation
// unit includes this header and instantiates launch_chain_class for one
// (NS, NI, precision); the units compile in parallel.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>

#include "chain.h"
#include "device_util.h"
#include "launch.h"

namespace msx {

// Per-thread column of the invariant store in LDS: kQRows doubles with
// stride kBlock (conflict-free across a wave).  It occupies the first
// kQBytes of the kernels' dynamic LDS; the VEGAS grid follows.
constexpr size_t kQBytes = sizeof(double) * kQRows * kBlock;

// The fused sample kernel first writes the VEGAS-mapped uniforms of all an
// event's dimensions into the same per-thread column (the chain reads them
// back in order; the integrand's invariant store reuses the column after the
// chain is done).  A channel of an (NS, NI) class has at most NS + NI + 1
// dimensions: s-hat and x1, the time-like invariants and two per operation.
template <int NS, int NI>
constexpr int stage_rows() {
    return (NS + NI + 1) > kQRows ? (NS + NI + 1) : kQRows;
}
struct LdsQ {
    double* b;
    __device__ __forceinline__ void set(int u, double x) { b[u * kBlock] = x; }
    __device__ __forceinline__ double get(int u) const { return b[u * kBlock]; }
};

// Beam boost, unphysical cut, integrand x channel weight and the stores of one
// event whose partonic-frame momenta sit in the slots.  The final-state
// momenta are first gathered by label into statically indexed arrays (NF =
// the most final-state particles an NS-slot channel has), so the stores and
// the integrand index registers with constants.
template <int NS, bool MIX>
__device__ __forceinline__ double finish_event(const ChannelTab* __restrict__ ct, const ProcessTab* __restrict__ pt,
                                               const ChainOut& o, double jv, double (&E)[NS], double (&X)[NS],
                                               double (&Y)[NS], double (&Z)[NS], int np, int64_t n, int64_t e,
                                               double* __restrict__ p, double* __restrict__ x1x2,
                                               double* __restrict__ jac_out, bool want_w, LdsQ q) {
    constexpr int NF = NS / 2 + 1;
    const int nf = ct->n_final;
    const int hadronic = ct->hadronic;
    double FE[NF], FX[NF], FY[NF], FZ[NF];
#pragma unroll
    for (int k = 0; k < NF; ++k) {
        FE[k] = FX[k] = FY[k] = FZ[k] = 0.0;
        if (k < nf) {
            const int s = slot_index<NS>(ct->final_slot[k]);
            FE[k] = E[s];
            FX[k] = X[s];
            FY[k] = Y[s];
            FZ[k] = Z[s];
        }
    }
    double g = 1.0, gb = 0.0;
    if (hadronic) {
        double inv = 1.0 / (2.0 * sqrt(o.x1 * o.x2));
        g = (o.x1 + o.x2) * inv;
        gb = (o.x1 - o.x2) * inv;
    }
    const double h = 0.5 * sqrt(o.shat);
    bool ok = true;
    auto store = [&](int i, double pe, double px, double py, double pz) {
        double le = pe, lz = pz;
        if (hadronic) {
            le = g * pe + gb * pz;
            lz = gb * pe + g * pz;
        }
        ok = ok && isfinite(le) && isfinite(px) && isfinite(py) && isfinite(lz) && le >= 0.0;
        p[((int64_t)0 * np + i) * n + e] = le;
        p[((int64_t)1 * np + i) * n + e] = px;
        p[((int64_t)2 * np + i) * n + e] = py;
        p[((int64_t)3 * np + i) * n + e] = lz;
    };
    // incoming partons, then final-state particles by label
    store(0, h, 0.0, 0.0, h);
    store(1, h, 0.0, 0.0, -h);
#pragma unroll
    for (int k = 0; k < NF; ++k)
        if (k < nf) store(k + 2, FE[k], FX[k], FY[k], FZ[k]);
    double jac = o.jac * jv;
    ok = ok && isfinite(jac) && jac > 0.0;
    if (hadronic) {
        ok = ok && o.x1 > 0.0 && o.x1 <= 1.0 && o.x2 > 0.0 && o.x2 <= 1.0;
        if (x1x2) {
            x1x2[e] = o.x1;
            x1x2[n + e] = o.x2;
        }
    }
    if (!ok) jac = 0.0;
    if (jac_out) jac_out[e] = jac;
    double w = 0.0;
    if (want_w && ok) {
        double alpha;
        auto get = [&](int k, int c) -> double {
            return c == 0 ? FE[k] : (c == 1 ? FX[k] : (c == 2 ? FY[k] : FZ[k]));
        };
        double af = integrand_alpha<MIX, NF>(pt, ct->alpha_index, o.x1, o.x2, o.logtau, h, 0.0, 0.0, h, get, q, alpha);
        w = af * jac;
    }
    return w;
}

template <int NS, int NI, int KINDS, bool MIX>
__global__ __launch_bounds__(kBlock) void k_map(const ChannelTab* __restrict__ ct, const ProcessTab* __restrict__ pt,
                                                const double* __restrict__ grid, int nb, double s_lab, int np,
                                                int64_t n, const double* __restrict__ y, double* __restrict__ p,
                                                double* __restrict__ x1x2, double* __restrict__ jac,
                                                double* __restrict__ w) {
    extern __shared__ double lds[];
    double* lg = lds + kQRows * kBlock;
    const LdsQ q{lds + threadIdx.x};
    const int dims = ct->dims;
    for (int i = threadIdx.x; i < dims * (nb + 1); i += blockDim.x) lg[i] = grid[i];
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        int k = 0;
        double jv = 1.0;
        auto next = [&]() -> double {
            double r = vegas_map(y[(int64_t)k * n + e], lg + k * (nb + 1), nb, jv);
            ++k;
            return r;
        };
        double E[NS], X[NS], Y[NS], Z[NS], S[NI], SQ[NI];
        ChainOut o;
        run_chain<NS, NI, KINDS, MIX>(ct, s_lab, next, E, X, Y, Z, S, SQ, o);
        double wv = finish_event<NS, MIX>(ct, pt, o, jv, E, X, Y, Z, np, n, e, p, x1x2, jac, w != nullptr, q);
        if (w) w[e] = wv;
    }
}

// All channels in one persistent launch.  The call table (per-channel tile
// and event ranges, events per thread) is read from device memory, so a
// captured graph can be replayed with new counts.  A tile is kBlock * ept
// events of one channel; block b takes tiles b, b + gridDim, ... (static, so
// per-tile statistics are reproducible for a given launch shape).  Each tile
// writes (sum w, sum w^2, n(w == 0), max w) to tile_stats.  Per-event results
// do not depend on the launch shape: the uniforms are keyed by event id.
template <int NS, int NI, int KINDS, bool MIX>
__global__ __launch_bounds__(kBlock) void k_sample(const ChannelTab* __restrict__ cts, const ProcessTab* __restrict__ pts,
                                                   const double* __restrict__ grids, const int64_t* __restrict__ grid_off,
                                                   const int32_t* __restrict__ chan_nb,
                                                   const SampleCall* __restrict__ call, uint64_t seed, uint64_t sid,
                                                   const uint64_t* __restrict__ ctr_dev, uint64_t ctr_off, int np,
                                                   int64_t ld, double* __restrict__ p, double* __restrict__ x1x2,
                                                   double* __restrict__ w, int32_t* __restrict__ chan_out,
                                                   double* __restrict__ tile_stats) {
    constexpr int kRows = stage_rows<NS, NI>();
    extern __shared__ double lds[];
    double* lg = lds + kRows * kBlock;
    double* const col = lds + threadIdx.x;
    const LdsQ q{col};
    __shared__ double red[4][kWaves];
    int cur = -1;
    int nb = 0, dims = 0;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t n_tiles = call->n_tiles;
    const int n_chan = call->n_chan;
    const int ept = call->ept;
    const uint64_t ctr0 = ctr_dev ? *ctr_dev : ctr_off;
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        int c = 0;
        while (c + 1 < n_chan && call->tile_start[c + 1] <= tile) ++c;
        const ChannelTab* ct = cts + c;
        if (c != cur) {
            __syncthreads();
            nb = chan_nb[c];
            dims = ct->dims;
            const double* g = grids + grid_off[c];
            for (int i = threadIdx.x; i < dims * (nb + 1); i += blockDim.x) lg[i] = g[i];
            __syncthreads();
            cur = c;
        }
        const ProcessTab* pt = pts + ct->process;
        const double s_lab = pt->s_lab;
        const int64_t base = call->ev_start[c] + (tile - call->tile_start[c]) * (int64_t)kBlock * ept;
        const int64_t end = call->ev_start[c + 1];
        double a1 = 0.0, a2 = 0.0, az = 0.0, am = 0.0;
        for (int sub = 0; sub < ept; ++sub) {
            const int64_t pos = base + (int64_t)sub * kBlock + threadIdx.x;
            if (pos >= end) break;
            const uint64_t e = ctr0 + (uint64_t)pos;
            // all dimensions first, four per Philox block, VEGAS-mapped into
            // this thread's LDS column: one copy of the generator in the code
            // instead of one per place the chain draws a number
            double jv = 1.0;
#pragma unroll 1
            for (int k4 = 0; k4 < dims; k4 += 4) {
                uint64_t c0 = e, c1 = (uint64_t)(k4 >> 2), c2 = 0, c3 = 0;
                philox4x64_10(c0, c1, c2, c3, seed, sid);
                const uint64_t wd[4] = {c0, c1, c2, c3};
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (k4 + j < dims) col[(k4 + j) * kBlock] = vegas_map(to_unit(wd[j]), lg + (k4 + j) * (nb + 1), nb, jv);
            }
            int k = 0;
            auto next = [&]() -> double { return col[(k++) * kBlock]; };
            double E[NS], X[NS], Y[NS], Z[NS], S[NI], SQ[NI];
            ChainOut o;
            run_chain<NS, NI, KINDS, MIX>(ct, s_lab, next, E, X, Y, Z, S, SQ, o);
            const double wv = finish_event<NS, MIX>(ct, pt, o, jv, E, X, Y, Z, np, ld, pos, p, x1x2, nullptr, true, q);
            w[pos] = wv;
            if (chan_out) chan_out[pos] = c;
            a1 += wv;
            a2 += wv * wv;
            az += wv == 0.0 ? 1.0 : 0.0;
            am = fmax(am, wv);
        }
        double s1 = wave_sum(a1), s2 = wave_sum(a2);
        double nz = wave_sum(az);
        double mx = wave_max(am);
        if (lane == 0) {
            red[0][wave] = s1;
            red[1][wave] = s2;
            red[2][wave] = nz;
            red[3][wave] = mx;
        }
        __syncthreads();
        if (threadIdx.x < 4) {
            int q = threadIdx.x;
            double acc = red[q][0];
            for (int v = 1; v < kWaves; ++v) acc = (q == 3) ? fmax(acc, red[q][v]) : acc + red[q][v];
            tile_stats[tile * 4 + q] = acc;
        }
        __syncthreads();
    }
}

// Launch of one register class: kind class `kc` picks the compiled map kinds
// (0: integer-root power laws, 1: plus Breit-Wigner, 2: all).
template <int NS, int NI, bool MIX>
hipError_t launch_chain_class(int kc, const ChainLaunch& a) {
    constexpr int K0 = KIND_POW_INT, K1 = KIND_POW_INT | KIND_BW, K2 = KINDS_ALL;
    auto go = [&](auto kt) {
        constexpr int K = decltype(kt)::value;
        const size_t lds = a.lds + (a.sample ? sizeof(double) * stage_rows<NS, NI>() * kBlock : kQBytes);
        if (lds > 65536) {
            // beyond the default 64 KiB per workgroup (gfx950 has 160 KiB per CU)
            const void* fn = a.sample ? (const void*)k_sample<NS, NI, K, MIX> : (const void*)k_map<NS, NI, K, MIX>;
            hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return;
        }
        if (a.sample)
            k_sample<NS, NI, K, MIX><<<a.grid, kBlock, lds, a.stream>>>(
                a.cts, a.pts, a.grids, a.grid_off, a.chan_nb, a.call, a.seed, a.sid, a.ctr_dev, a.ctr_off, a.np, a.n,
                a.p, a.x1x2, a.w, a.chan, a.tile_stats);
        else
            k_map<NS, NI, K, MIX><<<a.grid, kBlock, lds, a.stream>>>(a.cts, a.pts, a.grids, a.nb, a.s_lab, a.np, a.n,
                                                                         a.y, a.p, a.x1x2, a.jac, a.w);
    };
    if (kc == 0) go(std::integral_constant<int, K0>{});
    else if (kc <= 1) go(std::integral_constant<int, K1>{});
    else go(std::integral_constant<int, K2>{});
    return hipGetLastError();
}

#define MSX_INSTANTIATE_CHAIN(NS, NI, MIX) \
    template hipError_t launch_chain_class<NS, NI, MIX>(int kc, const ChainLaunch& a);

}  // namespace msx
