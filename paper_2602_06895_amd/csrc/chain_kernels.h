// The mapping-chain kernels (single-channel map and fused multichannel
// sample) as templates over the register class (NS momentum slots, NI
// invariants), the compiled map kinds and the precision.  Each instantiation
// unit includes this header and instantiates launch_chain_class for one
// (NS, NI, precision); the units compile in parallel.
#pragma once

#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#endif

#include "chain.h"
#include "device_util.h"

namespace msx {

// Per-thread column of the invariant store in LDS: kQRows doubles with
// stride kBlock (conflict-free across a wave).  It occupies the first
// kQBytes of the kernels' dynamic LDS; the VEGAS grid follows.
constexpr size_t kQBytes = sizeof(double) * kQRows * kBlock;

// The fused sample kernel first writes the VEGAS-mapped uniforms of all an
// event's dimensions into the same per-thread column (the chain reads them
// back in order; the integrand's invariant store reuses the column after the
// chain is done).  The channel compiler admits a channel of an (NS, NI)
// class only with at most max(kQRows, NS + NI + 1) dimensions (s-hat and x1,
// the time-like invariants and two per two-body operation fit NS + NI + 1; a
// 1 -> 3 decay takes five for its four slots, a Chili channel 3 n - 2).
template <int NS, int NI>
constexpr int stage_rows() {
    return (NS + NI + 1) > kQRows ? (NS + NI + 1) : kQRows;
}
struct LdsQ {
    double* b;
    __device__ __forceinline__ void set(int u, double x) { b[u * kBlock] = x; }
    __device__ __forceinline__ double get(int u) const { return b[u * kBlock]; }
};

// Beam boost, unphysical cut and (STORE) the stores of one event whose
// partonic-frame momenta sit in the slots.  The final-state momenta are
// gathered by label into statically indexed arrays (NF = the most
// final-state particles an NS-slot channel has), so the stores and the
// integrand index registers with constants; they stay there in the partonic
// frame, with h = sqrt(s-hat)/2.  Returns the event's Jacobian, 0 when it is
// cut.
template <int NS, bool STORE = true>
__device__ __forceinline__ double finish_store(const ChannelTab* __restrict__ ct, const ChainOut& o, double jv,
                                               double (&E)[NS], double (&X)[NS], double (&Y)[NS], double (&Z)[NS],
                                               int np, int64_t n, int64_t e, double* __restrict__ p,
                                               double* __restrict__ x1x2, double* __restrict__ jac_out,
                                               double (&FE)[NS / 2 + 1], double (&FX)[NS / 2 + 1],
                                               double (&FY)[NS / 2 + 1], double (&FZ)[NS / 2 + 1], double& h) {
    constexpr int NF = NS / 2 + 1;
    const int nf = ct->n_final;
    const int hadronic = ct->hadronic;
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
    h = 0.5 * sqrt(o.shat);
    bool ok = true;
    auto store = [&](int i, double pe, double px, double py, double pz) {
        double le = pe, lz = pz;
        if (hadronic) {
            le = g * pe + gb * pz;
            lz = gb * pe + g * pz;
        }
        ok = ok && isfinite(le) && isfinite(px) && isfinite(py) && isfinite(lz) && le >= 0.0;
        if (STORE) {
            p[((int64_t)0 * np + i) * n + e] = le;
            p[((int64_t)1 * np + i) * n + e] = px;
            p[((int64_t)2 * np + i) * n + e] = py;
            p[((int64_t)3 * np + i) * n + e] = lz;
        }
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
        if (STORE && x1x2) {
            x1x2[e] = o.x1;
            x1x2[n + e] = o.x2;
        }
    }
    if (!ok) jac = 0.0;
    if (STORE && jac_out) jac_out[e] = jac;
    return jac;
}

// Stores, then integrand x channel weight of an uncut event.
template <int NS, bool MIX>
__device__ __forceinline__ double finish_event(const ChannelTab* __restrict__ ct, const ProcessTab* __restrict__ pt,
                                               const ChainOut& o, double jv, double (&E)[NS], double (&X)[NS],
                                               double (&Y)[NS], double (&Z)[NS], int np, int64_t n, int64_t e,
                                               double* __restrict__ p, double* __restrict__ x1x2,
                                               double* __restrict__ jac_out, bool want_w, LdsQ q) {
    constexpr int NF = NS / 2 + 1;
    double FE[NF], FX[NF], FY[NF], FZ[NF], h;
    const double jac = finish_store<NS>(ct, o, jv, E, X, Y, Z, np, n, e, p, x1x2, jac_out, FE, FX, FY, FZ, h);
    double w = 0.0;
    if (want_w && jac != 0.0) {
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
            double r = vegas_map_checked(y[(int64_t)k * n + e], lg + k * (nb + 1), nb, jv);
            ++k;
            return r;
        };
        double E[NS], X[NS], Y[NS], Z[NS], S[NI], SQ[NI];
        ChainOut o;
        if ((KINDS & KIND_CHILI) && ct->chili)
            run_chili<NS>(ct, s_lab, next, E, X, Y, Z, o);
        else
            run_chain<NS, NI, KINDS, MIX>(ct, s_lab, next, E, X, Y, Z, S, SQ, o);
        if (!p) {
            // Jacobian only (the density of the inverse map)
            double FE[NS / 2 + 1], FX[NS / 2 + 1], FY[NS / 2 + 1], FZ[NS / 2 + 1], h;
            jac[e] = finish_store<NS, false>(ct, o, jv, E, X, Y, Z, np, n, e, nullptr, nullptr, nullptr, FE, FX, FY,
                                             FZ, h);
            continue;
        }
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
// What the events of one tile need besides their channel's tables.
struct TileArgs {
    int64_t base, end;  // first output position of the tile, end of the channel's range
    int ept;
    uint64_t ctr0, seed, sid;
    const double* lg;  // the channel's VEGAS grid in LDS
    int nb;
    double* col;  // this thread's staging column
    uint8_t* vbin;  // this thread's VEGAS bin bytes, NULL: no accumulation
    double* vh_wave;  // this wave's VEGAS histogram
    int lane, np;
    int64_t ld;
    double* p;
    double* x1x2;
    double* w;
    int32_t* chan_out;
};
struct TileAcc {
    double s1 = 0.0, s2 = 0.0, zeros = 0.0, wmax = 0.0;
};

// The events of one tile of channel c: uniforms (Philox, VEGAS-mapped into
// the staging column), chain, weight, stores, the tile's running statistics
// and (vbin) the VEGAS histogram.  ct and pt are the channel's tables; the
// kernel compiled for a fixed set of channels passes them as constants.
template <int NS, int NI, int KINDS, bool MIX>
__device__ __forceinline__ void sample_tile(const ChannelTab* __restrict__ ct, const ProcessTab* __restrict__ pt,
                                            int c, const TileArgs& t, TileAcc& acc) {
    const int dims = ct->dims;
    const double s_lab = pt->s_lab;
    const LdsQ q{t.col};
    double* const col = t.col;
    for (int sub = 0; sub < t.ept; ++sub) {
        const int64_t pos0 = t.base + (int64_t)sub * kBlock;
        if (pos0 >= t.end) break;
        const int64_t pos = pos0 + threadIdx.x;
        const bool live = pos < t.end;
        double wv = 0.0;
        if (live) {
            const uint64_t e = t.ctr0 + (uint64_t)pos;
            // all dimensions first, four per Philox block, VEGAS-mapped
            // into this thread's LDS column: one copy of the generator in
            // the code instead of one per place the chain draws a number
            double jv = 1.0;
#pragma unroll 1
            for (int k4 = 0; k4 < dims; k4 += 4) {
                uint64_t c0 = e, c1 = (uint64_t)(k4 >> 2), c2 = 0, c3 = 0;
                philox4x64_10(c0, c1, c2, c3, t.seed, t.sid);
                const uint64_t wd[4] = {c0, c1, c2, c3};
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (k4 + j < dims) {
                        const double u = to_unit(wd[j]);
                        if (t.vbin) t.vbin[(k4 + j) * kBlock] = (uint8_t)vegas_bin(u, t.nb);
                        col[(k4 + j) * kBlock] = vegas_map(u, t.lg + (k4 + j) * (t.nb + 1), t.nb, jv);
                    }
            }
            int k = 0;
            auto next = [&]() -> double { return col[(k++) * kBlock]; };
            double E[NS], X[NS], Y[NS], Z[NS], S[NI], SQ[NI];
            ChainOut o;
            if ((KINDS & KIND_CHILI) && ct->chili)
                run_chili<NS>(ct, s_lab, next, E, X, Y, Z, o);
            else
                run_chain<NS, NI, KINDS, MIX>(ct, s_lab, next, E, X, Y, Z, S, SQ, o);
            wv = finish_event<NS, MIX>(ct, pt, o, jv, E, X, Y, Z, t.np, t.ld, pos, t.p, t.x1x2, nullptr, true, q);
            t.w[pos] = wv;
            if (t.chan_out) t.chan_out[pos] = c;
            acc.s1 += wv;
            acc.s2 += wv * wv;
            acc.zeros += wv == 0.0 ? 1.0 : 0.0;
            acc.wmax = fmax(acc.wmax, wv);
        }
        if (t.vbin) vegas_wave_accumulate(t.vh_wave, t.vbin, dims, t.nb, t.lane, live, wv);
    }
}

// The persistent loop of the fused sample: block b takes the call's tiles
// b, b + gridDim.x, ... (each tile kBlock * ept events of one channel), one
// channel after the other: `channels(run)` calls run(c, tile) for every
// channel c in order, and run loads c's VEGAS grid into LDS, runs
// tile(t, acc) on each of the block's tiles of c and writes the tile's
// statistics and (vpart) VEGAS histogram.  ROWS is the staging column's
// height; the grid follows it in the dynamic LDS.  A kernel compiled for
// fixed channels passes one run call per channel, each with its own tile
// function, so every channel gets a loop of its own code.
template <int ROWS, class Channels>
__device__ __forceinline__ void sample_loop(const ChannelTab* __restrict__ cts, const double* __restrict__ grids,
                                            const int64_t* __restrict__ grid_off, const int32_t* __restrict__ chan_nb,
                                            const SampleCall* __restrict__ call, uint64_t seed, uint64_t sid,
                                            const uint64_t* __restrict__ ctr_dev, uint64_t ctr_off, int np, int64_t ld,
                                            double* __restrict__ p, double* __restrict__ x1x2, double* __restrict__ w,
                                            int32_t* __restrict__ chan_out, double* __restrict__ tile_stats,
                                            int grid_doubles, double* __restrict__ vpart, int vstride,
                                            Channels&& channels) {
    extern __shared__ double lds[];
    double* lg = lds + ROWS * kBlock;
    __shared__ double red[4][kWaves];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ept = call->ept;
    const int64_t G = gridDim.x;
    const uint64_t ctr0 = ctr_dev ? *ctr_dev : ctr_off;
    // VEGAS histogram accumulation (vpart != NULL): one private histogram
    // [dims][nb] per wave after the grid, then the events' bin numbers as
    // bytes [dims][kBlock]
    double* const vh = lg + grid_doubles;
    double* const vh_wave = vh + wave * vstride;
    uint8_t* const vbin = (uint8_t*)(vh + kWaves * vstride);
    if (vpart) {
        for (int i = threadIdx.x; i < kWaves * vstride; i += kBlock) vh[i] = 0.0;
    }
    auto run = [&](int c, auto&& tile) {
        const int64_t t0 = call->tile_start[c], t1 = call->tile_start[c + 1];
        // this block's first tile of the channel
        int64_t tl = t0 + ((((int64_t)blockIdx.x - t0) % G) + G) % G;
        if (tl >= t1) return;
        const int nb = chan_nb[c];
        const int dims = cts[c].dims;
        __syncthreads();
        const double* g = grids + grid_off[c];
        for (int i = threadIdx.x; i < dims * (nb + 1); i += blockDim.x) lg[i] = g[i];
        __syncthreads();
        for (; tl < t1; tl += G) {
            TileArgs t;
            t.base = call->ev_start[c] + (tl - t0) * (int64_t)kBlock * ept;
            t.end = call->ev_start[c + 1];
            t.ept = ept;
            t.ctr0 = ctr0;
            t.seed = seed;
            t.sid = sid;
            t.lg = lg;
            t.nb = nb;
            t.col = lds + threadIdx.x;
            t.vbin = vpart ? vbin + threadIdx.x : nullptr;
            t.vh_wave = vh_wave;
            t.lane = lane;
            t.np = np;
            t.ld = ld;
            t.p = p;
            t.x1x2 = x1x2;
            t.w = w;
            t.chan_out = chan_out;
            TileAcc acc;
            tile(t, acc);
            double s1 = wave_sum(acc.s1), s2 = wave_sum(acc.s2);
            double nz = wave_sum(acc.zeros);
            double mx = wave_max(acc.wmax);
            if (lane == 0) {
                red[0][wave] = s1;
                red[1][wave] = s2;
                red[2][wave] = nz;
                red[3][wave] = mx;
            }
            __syncthreads();
            if (threadIdx.x < 4) {
                int q = threadIdx.x;
                double a = red[q][0];
                for (int v = 1; v < kWaves; ++v) a = (q == 3) ? fmax(a, red[q][v]) : a + red[q][v];
                tile_stats[tl * 4 + q] = a;
            }
            __syncthreads();
            if (vpart) {
                // the tile's histogram: the wave histograms summed in wave
                // order, then cleared for the next tile
                double* dst = vpart + tl * (int64_t)vstride;
                const int rows = dims * nb;
                for (int i = threadIdx.x; i < rows; i += kBlock) {
                    double a = vh[i];
#pragma unroll
                    for (int v = 1; v < kWaves; ++v) a += vh[v * vstride + i];
                    dst[i] = a;
#pragma unroll
                    for (int v = 0; v < kWaves; ++v) vh[v * vstride + i] = 0.0;
                }
                __syncthreads();
            }
        }
    };
    channels(run);
}

// The fused multichannel sample with the channel tables read from device
// memory (every channel of a context through one register and kind class).
template <int NS, int NI, int KINDS, bool MIX>
__global__ __launch_bounds__(kBlock) void k_sample(const ChannelTab* __restrict__ cts, const ProcessTab* __restrict__ pts,
                                                   const double* __restrict__ grids, const int64_t* __restrict__ grid_off,
                                                   const int32_t* __restrict__ chan_nb,
                                                   const SampleCall* __restrict__ call, uint64_t seed, uint64_t sid,
                                                   const uint64_t* __restrict__ ctr_dev, uint64_t ctr_off, int np,
                                                   int64_t ld, double* __restrict__ p, double* __restrict__ x1x2,
                                                   double* __restrict__ w, int32_t* __restrict__ chan_out,
                                                   double* __restrict__ tile_stats, int grid_doubles,
                                                   double* __restrict__ vpart, int vstride) {
    sample_loop<stage_rows<NS, NI>()>(
        cts, grids, grid_off, chan_nb, call, seed, sid, ctr_dev, ctr_off, np, ld, p, x1x2, w, chan_out, tile_stats,
        grid_doubles, vpart, vstride, [&](auto& run) {
            const int n_chan = call->n_chan;
            for (int c = 0; c < n_chan; ++c)
                run(c, [&](const TileArgs& t, TileAcc& acc) {
                    const ChannelTab* ct = cts + c;
                    sample_tile<NS, NI, KINDS, MIX>(ct, pts + ct->process, c, t, acc);
                });
        });
}

// Inverse of run_chili from the lab-frame momenta p [4][np][n] of event e:
// per particle but the last, p_T -> r (eq. chili_pt_withcut or
// chili_pt_nocut inverted), the rapidity asinh(p_z / m_T) -> r within
// +-y_max, the azimuth measured from the recoil direction of the particles
// before it -> r; then the last particle's rapidity within its range.  The
// uniforms go to the thread's staging column col (stride kBlock).
template <int NF>
__device__ __forceinline__ void chili_unmap(const ChannelTab* __restrict__ ct, double s_lab, int np, int64_t n,
                                            int64_t e, const double* __restrict__ p, double* col) {
    const int nf = ct->n_final;
    const double sq = sqrt(s_lab), ptmax = 0.5 * sq;
    const double ptmin2 = ct->chili_ptmin2;
    double sx = 0.0, sy = 0.0, ep = 0.0, em = 0.0;
    int kd = 0;
    auto put = [&](double r) { col[(kd++) * kBlock] = r; };
    for (int i = 0; i < nf - 1; ++i) {
        const double m = ct->chili_m[i];
        const double px = p[((int64_t)1 * np + i + 2) * n + e], py = p[((int64_t)2 * np + i + 2) * n + e];
        const double pz = p[((int64_t)3 * np + i + 2) * n + e];
        const double pt2 = px * px + py * py;
        if (ptmin2 > 0.0) {
            const double a = 1.0 / (ptmax * ptmax), b = 1.0 / ptmin2;
            put((b - 1.0 / pt2) / (b - a));
        } else {
            const double lam = m > 0.0 ? m : 1.0;
            const double pt = sqrt(pt2);
            put(pt * (2.0 * lam + ptmax) / (ptmax * (2.0 * lam + pt)));
        }
        const double mt = sqrt(pt2 + m * m);
        const double z = sq / (2.0 * mt);
        const double ymax = log(z + sqrt(z * z - 1.0));
        const double yv = asinh(pz / mt);
        put(0.5 * (yv / ymax + 1.0));
        const double ux = i == 0 ? 1.0 : -sx, uy = i == 0 ? 0.0 : -sy;
        put(turn_fraction(ux * px + uy * py, ux * py - uy * px));
        sx += px;
        sy += py;
        ep += mt * exp(yv);
        em += mt * exp(-yv);
    }
    const double m = ct->chili_m[nf - 1];
    const double mt = sqrt(sx * sx + sy * sy + m * m);
    const double ylo = -log((sq - em) / mt), yhi = log((sq - ep) / mt);
    const double yv = asinh(p[((int64_t)3 * np + nf - 1 + 2) * n + e] / mt);
    put((yv - ylo) / (yhi - ylo));
}

// Inverse map of one channel (section 2.1): lab-frame momenta p and momentum
// fractions -> the uniforms y that the chain maps to them (k_map without
// momentum stores then gives the forward Jacobian at y).  Every step of
// run_chain undone in its order: beam boost, s-hat and x1 from x1 x2, the
// invariants from the momenta of their clusters, per 2->2 block |t| =
// -(p_A - p_1)^2 and the azimuth of p_1 about p_A in the rest frame of
// P = p_A + p_B, per decay the angles of the first child in its parent's
// rest frame, then the inverse VEGAS map.  FP64.
template <int NS, int NI, int KINDS>
__global__ __launch_bounds__(kBlock) void k_inverse(const ChannelTab* __restrict__ ct, const double* __restrict__ grid,
                                                    int nb, double s_lab, int np, int64_t n,
                                                    const double* __restrict__ p, const double* __restrict__ x1x2,
                                                    double* __restrict__ y) {
    constexpr int NF = NS / 2 + 1;
    constexpr int kRows = stage_rows<NS, NI>();
    extern __shared__ double lds[];
    double* lg = lds + kRows * kBlock;
    double* const col = lds + threadIdx.x;
    const int dims = ct->dims;
    for (int i = threadIdx.x; i < dims * (nb + 1); i += blockDim.x) lg[i] = grid[i];
    __syncthreads();
    const int nf = ct->n_final;
    const int hadronic = ct->hadronic;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        if ((KINDS & KIND_CHILI) && ct->chili) {
            chili_unmap<NF>(ct, s_lab, np, n, e, p, col);
        } else {
            double x1 = 1.0, x2 = 1.0, g = 1.0, gb = 0.0;
            if (hadronic) {
                x1 = x1x2[e];
                x2 = x1x2[n + e];
                const double inv = 1.0 / (2.0 * sqrt(x1 * x2));
                g = (x1 + x2) * inv;
                gb = (x1 - x2) * inv;
            }
            double FE[NF], FX[NF], FY[NF], FZ[NF];
#pragma unroll
            for (int k = 0; k < NF; ++k) {
                FE[k] = FX[k] = FY[k] = FZ[k] = 0.0;
                if (k < nf) {
                    const double le = p[((int64_t)0 * np + k + 2) * n + e], lz = p[((int64_t)3 * np + k + 2) * n + e];
                    FE[k] = g * le - gb * lz;
                    FX[k] = p[((int64_t)1 * np + k + 2) * n + e];
                    FY[k] = p[((int64_t)2 * np + k + 2) * n + e];
                    FZ[k] = -gb * le + g * lz;
                }
            }
            int kd = 0;
            auto put = [&](double r) { col[(kd++) * kBlock] = r; };
            double S[NI], SQ[NI];
            // (1) s-hat = x1 x2 s_lab
            double shat = s_lab;
            if (hadronic) {
                shat = x1 * x2 * s_lab;
                put(unmap_static<KINDS>(ct->inv[0], shat));
            }
            S[0] = shat;
            SQ[0] = sqrt(shat);
            // (2) time-like invariants from the momenta of their clusters
            const int n_inv = ct->n_inv;
            for (int i = 1; i < n_inv; ++i) {
                const InvSpec& iv = ct->inv[i];
                const double mmin = iv.min_const + masked_sum(iv.min_mask, SQ);
                const double mmax = SQ[iv.parent] - iv.max_const - masked_sum(iv.max_mask, SQ);
                double qe, qx, qy, qz;
                sum_set<NF>(iv.set, FE, FX, FY, FZ, qe, qx, qy, qz);
                const double s = qe * qe - qx * qx - qy * qy - qz * qz;
                put(unmap_dyn<KINDS>(iv.map, s, mmin * mmin, mmax * mmax));
                S[i] = s;
                SQ[i] = sqrt(s);
            }
            // (3) x1 = tau^r
            if (hadronic) put(log(x1) / log(shat / s_lab));
            // (4) 2->2 blocks
            const double h = 0.5 * SQ[0];
            double Ae = h, Ax = 0.0, Ay = 0.0, Az = h;
            double Be = h, Bx = 0.0, By = 0.0, Bz = -h;
            double ma2 = 0.0, mb2 = 0.0;
            const int n_blocks = ct->n_blocks;
#pragma unroll
            for (int bi = 0; bi < NS / 2; ++bi) {
                if (bi >= n_blocks) break;
                const BlockSpec& bs = ct->blk[bi];
                const double m1 = src_mass(bs.m1, SQ), m2 = src_mass(bs.m2, SQ);
                // the leg is a sum of final-state momenta, the remaining cluster
                // P - leg (P = p_A + p_B), as the chain built them
                double p1e, p1x, p1y, p1z, p2e, p2x, p2y, p2z;
                if (bs.side == 1) {
                    sum_set<NF>(bs.set2, FE, FX, FY, FZ, p2e, p2x, p2y, p2z);
                    p1e = (Ae + Be) - p2e;
                    p1x = (Ax + Bx) - p2x;
                    p1y = (Ay + By) - p2y;
                    p1z = (Az + Bz) - p2z;
                } else {
                    sum_set<NF>(bs.set1, FE, FX, FY, FZ, p1e, p1x, p1y, p1z);
                    p2e = (Ae + Be) - p1e;
                    p2x = (Ax + Bx) - p1x;
                    p2y = (Ay + By) - p1y;
                    p2z = (Az + Bz) - p1z;
                }
                const double m0sq = S[bs.m0_inv], m0 = SQ[bs.m0_inv];
                const double m1s = m1 * m1, m2s = m2 * m2;
                const double C = (m0sq + (m1s - m2s)) * (m0sq + (ma2 - mb2));
                const double R = sqrt(kallen(m0sq, m1s, m2s) * kallen(m0sq, ma2, mb2));
                const double inv2 = 1.0 / (2.0 * m0sq);
                const double t_minus = m1s + ma2 - (C + R) * inv2;
                const double prod = (m1s - ma2) * (m2s - mb2) + (ma2 - mb2 - m1s + m2s) * (ma2 * m2s - m1s * mb2) / m0sq;
                const double t_plus = (t_minus != 0.0) ? prod / t_minus : 0.0;
                const double tmin = fmax(0.0, -t_plus), tmax = -t_minus;
                const double de = Ae - p1e, dx = Ax - p1x, dy = Ay - p1y, dz = Az - p1z;
                const double abst = -(de * de - dx * dx - dy * dy - dz * dz);
                double vx = p1x, vy = p1y;
                if ((KINDS & KIND_ST) && ct->st && bi > 0 && !bs.com) {
                    // (s~, t) block: s~ = (p1 + rec)^2 and the orientation of
                    // p1 about the plane of p_A and rec give r (two branches)
                    const BlockSpec& pb = ct->blk[bi > 0 ? bi - 1 : 0];
                    double re, rx, ry, rz;
                    sum_set<NF>(pb.side == 1 ? pb.set2 : pb.set1, FE, FX, FY, FZ, re, rx, ry, rz);
                    const double Pe = Ae + Be, Px = Ax + Bx, Py = Ay + By, Pz = Az + Bz;
                    const double inv_m0 = 1.0 / m0, inv_em = 1.0 / (Pe + m0);
                    double ae = Ae, ax = Ax, ay = Ay, az = Az;
                    boost_by(Pe, -Px, -Py, -Pz, inv_m0, inv_em, ae, ax, ay, az);
                    double ce = re, cx = rx, cy = ry, cz = rz;
                    boost_by(Pe, -Px, -Py, -Pz, inv_m0, inv_em, ce, cx, cy, cz);
                    double ke = p1e, kx = p1x, ky = p1y, kz = p1z;
                    boost_by(Pe, -Px, -Py, -Pz, inv_m0, inv_em, ke, kx, ky, kz);
                    const double inv_len = 1.0 / sqrt(ax * ax + ay * ay + az * az);
                    const double nx = ax * inv_len, ny = ay * inv_len, nz = az * inv_len;
                    const double st = sqrt(nx * nx + ny * ny);
                    double cp = 1.0, sp = 0.0;
                    if (st > 0.0) {
                        const double ist = 1.0 / st;
                        cp = nx * ist;
                        sp = ny * ist;
                    }
                    const double xr = cx * cp + cy * sp, yr = -cx * sp + cy * cp;
                    const double r0 = xr * nz - cz * st, r1 = yr;
                    const double xk = kx * cp + ky * sp, yk = -kx * sp + ky * cp;
                    const double k0 = xk * nz - kz * st, k1 = yk;
                    // u = (s~ - (A - B)) / (2 B) = (1 - cos(phi)) / 2, phi the
                    // angle between the transverse parts of rec and p1
                    const double rperp = sqrt(r0 * r0 + r1 * r1), kperp = sqrt(k0 * k0 + k1 * k1);
                    const double c = fmin(1.0, fmax(-1.0, (r0 * k0 + r1 * k1) / (rperp * kperp)));
                    const double u = 0.5 * (1.0 - c);
                    (void)ce;
                    (void)ke;
                    put(r0 * k1 - r1 * k0 >= 0.0 ? 0.5 * u : 0.5 * (u + 1.0));
                    put(unmap_dyn<KINDS>(bs.tmap, abst, tmin, tmax));
                } else {
                if (!bs.com) {
                    // into the rest frame of P, then R(phi_A, theta_A)^-1 = R_y(-theta_A) R_z(-phi_A)
                    const double Pe = Ae + Be, Px = Ax + Bx, Py = Ay + By, Pz = Az + Bz;
                    const double inv_m0 = 1.0 / m0, inv_em = 1.0 / (Pe + m0);
                    double ae = Ae, ax = Ax, ay = Ay, az = Az;
                    boost_by(Pe, -Px, -Py, -Pz, inv_m0, inv_em, ae, ax, ay, az);
                    double ke = p1e, kx = p1x, ky = p1y, kz = p1z;
                    boost_by(Pe, -Px, -Py, -Pz, inv_m0, inv_em, ke, kx, ky, kz);
                    const double inv_len = 1.0 / sqrt(ax * ax + ay * ay + az * az);
                    const double nx = ax * inv_len, ny = ay * inv_len, nz = az * inv_len;
                    const double st = sqrt(nx * nx + ny * ny);
                    double cp = 1.0, sp = 0.0;
                    if (st > 0.0) {
                        const double ist = 1.0 / st;
                        cp = nx * ist;
                        sp = ny * ist;
                    }
                    const double xr = kx * cp + ky * sp, yr = -kx * sp + ky * cp;
                    vx = xr * nz - kz * st;
                    vy = yr;
                }
                put(turn_fraction(vx, vy));
                put(unmap_dyn<KINDS>(bs.tmap, abst, tmin, tmax));
                }
                const int side = bs.side;
                const double fa = side == 0 ? 1.0 : 0.0, fb = side == 1 ? 1.0 : 0.0;
                Ae -= fa * p1e;
                Ax -= fa * p1x;
                Ay -= fa * p1y;
                Az -= fa * p1z;
                Be -= fb * p2e;
                Bx -= fb * p2x;
                By -= fb * p2y;
                Bz -= fb * p2z;
                ma2 = side == 0 ? -abst : ma2;
                mb2 = side == 1 ? -abst : mb2;
            }
            // (5) decays: angles of the first child in the rest frame of its parent
            const int n_dec = ct->n_decays;
#pragma unroll
            for (int di = 0; di < NS / 2; ++di) {
                if (di >= n_dec) break;
                const DecaySpec& ds = ct->dec[di];
                if ((KINDS & KIND_DEC3) && ds.kind == 2) continue;
                double ke, kx, ky, kz;
                sum_set<NF>(ds.set1, FE, FX, FY, FZ, ke, kx, ky, kz);
                double Pe = 0.0, Px = 0.0, Py = 0.0, Pz = 0.0;
                const double m0 = SQ[ds.parent_inv];
                if (!ds.parent_rest) {
                    sum_set<NF>(ds.parent_set, FE, FX, FY, FZ, Pe, Px, Py, Pz);
                    boost_by(Pe, -Px, -Py, -Pz, 1.0 / m0, 1.0 / (Pe + m0), ke, kx, ky, kz);
                }
                if ((KINDS & KIND_DEC3) && ds.kind == 1) {
                    // 1 -> 3: E1, E2, the direction of p1, and the azimuth of
                    // p2 about p1 (p2 turned by R(phi, theta)^-1 = R_y(-theta) R_z(-phi))
                    double qe, qx, qy, qz;
                    sum_set<NF>(ds.set2, FE, FX, FY, FZ, qe, qx, qy, qz);
                    if (!ds.parent_rest) boost_by(Pe, -Px, -Py, -Pz, 1.0 / m0, 1.0 / (Pe + m0), qe, qx, qy, qz);
                    const double m1 = src_mass(ds.m1, SQ), m2 = src_mass(ds.m2, SQ), m3 = src_mass(ds.m3, SQ);
                    const double w1 = (m0 - m1 - (m2 + m3)) * (m0 - m1 + (m2 + m3)) / (2.0 * m0);
                    put((ke - m1) / w1);
                    const double q1sq = ke * ke - m1 * m1;
                    const double dl = 2.0 * m0 * (0.5 * m0 - ke) + m1 * m1;
                    const double d23 = m2 * m2 - m3 * m3;
                    const double root = sqrt(fmax(0.0, q1sq * ((dl + d23) * (dl + d23) - 4.0 * m2 * m2 * dl)));
                    const double e2min = ((m0 - ke) * (dl + d23) - root) / (2.0 * dl);
                    put((qe - e2min) / (root / dl));
                    const double len = sqrt(kx * kx + ky * ky + kz * kz);
                    const double ux = kx / len, uy = ky / len, uz = kz / len;
                    put(turn_fraction(ux, uy));
                    put(0.5 * (uz + 1.0));
                    const double st = sqrt(ux * ux + uy * uy);
                    const double cp = st > 0.0 ? ux / st : 1.0, sp = st > 0.0 ? uy / st : 0.0;
                    const double ax = cp * qx + sp * qy, ay = -sp * qx + cp * qy;
                    put(turn_fraction(uz * ax - st * qz, ay));
                    continue;
                }
                const double len = sqrt(kx * kx + ky * ky + kz * kz);
                put(turn_fraction(kx, ky));
                put(0.5 * (kz / len + 1.0));
            }
        }
        // (6) inverse VEGAS map
        // recovered uniforms farther than kSupportMargin outside [0, 1]: the
        // event is not in the channel's image; y = NaN marks it (the density
        // pass then gives J = 0)
        bool outside = false;
        for (int k = 0; k < dims; ++k) {
            const double r = col[k * kBlock];
            outside = outside || !(r >= -kSupportMargin && r <= 1.0 + kSupportMargin);
        }
        for (int k = 0; k < dims; ++k)
            y[(int64_t)k * n + e] = outside ? __builtin_nan("") : vegas_unmap(col[k * kBlock], lg + k * (nb + 1), nb);
    }
}

}  // namespace msx
