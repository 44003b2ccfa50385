// gfx950 kernels of the phase-space hot path and their host launchers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>

#include "chain.h"
#include "device_util.h"
#include "launch.h"

namespace msx {

namespace {

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_uniform(uint64_t seed, uint64_t sid, uint64_t e0, int64_t n, int d,
                                                    double* __restrict__ y) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t e = e0 + (uint64_t)i;
    for (int g = 0; g < (d + 3) / 4; ++g) {
        uint64_t c0 = e, c1 = (uint64_t)g, c2 = 0, c3 = 0;
        philox4x64_10(c0, c1, c2, c3, seed, sid);
        const uint64_t wv[4] = {c0, c1, c2, c3};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            int k = 4 * g + j;
            if (k < d) y[(int64_t)k * n + i] = to_unit(wv[j]);
        }
    }
}

template <bool MIX>
__global__ __launch_bounds__(kBlock) void k_weight(const ChannelTab* __restrict__ ct, const ProcessTab* __restrict__ pt,
                                                   int np, int64_t n, const double* __restrict__ p,
                                                   const double* __restrict__ x1x2, const double* __restrict__ jac,
                                                   double* __restrict__ w, double* __restrict__ alpha) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    double j = jac[e];
    double wv = 0.0, av = 0.0;
    if (j != 0.0) {
        double x1 = 1.0, x2 = 1.0, L = 0.0;
        if (ct->hadronic) {
            x1 = x1x2[e];
            x2 = x1x2[n + e];
            L = t_log<MIX>(x1 * x2);
        }
        auto get = [&](int k, int c) -> double { return p[((int64_t)c * np + k + 2) * n + e]; };
        double pae = p[((int64_t)0 * np) * n + e], pax = p[((int64_t)1 * np) * n + e];
        double pay = p[((int64_t)2 * np) * n + e], paz = p[((int64_t)3 * np) * n + e];
        RegQ q;
        double af = integrand_alpha<MIX, kMaxFinal>(pt, ct->alpha_index, x1, x2, L, pae, pax, pay, paz, get, q, av);
        wv = af * j;
    }
    w[e] = wv;
    if (alpha) alpha[e] = av;
}

// Reduce the tiles of each channel in order and add to the accumulators
// stats[c] = (sum w, sum w^2, n, n(w == 0), max w).
__global__ __launch_bounds__(kBlock) void k_stats_final(const SampleCall* __restrict__ call,
                                                        const double* __restrict__ tile_stats,
                                                        double* __restrict__ stats) {
    const int c = blockIdx.x;
    __shared__ double red[4][kWaves];
    if (c >= call->n_chan || ((call->skip_mask >> c) & 1)) return;
    const int64_t t0 = call->tile_start[c], t1 = call->tile_start[c + 1];
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t t = t0 + threadIdx.x; t < t1; t += blockDim.x) {
        a[0] += tile_stats[t * 4 + 0];
        a[1] += tile_stats[t * 4 + 1];
        a[2] += tile_stats[t * 4 + 2];
        a[3] = fmax(a[3], tile_stats[t * 4 + 3]);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double r0 = wave_sum(a[0]), r1 = wave_sum(a[1]), r2 = wave_sum(a[2]), r3 = wave_max(a[3]);
    if (lane == 0) {
        red[0][wave] = r0;
        red[1][wave] = r1;
        red[2][wave] = r2;
        red[3][wave] = r3;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s0 = red[0][0], s1 = red[1][0], s2 = red[2][0], mx = red[3][0];
        for (int v = 1; v < kWaves; ++v) {
            s0 += red[0][v];
            s1 += red[1][v];
            s2 += red[2][v];
            mx = fmax(mx, red[3][v]);
        }
        double* st = stats + 5 * c;
        st[0] += s0;
        st[1] += s1;
        st[2] += (double)(call->ev_start[c + 1] - call->ev_start[c]);
        st[3] += s2;
        st[4] = fmax(st[4], mx);
    }
}

// Hit-or-miss unweighting (the paper's channel-wise unweighting against an
// estimated maximum weight): event i is kept when u_i w_max < w_i, u_i the
// Philox uniform of event id e0 + i (dimension 0, as msx_uniform), and
// carries the unit weight max(1, w_i / w_max) (overweight events above 1).
// Pass 1 counts the kept events of every block of kUnwPer events; a one-
// workgroup scan turns the counts into offsets; pass 2 writes the kept
// indices in increasing order (ranks within a block from wave ballots).
constexpr int kUnwPer = kBlock * 4;  // events per block

__device__ __forceinline__ bool unw_keep(const double* __restrict__ w, int64_t i, double w_max, uint64_t seed,
                                         uint64_t sid, uint64_t e0) {
    uint64_t c0 = e0 + (uint64_t)i, c1 = 0, c2 = 0, c3 = 0;
    philox4x64_10(c0, c1, c2, c3, seed, sid);
    return to_unit(c0) * w_max < w[i];
}

__global__ __launch_bounds__(kBlock) void k_unw_count(const double* __restrict__ w, int64_t n, double w_max,
                                                      uint64_t seed, uint64_t sid, uint64_t e0,
                                                      int64_t* __restrict__ blk) {
    __shared__ int red[kWaves];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int c = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t i = (int64_t)blockIdx.x * kUnwPer + q * kBlock + threadIdx.x;
        if (i < n && unw_keep(w, i, w_max, seed, sid, e0)) ++c;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if (lane == 0) red[wave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int v = 0; v < kWaves; ++v) t += red[v];
        blk[blockIdx.x] = t;
    }
}

// Exclusive scan of nb block counts in place (one workgroup: every thread
// sums a contiguous run, the run totals are scanned in LDS); total to *count.
__global__ __launch_bounds__(1024) void k_unw_scan(int64_t* __restrict__ blk, int64_t nb, int64_t* __restrict__ count) {
    __shared__ int64_t tot[1024];
    const int t = threadIdx.x;
    const int64_t per = (nb + 1023) / 1024;
    const int64_t b0 = t * per, b1 = min(nb, b0 + per);
    int64_t s = 0;
    for (int64_t b = b0; b < b1; ++b) s += blk[b];
    tot[t] = s;
    __syncthreads();
    if (t == 0) {
        int64_t acc = 0;
        for (int v = 0; v < 1024; ++v) {
            const int64_t x = tot[v];
            tot[v] = acc;
            acc += x;
        }
        *count = acc;
    }
    __syncthreads();
    int64_t acc = tot[t];
    for (int64_t b = b0; b < b1; ++b) {
        const int64_t x = blk[b];
        blk[b] = acc;
        acc += x;
    }
}

__global__ __launch_bounds__(kBlock) void k_unw_write(const double* __restrict__ w, int64_t n, double w_max,
                                                      uint64_t seed, uint64_t sid, uint64_t e0,
                                                      const int64_t* __restrict__ blk, int64_t* __restrict__ keep,
                                                      double* __restrict__ uw) {
    __shared__ int wcnt[kWaves];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int64_t base = blk[blockIdx.x];
#pragma unroll 1
    for (int q = 0; q < 4; ++q) {
        const int64_t i = (int64_t)blockIdx.x * kUnwPer + q * kBlock + threadIdx.x;
        const bool k = i < n && unw_keep(w, i, w_max, seed, sid, e0);
        const uint64_t bal = __ballot(k);
        if (lane == 0) wcnt[wave] = __popcll(bal);
        __syncthreads();
        int off = 0, all = 0;
#pragma unroll
        for (int v = 0; v < kWaves; ++v) {
            off += v < wave ? wcnt[v] : 0;
            all += wcnt[v];
        }
        if (k) {
            const int64_t pos = base + off + __popcll(bal & ((1ull << lane) - 1));
            keep[pos] = i;
            if (uw) uw[pos] = fmax(1.0, w[i] / w_max);
        }
        base += all;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Observables, cuts and weighted histograms of lab-frame events
// ---------------------------------------------------------------------------
struct ObsK {
    int32_t kind;   // MSX_OBS_* of msx.h
    uint32_t set;   // final-state particle labels
    int32_t rank;   // MSX_OBS_PT_RANK: 0 = hardest
    int32_t pad;
};
constexpr int kObsE = 0, kObsPt = 1, kObsEta = 2, kObsPhi = 3, kObsM = 4, kObsPtRank = 5, kObsDrHardest = 6;
constexpr int kObsMaxFinal = 16;

__device__ __forceinline__ double pt_of(double px, double py) { return sqrt(px * px + py * py); }
__device__ __forceinline__ double eta_of(double px, double py, double pz) { return asinh(pz / pt_of(px, py)); }

// The two hardest particles of `set` (pT descending, lower label first on
// ties): their labels; rank-th hardest pT.
__device__ __forceinline__ void hardest(const double* __restrict__ p, int np, int64_t n, int64_t e, uint32_t set,
                                        int rank, double& pt_rank, int& a, int& b) {
    a = -1;
    b = -1;
    double pa = -1.0, pb = -1.0;
    pt_rank = 0.0;
    // selection of the rank-th largest by counting: pT_i is the rank-th hardest
    // when exactly rank particles are harder (or as hard with a lower label)
    for (int i = 0; i < np - 2; ++i) {
        if (!(set & (1u << i))) continue;
        const double pi = pt_of(p[((int64_t)1 * np + i + 2) * n + e], p[((int64_t)2 * np + i + 2) * n + e]);
        if (pi > pa) {
            pb = pa;
            b = a;
            pa = pi;
            a = i;
        } else if (pi > pb) {
            pb = pi;
            b = i;
        }
        int harder = 0;
        for (int j = 0; j < np - 2; ++j) {
            if (j == i || !(set & (1u << j))) continue;
            const double pj = pt_of(p[((int64_t)1 * np + j + 2) * n + e], p[((int64_t)2 * np + j + 2) * n + e]);
            if (pj > pi || (pj == pi && j < i)) ++harder;
        }
        if (harder == rank) pt_rank = pi;
    }
}

__device__ double obs_value(const ObsK& o, const double* __restrict__ p, int np, int64_t n, int64_t e) {
    if (o.kind == kObsPtRank || o.kind == kObsDrHardest) {
        double ptr;
        int a, b;
        hardest(p, np, n, e, o.set, o.rank, ptr, a, b);
        if (o.kind == kObsPtRank) return ptr;
        if (a < 0 || b < 0) return 0.0;
        const double ax = p[((int64_t)1 * np + a + 2) * n + e], ay = p[((int64_t)2 * np + a + 2) * n + e],
                     az = p[((int64_t)3 * np + a + 2) * n + e];
        const double bx = p[((int64_t)1 * np + b + 2) * n + e], by = p[((int64_t)2 * np + b + 2) * n + e],
                     bz = p[((int64_t)3 * np + b + 2) * n + e];
        const double deta = eta_of(ax, ay, az) - eta_of(bx, by, bz);
        double dphi = fabs(atan2(ay, ax) - atan2(by, bx));
        if (dphi > kPiD) dphi = 2.0 * kPiD - dphi;
        return sqrt(deta * deta + dphi * dphi);
    }
    double E = 0.0, X = 0.0, Y = 0.0, Z = 0.0;
    for (int i = 0; i < np - 2; ++i) {
        if (!(o.set & (1u << i))) continue;
        E += p[((int64_t)0 * np + i + 2) * n + e];
        X += p[((int64_t)1 * np + i + 2) * n + e];
        Y += p[((int64_t)2 * np + i + 2) * n + e];
        Z += p[((int64_t)3 * np + i + 2) * n + e];
    }
    switch (o.kind) {
        case kObsE: return E;
        case kObsPt: return pt_of(X, Y);
        case kObsEta: return eta_of(X, Y, Z);
        case kObsPhi: return atan2(Y, X);
        default: return sqrt(fmax(E * E - X * X - Y * Y - Z * Z, 0.0));
    }
}

struct ObsList {
    ObsK o[8];
};

__global__ __launch_bounds__(kBlock) void k_observables(const double* __restrict__ p, int np, int64_t n, ObsList ol,
                                                        int k, double* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    for (int j = 0; j < k; ++j) out[(int64_t)j * n + e] = obs_value(ol.o[j], p, np, n, e);
}

struct CutList {
    double lo[8], hi[8];
};

// w[e] = 0 unless lo_j <= x[j][e] < hi_j for every observable j.
__global__ __launch_bounds__(kBlock) void k_cut(const double* __restrict__ x, int k, int64_t n, CutList cl,
                                                double* __restrict__ w) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    bool pass = true;
    for (int j = 0; j < k; ++j) {
        const double v = x[(int64_t)j * n + e];
        pass = pass && v >= cl.lo[j] && v < cl.hi[j];
    }
    if (!pass) w[e] = 0.0;
}

// Weighted histogram, deterministic: a workgroup takes kHistPer consecutive
// events, stages (bin, w) in LDS, and thread t sums the events of bins t,
// t + 256, ... in event order; partials [block][2][nb] are then added over
// blocks in a fixed order.  bin = floor((x - lo) * scale), events with
// x outside [lo, hi) skipped.
constexpr int kHistPer = 2048;

__global__ __launch_bounds__(kBlock) void k_hist_block(const double* __restrict__ x, const double* __restrict__ w,
                                                       int64_t n, int nb, double lo, double hi, double scale,
                                                       double* __restrict__ part) {
    __shared__ int sb[kHistPer];
    __shared__ double sw[kHistPer];
    const int64_t e0 = (int64_t)blockIdx.x * kHistPer;
    const int cnt = (int)min<int64_t>(kHistPer, n - e0);
    for (int i = threadIdx.x; i < kHistPer; i += blockDim.x) {
        int b = -1;
        double wv = 0.0;
        if (i < cnt) {
            const double v = x[e0 + i];
            wv = w[e0 + i];
            if (v >= lo && v < hi) {
                b = (int)floor((v - lo) * scale);
                b = b < 0 ? 0 : (b > nb - 1 ? nb - 1 : b);
            }
        }
        sb[i] = b;
        sw[i] = wv;
    }
    __syncthreads();
    for (int bin = threadIdx.x; bin < nb; bin += blockDim.x) {
        double s1 = 0.0, s2 = 0.0;
        for (int i = 0; i < cnt; ++i) {
            if (sb[i] == bin) {
                const double wv = sw[i];
                s1 += wv;
                s2 += wv * wv;
            }
        }
        part[((int64_t)blockIdx.x * 2 + 0) * nb + bin] = s1;
        part[((int64_t)blockIdx.x * 2 + 1) * nb + bin] = s2;
    }
}

// out[i] = sum over blocks z of part[z][i] (i < M), four waves over z = w,
// w + 4, ... with four accumulators each, fixed combination order.
__global__ __launch_bounds__(256) void k_reduce_blocks(const double* __restrict__ part, int64_t nz, int64_t M,
                                                       double* __restrict__ out) {
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t i = (int64_t)blockIdx.x * 64 + lane;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    if (i < M) {
        int64_t z = wv;
        for (; z + 12 < nz; z += 16) {
            a0 += part[z * M + i];
            a1 += part[(z + 4) * M + i];
            a2 += part[(z + 8) * M + i];
            a3 += part[(z + 12) * M + i];
        }
        for (; z < nz; z += 4) a0 += part[z * M + i];
    }
    red[wv][lane] = (a0 + a1) + (a2 + a3);
    __syncthreads();
    if (wv == 0 && i < M) out[i] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
}

// Global multichannel density: g += alpha / J of one channel (g = alpha / J
// for the first channel).  A channel whose chain cuts the event (J = 0)
// contributes nothing.
__global__ __launch_bounds__(kBlock) void k_density_add(double* __restrict__ g, const double* __restrict__ jac,
                                                        double alpha, int64_t n, int first) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double j = jac[i];
    const double t = j > 0.0 ? alpha / j : 0.0;
    g[i] = first ? t : g[i] + t;
}

__global__ void k_set_call(SampleCall call, SampleCall* __restrict__ dev) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dev = call;
}

// VEGAS histograms of a fused sample: entry i of the context's histogram
// array (channel c from the offsets, i - hist_off[c] within its [dims][nb]
// block) gets the sum over c's tiles, in tile order, of the tiles' partials.
__global__ __launch_bounds__(kBlock) void k_vegas_tiles(const SampleCall* __restrict__ call,
                                                        const int64_t* __restrict__ hist_off, int64_t hist_total,
                                                        int vstride, const double* __restrict__ vpart,
                                                        double* __restrict__ hist) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= hist_total) return;
    const int n_chan = call->n_chan;
    int c = 0;
    while (c + 1 < n_chan && hist_off[c + 1] <= i) ++c;
    const int64_t r = i - hist_off[c];
    const int64_t t0 = call->tile_start[c], t1 = call->tile_start[c + 1];
    double acc = 0.0;
    for (int64_t t = t0; t < t1; ++t) acc += vpart[t * vstride + r];
    hist[i] += acc;
}

// Call table from device-resident counts (one thread: at most kMaxChannels).
__global__ void k_plan(const int64_t* __restrict__ counts, int n_chan, int64_t capacity, int ept,
                       SampleCall* __restrict__ dev, int32_t* __restrict__ status) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int64_t T = (int64_t)kBlock * ept;
    int64_t N = 0, tiles = 0;
    int bad = 0;
    dev->n_chan = n_chan;
    dev->ept = ept;
    dev->skip_mask = 0;
    for (int c = 0; c < n_chan; ++c) {
        const int64_t k = counts[c];
        dev->ev_start[c] = N;
        dev->tile_start[c] = tiles;
        if (k < 0 || k > capacity - N) {
            bad = 1;
        } else {
            N += k;
            tiles += (k + T - 1) / T;
        }
    }
    dev->ev_start[n_chan] = N;
    dev->tile_start[n_chan] = tiles;
    dev->n_tiles = bad ? 0 : tiles;
    if (bad) {
        // no events: empty ranges everywhere
        for (int c = 0; c <= n_chan; ++c) {
            dev->ev_start[c] = 0;
            dev->tile_start[c] = 0;
        }
    }
    if (status) *status = bad;
}

// VEGAS histogram, pass 1: block (chunk, k) accumulates sum w^2 per bin of
// dimension k over its contiguous event chunk; each thread keeps a private
// row in LDS (visited in event order), rows are then summed in thread order.
__global__ __launch_bounds__(128) void k_vegas_partial(int64_t n, int nb, const double* __restrict__ y,
                                                       const double* __restrict__ w, int64_t chunk,
                                                       double* __restrict__ part) {
    extern __shared__ double rows[];  // [blockDim][nb]
    const int k = blockIdx.y;
    const int64_t b = blockIdx.x;
    const int tid = threadIdx.x;
    double* mine = rows + (int64_t)tid * nb;
    for (int i = 0; i < nb; ++i) mine[i] = 0.0;
    const int64_t lo = b * chunk, hi = min(n, lo + chunk);
    for (int64_t e = lo + tid; e < hi; e += blockDim.x) {
        double t = y[(int64_t)k * n + e] * nb;
        int i = (int)t;
        i = i < 0 ? 0 : (i > nb - 1 ? nb - 1 : i);
        double wv = w[e];
        mine[i] += wv * wv;
    }
    __syncthreads();
    for (int i = tid; i < nb; i += blockDim.x) {
        double acc = 0.0;
        for (int q = 0; q < (int)blockDim.x; ++q) acc += rows[(int64_t)q * nb + i];
        part[((int64_t)k * gridDim.x + b) * nb + i] = acc;
    }
}

// Pass 2: hist[k][i] += sum over chunks in order.
__global__ void k_vegas_reduce(int dims, int nb, int64_t nchunk, const double* __restrict__ part,
                               double* __restrict__ hist) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= dims * nb) return;
    int k = idx / nb, i = idx % nb;
    double acc = 0.0;
    for (int64_t b = 0; b < nchunk; ++b) acc += part[((int64_t)k * nchunk + b) * nb + i];
    hist[(int64_t)k * nb + i] += acc;
}

// Grid refinement, one thread per (channel, dimension): smoothing (1,6,1)/8
// with (7,1)/8 at the ends, normalisation, damping
// omega_i = ((1 - d_i)/ln(1/d_i))^alpha, then new edges holding equal shares
// of sum(omega), linear inside old bins.  The histogram is cleared.
__global__ void k_vegas_refine(int n_rows, const int32_t* __restrict__ row_nb, const int64_t* __restrict__ row_grid,
                               const int64_t* __restrict__ row_hist, double alpha, double* __restrict__ grids,
                               double* __restrict__ hist) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rows) return;
    const int nb = row_nb[r];
    double* e = grids + row_grid[r];
    double* d = hist + row_hist[r];
    double tot = 0.0;
    for (int i = 0; i < nb; ++i) tot += d[i];
    if (tot > 0.0) {
        double sm[kMaxBins], om[kMaxBins], old[kMaxBins + 1];
        if (nb == 1) {
            sm[0] = d[0];
        } else {
            sm[0] = (7.0 * d[0] + d[1]) / 8.0;
            sm[nb - 1] = (d[nb - 2] + 7.0 * d[nb - 1]) / 8.0;
            for (int i = 1; i < nb - 1; ++i) sm[i] = (d[i - 1] + 6.0 * d[i] + d[i + 1]) / 8.0;
        }
        double ssum = 0.0;
        for (int i = 0; i < nb; ++i) ssum += sm[i];
        double total = 0.0;
        for (int i = 0; i < nb; ++i) {
            double v = sm[i] / ssum;
            double o;
            if (v <= 0.0) o = 0.0;
            else if (v >= 1.0) o = 1.0;
            else o = pow((1.0 - v) / log(1.0 / v), alpha);
            om[i] = o;
            total += o;
        }
        if (total > 0.0) {
            for (int i = 0; i <= nb; ++i) old[i] = e[i];
            double share = total / nb;
            int i = 0;
            double acc = 0.0;
            for (int j = 1; j < nb; ++j) {
                double target = j * share;
                while (i < nb - 1 && acc + om[i] < target) {
                    acc += om[i];
                    ++i;
                }
                double frac = om[i] > 0.0 ? (target - acc) / om[i] : 0.0;
                frac = fmin(fmax(frac, 0.0), 1.0);
                e[j] = old[i] + (old[i + 1] - old[i]) * frac;
            }
            e[0] = 0.0;
            e[nb] = 1.0;
        }
    }
    for (int i = 0; i < nb; ++i) d[i] = 0.0;
}

// Register-file class of a launch: momentum slots (2 per operation) and
// invariants per event.
int reg_class(int slots, int inv) {
    if (slots <= 6 && inv <= 4) return 0;
    if (slots <= 10 && inv <= 8) return 1;
    return 2;
}

// Map-kind class of a launch: 0 integer-root power laws only, 1 plus
// Breit-Wigner, 2 every tree kind; when the tree kinds fit class 1, 3 with
// Chili channels, 4 with 1 -> 3 decays; 5 for anything else and for (s~, t)
// blocks.
int kind_class(int kinds) {
    if (kinds & KIND_ST) return 5;
    if (kinds & (KIND_CHILI | KIND_DEC3)) {
        if (kinds & ~(KIND_POW_INT | KIND_BW | KIND_CHILI | KIND_DEC3)) return 5;
        if ((kinds & KIND_CHILI) && (kinds & KIND_DEC3)) return 5;
        return (kinds & KIND_CHILI) ? 3 : 4;
    }
    if ((kinds & ~KIND_POW_INT) == 0) return 0;
    if ((kinds & ~(KIND_POW_INT | KIND_BW)) == 0) return 1;
    return 2;
}

int grid_for(int64_t n, int cap) {
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g > cap) g = cap;
    return (int)std::max<int64_t>(g, 1);
}

// Register class -> the instantiation unit compiled for it.
hipError_t launch_chain(int rc, int kc, int mixed, const ChainLaunch& a) {
    if (a.inverse) {
        if (rc == 0) return launch_inverse_class<6, 4>(kc, a);
        if (rc == 1) return launch_inverse_class<10, 8>(kc, a);
        return launch_inverse_class<14, 8>(kc, a);
    }
    if (mixed) {
        if (rc == 0) return launch_chain_class<6, 4, true>(kc, a);
        if (rc == 1) return launch_chain_class<10, 8, true>(kc, a);
        return launch_chain_class<14, 8, true>(kc, a);
    }
    if (rc == 0) return launch_chain_class<6, 4, false>(kc, a);
    if (rc == 1) return launch_chain_class<10, 8, false>(kc, a);
    return launch_chain_class<14, 8, false>(kc, a);
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

hipError_t launch_observables(const double* p, int np, int64_t n, const int32_t* spec, int k, double* out,
                              hipStream_t s) {
    if (n == 0) return hipSuccess;
    ObsList ol{};
    for (int j = 0; j < k; ++j) {
        ol.o[j].kind = spec[4 * j];
        ol.o[j].set = (uint32_t)spec[4 * j + 1];
        ol.o[j].rank = spec[4 * j + 2];
    }
    const int64_t b = (n + kBlock - 1) / kBlock;
    k_observables<<<dim3((unsigned)b), dim3(kBlock), 0, s>>>(p, np, n, ol, k, out);
    return hipGetLastError();
}

hipError_t launch_cut(const double* x, int k, int64_t n, const double* lo, const double* hi, double* w, hipStream_t s) {
    if (n == 0) return hipSuccess;
    CutList cl{};
    for (int j = 0; j < k; ++j) {
        cl.lo[j] = lo[j];
        cl.hi[j] = hi[j];
    }
    const int64_t b = (n + kBlock - 1) / kBlock;
    k_cut<<<dim3((unsigned)b), dim3(kBlock), 0, s>>>(x, k, n, cl, w);
    return hipGetLastError();
}

int64_t histogram_blocks(int64_t n) { return std::max<int64_t>(1, (n + kHistPer - 1) / kHistPer); }

hipError_t launch_histogram(const double* x, const double* w, int64_t n, int nb, double lo, double hi, double* part,
                            double* out, hipStream_t s) {
    const int64_t nz = histogram_blocks(n);
    const double scale = nb / (hi - lo);
    k_hist_block<<<dim3((unsigned)nz), dim3(kBlock), 0, s>>>(x, w, n, nb, lo, hi, scale, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t M = 2 * (int64_t)nb;
    k_reduce_blocks<<<dim3((unsigned)((M + 63) / 64)), dim3(256), 0, s>>>(part, nz, M, out);
    return hipGetLastError();
}

int64_t unweight_blocks(int64_t n) { return (n + kUnwPer - 1) / kUnwPer; }

hipError_t launch_unweight(const double* w, int64_t n, double w_max, uint64_t seed, uint64_t sid, uint64_t e0,
                           int64_t* blk, int64_t* keep, double* uw, int64_t* count, hipStream_t s) {
    const int64_t nb = unweight_blocks(n);
    if (nb == 0) {
        k_unw_scan<<<1, 1024, 0, s>>>(blk, 0, count);
        return hipGetLastError();
    }
    k_unw_count<<<dim3((unsigned)nb), dim3(kBlock), 0, s>>>(w, n, w_max, seed, sid, e0, blk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_unw_scan<<<1, 1024, 0, s>>>(blk, nb, count);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_unw_write<<<dim3((unsigned)nb), dim3(kBlock), 0, s>>>(w, n, w_max, seed, sid, e0, blk, keep, uw);
    return hipGetLastError();
}

hipError_t launch_density_add(double* g, const double* jac, double alpha, int64_t n, bool first, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int64_t b = (n + kBlock - 1) / kBlock;
    k_density_add<<<dim3((unsigned)b), dim3(kBlock), 0, s>>>(g, jac, alpha, n, first ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_uniform(uint64_t seed, uint64_t sid, uint64_t e0, int64_t n, int d, double* y, hipStream_t s) {
    if (n == 0) return hipSuccess;
    int64_t g = (n + kBlock - 1) / kBlock;
    k_uniform<<<dim3((unsigned)g), dim3(kBlock), 0, s>>>(seed, sid, e0, n, d, y);
    return hipGetLastError();
}

hipError_t launch_map(const ChannelTab* ct, const ProcessTab* pt, const double* grid, int nb, int dims, int n_slots,
                      int n_inv, int kinds, int mixed, double s_lab, int np, int64_t n, const double* y, double* p,
                      double* x1x2, double* jac, double* w, int cu_count, hipStream_t s) {
    if (n == 0) return hipSuccess;
    ChainLaunch a{};
    a.sample = false;
    a.lds = sizeof(double) * (size_t)dims * (nb + 1);
    a.grid = grid_for(n, cu_count * 8);
    a.stream = s;
    a.cts = ct;
    a.pts = pt;
    a.grids = grid;
    a.nb = nb;
    a.s_lab = s_lab;
    a.np = np;
    a.n = n;
    a.y = y;
    a.p = p;
    a.x1x2 = x1x2;
    a.jac = jac;
    a.w = w;
    return launch_chain(reg_class(n_slots, n_inv), kind_class(kinds), mixed, a);
}

hipError_t launch_inverse(const ChannelTab* ct, const double* grid, int nb, int dims, int n_slots, int n_inv, int kinds,
                          double s_lab, int np, int64_t n, const double* p, const double* x1x2, double* y, double* jac,
                          int cu_count, hipStream_t s) {
    if (n == 0) return hipSuccess;
    ChainLaunch a{};
    a.inverse = true;
    a.lds = sizeof(double) * (size_t)dims * (nb + 1);
    a.grid = grid_for(n, cu_count * 8);
    a.stream = s;
    a.cts = ct;
    a.grids = grid;
    a.nb = nb;
    a.s_lab = s_lab;
    a.np = np;
    a.n = n;
    a.p_in = p;
    a.x1x2_in = x1x2;
    a.y_out = y;
    // always the FP64 units
    hipError_t err = launch_chain(reg_class(n_slots, n_inv), kind_class(kinds), 0, a);
    if (err != hipSuccess || !jac) return err;
    // the forward Jacobian at y: the map kernel without momentum stores
    ChainLaunch m{};
    m.lds = a.lds;
    m.grid = a.grid;
    m.stream = s;
    m.cts = ct;
    m.grids = grid;
    m.nb = nb;
    m.s_lab = s_lab;
    m.np = np;
    m.n = n;
    m.y = y;
    m.jac = jac;
    return launch_chain(reg_class(n_slots, n_inv), kind_class(kinds), 0, m);
}

hipError_t launch_weight(const ChannelTab* ct, const ProcessTab* pt, int mixed, int np, int64_t n, const double* p,
                         const double* x1x2, const double* jac, double* w, double* alpha, hipStream_t s) {
    if (n == 0) return hipSuccess;
    int64_t g = (n + kBlock - 1) / kBlock;
    if (mixed)
        k_weight<true><<<dim3((unsigned)g), dim3(kBlock), 0, s>>>(ct, pt, np, n, p, x1x2, jac, w, alpha);
    else
        k_weight<false><<<dim3((unsigned)g), dim3(kBlock), 0, s>>>(ct, pt, np, n, p, x1x2, jac, w, alpha);
    return hipGetLastError();
}

hipError_t launch_sample(const ChannelTab* cts, const ProcessTab* pts, const double* grids, const int64_t* grid_off,
                         const int32_t* chan_nb, const SampleCall* call, int n_chan, int max_slots, int max_inv,
                         int kinds, int mixed, size_t lds_bytes, uint64_t seed, uint64_t sid, const uint64_t* ctr_dev,
                         uint64_t ctr_off, int np, int64_t ld, double* p, double* x1x2, double* w, int32_t* chan,
                         double* tile_stats, double* stats, int grid, hipStream_t s, double* vpart, int vstride,
                         const int64_t* hist_off, int64_t hist_total, double* hist, const JitSampleSet* jit) {
    if (jit && jit->n > 0) {
        int grid_doubles = (int)(lds_bytes / sizeof(double));
        void* args[] = {&cts, &pts, &grids, &grid_off, &chan_nb, &call, &seed, &sid, &ctr_dev, &ctr_off, &np, &ld,
                        &p, &x1x2, &w, &chan, &tile_stats, &grid_doubles, &vpart, &vstride};
        for (int g = 0; g < jit->n; ++g) {
            const size_t lds =
                lds_bytes + sizeof(double) * (size_t)jit->k[g].rows * kBlock + (vpart ? vegas_acc_lds(vstride) : 0);
            hipError_t err = hipModuleLaunchKernel(jit->k[g].fn, (unsigned)std::max(grid, 1), 1, 1, kBlock, 1, 1,
                                                   (unsigned)lds, s, args, nullptr);
            if (err != hipSuccess) return err;
        }
    } else {
        ChainLaunch a{};
        a.sample = true;
        a.lds = lds_bytes;
        a.grid = std::max(grid, 1);
        a.stream = s;
        a.cts = cts;
        a.pts = pts;
        a.grids = grids;
        a.grid_off = grid_off;
        a.chan_nb = chan_nb;
        a.call = call;
        a.seed = seed;
        a.sid = sid;
        a.ctr_dev = ctr_dev;
        a.ctr_off = ctr_off;
        a.np = np;
        a.n = ld;
        a.p = p;
        a.x1x2 = x1x2;
        a.w = w;
        a.chan = chan;
        a.tile_stats = tile_stats;
        a.vpart = vpart;
        a.vstride = vstride;
        hipError_t err = launch_chain(reg_class(max_slots, max_inv), kind_class(kinds), mixed, a);
        if (err != hipSuccess) return err;
    }
    k_stats_final<<<n_chan, kBlock, 0, s>>>(call, tile_stats, stats);
    if (vpart && hist_total > 0) {
        const int64_t g = (hist_total + kBlock - 1) / kBlock;
        k_vegas_tiles<<<dim3((unsigned)g), dim3(kBlock), 0, s>>>(call, hist_off, hist_total, vstride, vpart, hist);
    }
    return hipGetLastError();
}

namespace {
// rows of the sample kernel's per-thread staging column (stage_rows of the
// chain kernels)
int stage_rows_host(int ns, int ni) { return (ns + ni + 1) > kQRows ? (ns + ni + 1) : kQRows; }
}  // namespace

size_t sample_lds_bytes(int max_slots, int max_inv, size_t lds_bytes, int vstride) {
    const int rc = reg_class(max_slots, max_inv);
    const int rows = rc == 0 ? stage_rows_host(6, 4) : (rc == 1 ? stage_rows_host(10, 8) : stage_rows_host(14, 8));
    return lds_bytes + sizeof(double) * (size_t)rows * kBlock + (vstride > 0 ? vegas_acc_lds(vstride) : 0);
}

hipError_t launch_set_call(const SampleCall& host, SampleCall* dev, hipStream_t s) {
    k_set_call<<<1, 64, 0, s>>>(host, dev);
    return hipGetLastError();
}

hipError_t launch_plan(const int64_t* counts, int n_chan, int64_t capacity, int ept, SampleCall* dev,
                       int32_t* status, hipStream_t s) {
    k_plan<<<1, 64, 0, s>>>(counts, n_chan, capacity, ept, dev, status);
    return hipGetLastError();
}

int sample_block() { return kBlock; }

// ---------------------------------------------------------------------------
// Fixed device scratch of the allocation-free sample entry point: the tile
// statistics of one launch (4 doubles per tile).  Each GPU that runs the
// library holds one copy for the life of the process; its device address is
// looked up once per device (hipGetSymbolAddress) and used from then on --
// the array's name in host code is only a host-side stand-in.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[4 * kNoAllocTiles];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};
}  // namespace

hipError_t noalloc_scratch(int device, double** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = ptr;
    }
    *out = (double*)g_scratch_ptr[device];
    return hipSuccess;
}

hipError_t launch_vegas_accumulate(int64_t n, int dims, int nb, const double* y, const double* w, double* part,
                                   int64_t nchunk, int64_t chunk, double* hist, hipStream_t s) {
    if (n == 0) return hipSuccess;
    // one private LDS row per thread, 64 KiB at most
    int threads = nb <= 64 ? 128 : 64;
    size_t lds = sizeof(double) * threads * (size_t)nb;
    k_vegas_partial<<<dim3((unsigned)nchunk, (unsigned)dims), dim3(threads), lds, s>>>(n, nb, y, w, chunk, part);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    int tot = dims * nb;
    k_vegas_reduce<<<(tot + 127) / 128, 128, 0, s>>>(dims, nb, nchunk, part, hist);
    return hipGetLastError();
}

hipError_t launch_vegas_refine(int n_rows, const int32_t* row_nb, const int64_t* row_grid, const int64_t* row_hist,
                               double alpha, double* grids, double* hist, hipStream_t s) {
    if (n_rows == 0) return hipSuccess;
    k_vegas_refine<<<(n_rows + 63) / 64, 64, 0, s>>>(n_rows, row_nb, row_grid, row_hist, alpha, grids, hist);
    return hipGetLastError();
}

}  // namespace msx

// ---------------------------------------------------------------------------
// Unweighting efficiency: bucket histograms over the IEEE bit pattern, which
// orders non-negative doubles like their values.
// ---------------------------------------------------------------------------
namespace msx {
namespace {

constexpr int kUnwBuckets = 4096;
static_assert(kUnwBuckets == kUnwMaxBuckets, "bucket count");

// Counts and sums of the weights per bucket, with integer atomics only, so
// the result does not depend on the order of the additions: every weight of
// a bucket has the bucket's binary exponent (the buckets of every pass lie
// within one exponent), so its value is m 2^(e - 1075) with the integer
// significand m < 2^53, and the bucket sum is kept exactly as the sums of
// m's upper 27 and lower 26 bits (each < 2^63 for n < 2^36 weights).
__global__ __launch_bounds__(256) void k_unw_hist(int64_t n, const double* __restrict__ w, int shift, int width,
                                                  const UnwState* __restrict__ st, int first,
                                                  unsigned long long* __restrict__ counts,
                                                  unsigned long long* __restrict__ sum_hi,
                                                  unsigned long long* __restrict__ sum_lo) {
    const uint64_t prefix = st->prefix;
    __shared__ unsigned int c_l[kUnwBuckets];
    __shared__ unsigned long long h_l[kUnwBuckets];
    __shared__ unsigned long long l_l[kUnwBuckets];
    const int nbk = 1 << width;
    for (int i = threadIdx.x; i < nbk; i += blockDim.x) {
        c_l[i] = 0u;
        h_l[i] = 0ull;
        l_l[i] = 0ull;
    }
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        double v = w[e];
        if (!(v > 0.0)) continue;  // zero weights carry no excess
        uint64_t bits = (uint64_t)__double_as_longlong(v);
        if (!first && (bits >> (shift + width)) != prefix) continue;
        int b = (int)((bits >> shift) & (uint64_t)(nbk - 1));
        const uint64_t ex = bits >> 52;
        const uint64_t m = (bits & ((1ull << 52) - 1)) | (ex ? (1ull << 52) : 0ull);
        atomicAdd(&c_l[b], 1u);
        atomicAdd(&h_l[b], (unsigned long long)(m >> 26));
        atomicAdd(&l_l[b], (unsigned long long)(m & ((1ull << 26) - 1)));
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nbk; i += blockDim.x) {
        if (c_l[i]) {
            atomicAdd(&counts[i], (unsigned long long)c_l[i]);
            atomicAdd(&sum_hi[i], h_l[i]);
            atomicAdd(&sum_lo[i], l_l[i]);
        }
    }
}

// The crossing bucket of one pass: the workgroup converts the bucket sums
// and counts into LDS, then one thread scans from the top bucket down (the
// order and arithmetic of a sequential scan): the excess at the lower edge
// L_b of bucket b, S - L_b N over the weights in buckets >= b and above the
// earlier passes' crossing buckets, reaches the target first at the crossing
// bucket; st gets the extended prefix and the sums above it.  The bucket
// arrays are cleared for the next pass.
__global__ __launch_bounds__(256) void k_unw_search(int shift, int width, double overweight,
                                                    const double* __restrict__ tot, UnwState* __restrict__ st,
                                                    unsigned long long* __restrict__ counts,
                                                    unsigned long long* __restrict__ sum_hi,
                                                    unsigned long long* __restrict__ sum_lo) {
    __shared__ double s_b[kUnwBuckets];
    __shared__ double n_b[kUnwBuckets];
    const int nbk = 1 << width;
    const uint64_t prefix = st->prefix;
    // every bucket's sum (its significand sum times 2^(e - 1075), e its
    // biased exponent; 1 - 1075 for subnormals) and count, in parallel
    for (int b = threadIdx.x; b < nbk; b += blockDim.x) {
        const uint64_t lb_bits = ((prefix << width) | (uint64_t)b) << shift;
        const int ex = (int)(lb_bits >> 52);
        s_b[b] = ldexp((double)sum_hi[b] * 67108864.0 + (double)sum_lo[b], (ex ? ex : 1) - 1075);
        n_b[b] = (double)counts[b];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double target = overweight * tot[0];
        double S = st->S_up, N = st->N_up;
        double S_above = S, N_above = N;
        int found = -1;
        // eight buckets per step, their LDS reads issued before the
        // sequential additions (the scan is otherwise bound by LDS latency)
        for (int b0 = nbk - 1; b0 >= 0 && found < 0; b0 -= 8) {
            double sv[8], nv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                sv[u] = b0 - u >= 0 ? s_b[b0 - u] : 0.0;
                nv[u] = b0 - u >= 0 ? n_b[b0 - u] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int b = b0 - u;
                if (b < 0 || found >= 0) break;
                S_above = S;
                N_above = N;
                S += sv[u];
                N += nv[u];
                const uint64_t lb_bits = ((prefix << width) | (uint64_t)b) << shift;
                if (S - __longlong_as_double((long long)lb_bits) * N >= target) found = b;
            }
        }
        if (found < 0) found = 0;  // only the zero bucket: W lies below every positive weight
        st->S_up = S_above;
        st->N_up = N_above;
        st->prefix = (prefix << width) | (uint64_t)found;
    }
    for (int i = threadIdx.x; i < kUnwBuckets; i += blockDim.x) {
        counts[i] = 0ull;
        sum_hi[i] = 0ull;
        sum_lo[i] = 0ull;
    }
}

__global__ __launch_bounds__(256) void k_sum_max(int64_t n, const double* __restrict__ w, double* __restrict__ part) {
    double s = 0.0, m = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        double v = w[e];
        s += v;
        m = fmax(m, v);
    }
    __shared__ double rs[4], rm[4];
    double ws = wave_sum(s), wm = wave_max(m);
    if ((threadIdx.x & 63) == 0) {
        rs[threadIdx.x >> 6] = ws;
        rm[threadIdx.x >> 6] = wm;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = rs[0], b = rm[0];
        for (int i = 1; i < 4; ++i) {
            a += rs[i];
            b = fmax(b, rm[i]);
        }
        part[2 * blockIdx.x] = a;
        part[2 * blockIdx.x + 1] = b;
    }
}

__global__ void k_sum_max_final(int nblk, const double* __restrict__ part, double* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double a = 0.0, b = 0.0;
    for (int i = 0; i < nblk; ++i) {
        a += part[2 * i];
        b = fmax(b, part[2 * i + 1]);
    }
    out[0] = a;
    out[1] = b;
}

// Moments of a weight array: block b reduces its grid-stride share into
// part[b] = (sum w, sum w^2, n(w == 0), max w); the final pass sums blocks in
// order and adds to out = (sum w, sum w^2, n, n(w == 0), max w).
constexpr int kMomBlocks = 256;
__global__ __launch_bounds__(256) void k_moments(int64_t n, const double* __restrict__ w, double* __restrict__ part) {
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        const double v = w[e];
        a[0] += v;
        a[1] += v * v;
        a[2] += v == 0.0 ? 1.0 : 0.0;
        a[3] = fmax(a[3], v);
    }
    __shared__ double r[4][4];
    const double r0 = wave_sum(a[0]), r1 = wave_sum(a[1]), r2 = wave_sum(a[2]), r3 = wave_max(a[3]);
    if ((threadIdx.x & 63) == 0) {
        r[0][threadIdx.x >> 6] = r0;
        r[1][threadIdx.x >> 6] = r1;
        r[2][threadIdx.x >> 6] = r2;
        r[3][threadIdx.x >> 6] = r3;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const int q = threadIdx.x;
        double acc = r[q][0];
        for (int v = 1; v < 4; ++v) acc = q == 3 ? fmax(acc, r[q][v]) : acc + r[q][v];
        part[4 * blockIdx.x + q] = acc;
    }
}

__global__ void k_moments_final(int nblk, int64_t n, const double* __restrict__ part, double* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double a = 0.0, b = 0.0, z = 0.0, m = 0.0;
    for (int i = 0; i < nblk; ++i) {
        a += part[4 * i];
        b += part[4 * i + 1];
        z += part[4 * i + 2];
        m = fmax(m, part[4 * i + 3]);
    }
    out[0] += a;
    out[1] += b;
    out[2] += (double)n;
    out[3] += z;
    out[4] = fmax(out[4], m);
}

__global__ void k_advance_counter(const SampleCall* __restrict__ call, uint64_t* __restrict__ ctr) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *ctr += (uint64_t)call->ev_start[call->n_chan];
}

__global__ void k_fill_i32(int32_t* __restrict__ x, int64_t n, int32_t v) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) x[i] = v;
}

}  // namespace

int64_t moments_blocks() { return kMomBlocks; }

hipError_t launch_moments_add(const double* w, int64_t n, double* part, double* out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int g = (int)std::min<int64_t>(kMomBlocks, (n + 255) / 256);
    k_moments<<<g, 256, 0, s>>>(n, w, part);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    k_moments_final<<<1, 64, 0, s>>>(g, n, part, out);
    return hipGetLastError();
}

hipError_t launch_advance_counter(const SampleCall* call, uint64_t* ctr, hipStream_t s) {
    k_advance_counter<<<1, 64, 0, s>>>(call, ctr);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* x, int64_t n, int32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int g = (int)std::min<int64_t>(4096, (n + 255) / 256);
    k_fill_i32<<<g, 256, 0, s>>>(x, n, v);
    return hipGetLastError();
}

hipError_t launch_unw_search(int64_t n, const double* w, double overweight, const double* tot, UnwState* st,
                             uint64_t* counts, uint64_t* sum_hi, uint64_t* sum_lo, int cu_count, hipStream_t s) {
    // passes over the 63 value bits of non-negative doubles: buckets of 12
    // bits, the last pass 3
    const int shifts[6] = {51, 39, 27, 15, 3, 0};
    const int widths[6] = {12, 12, 12, 12, 12, 3};
    const int g = grid_for(n, cu_count * 4);
    for (int pass = 0; pass < 6; ++pass) {
        k_unw_hist<<<g, 256, 0, s>>>(n, w, shifts[pass], widths[pass], st, pass == 0, (unsigned long long*)counts,
                                     (unsigned long long*)sum_hi, (unsigned long long*)sum_lo);
        k_unw_search<<<1, 256, 0, s>>>(shifts[pass], widths[pass], overweight, tot, st, (unsigned long long*)counts,
                                       (unsigned long long*)sum_hi, (unsigned long long*)sum_lo);
    }
    return hipGetLastError();
}

hipError_t launch_sum_max(int64_t n, const double* w, double* out, double* part, int nblk, hipStream_t s) {
    k_sum_max<<<nblk, 256, 0, s>>>(n, w, part);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    k_sum_max_final<<<1, 64, 0, s>>>(nblk, part, out);
    return hipGetLastError();
}

}  // namespace msx
