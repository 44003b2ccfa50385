// gfx950 kernels of the phase-space hot path and their host launchers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "chain.h"
#include "launch.h"

namespace msx {

namespace {

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

// Beam boost, unphysical cut, integrand x channel weight and the stores of one
// event whose partonic-frame momenta sit in the slots.
template <int NS>
__device__ __forceinline__ double finish_event(const ChannelTab* __restrict__ ct, const ProcessTab* __restrict__ pt,
                                               const ChainOut& o, double jv, double (&E)[NS], double (&X)[NS],
                                               double (&Y)[NS], double (&Z)[NS], int np, int64_t n, int64_t e,
                                               double* __restrict__ p, double* __restrict__ x1x2,
                                               double* __restrict__ jac_out, bool want_w) {
    const int nf = ct->n_final;
    const int hadronic = ct->hadronic;
    double g = 1.0, gb = 0.0;
    if (hadronic) {
        double inv = 1.0 / (2.0 * sqrt(o.x1 * o.x2));
        g = (o.x1 + o.x2) * inv;
        gb = (o.x1 - o.x2) * inv;
    }
    const double h = 0.5 * sqrt(o.shat);
    bool ok = true;
    // incoming partons, then final-state particles by label
    for (int i = 0; i < nf + 2; ++i) {
        double pe, px, py, pz;
        if (i < 2) {
            pe = h;
            px = 0.0;
            py = 0.0;
            pz = i == 0 ? h : -h;
        } else {
            int s = slot_index<NS>(ct->final_slot[i - 2]);
            pe = E[s];
            px = X[s];
            py = Y[s];
            pz = Z[s];
        }
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
    }
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
            int s = slot_index<NS>(ct->final_slot[k]);
            return c == 0 ? E[s] : (c == 1 ? X[s] : (c == 2 ? Y[s] : Z[s]));
        };
        double af = integrand_alpha(pt, ct->alpha_index, o.x1, o.x2, o.logtau, h, 0.0, 0.0, h, get, alpha);
        w = af * jac;
    }
    return w;
}

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

template <int NS, int NI, int KINDS>
__global__ __launch_bounds__(kBlock) void k_map(const ChannelTab* __restrict__ ct, const ProcessTab* __restrict__ pt,
                                                const double* __restrict__ grid, int nb, double s_lab, int np,
                                                int64_t n, const double* __restrict__ y, double* __restrict__ p,
                                                double* __restrict__ x1x2, double* __restrict__ jac,
                                                double* __restrict__ w) {
    extern __shared__ double lg[];
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
        run_chain<NS, NI, KINDS>(ct, s_lab, next, E, X, Y, Z, S, SQ, o);
        double wv = finish_event<NS>(ct, pt, o, jv, E, X, Y, Z, np, n, e, p, x1x2, jac, w != nullptr);
        if (w) w[e] = wv;
    }
}

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
            L = log(x1 * x2);
        }
        auto get = [&](int k, int c) -> double { return p[((int64_t)c * np + k + 2) * n + e]; };
        double pae = p[((int64_t)0 * np) * n + e], pax = p[((int64_t)1 * np) * n + e];
        double pay = p[((int64_t)2 * np) * n + e], paz = p[((int64_t)3 * np) * n + e];
        double af = integrand_alpha(pt, ct->alpha_index, x1, x2, L, pae, pax, pay, paz, get, av);
        wv = af * j;
    }
    w[e] = wv;
    if (alpha) alpha[e] = av;
}

// All channels in one persistent launch.  Tiles of kBlock events never mix
// channels; block b takes tiles b, b + gridDim, ... (static, so per-tile
// statistics are reproducible).  Each tile writes (sum w, sum w^2, n(w == 0),
// max w) to tile_stats.
template <int NS, int NI, int KINDS>
__global__ __launch_bounds__(kBlock) void k_sample(const ChannelTab* __restrict__ cts, const ProcessTab* __restrict__ pts,
                                                   const double* __restrict__ grids, const int64_t* __restrict__ grid_off,
                                                   const int32_t* __restrict__ chan_nb, SampleCall call, uint64_t seed,
                                                   uint64_t sid, uint64_t ctr_off, double s_lab_unused, int np,
                                                   int64_t N, double* __restrict__ p, double* __restrict__ x1x2,
                                                   double* __restrict__ w, int32_t* __restrict__ chan_out,
                                                   double* __restrict__ tile_stats) {
    extern __shared__ double lg[];
    __shared__ double red[4][kWaves];
    int cur = -1;
    int nb = 0, dims = 0;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int64_t tile = blockIdx.x; tile < call.n_tiles; tile += gridDim.x) {
        int c = 0;
        while (c + 1 < call.n_chan && call.tile_start[c + 1] <= tile) ++c;
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
        const int64_t pos = call.ev_start[c] + (tile - call.tile_start[c]) * kBlock + threadIdx.x;
        const bool active = pos < call.ev_start[c + 1];
        double wv = 0.0;
        if (active) {
            const uint64_t e = ctr_off + (uint64_t)pos;
            // uniforms on demand, four per Philox block (dimensions are consumed in order)
            double ub[4];
            int k = 0;
            double jv = 1.0;
            auto next = [&]() -> double {
                if ((k & 3) == 0) {
                    uint64_t c0 = e, c1 = (uint64_t)(k >> 2), c2 = 0, c3 = 0;
                    philox4x64_10(c0, c1, c2, c3, seed, sid);
                    ub[0] = to_unit(c0);
                    ub[1] = to_unit(c1);
                    ub[2] = to_unit(c2);
                    ub[3] = to_unit(c3);
                }
                double r = vegas_map(ub[k & 3], lg + k * (nb + 1), nb, jv);
                ++k;
                return r;
            };
            double E[NS], X[NS], Y[NS], Z[NS], S[NI], SQ[NI];
            ChainOut o;
            run_chain<NS, NI, KINDS>(ct, s_lab, next, E, X, Y, Z, S, SQ, o);
            wv = finish_event<NS>(ct, pt, o, jv, E, X, Y, Z, np, N, pos, p, x1x2, nullptr, true);
            w[pos] = wv;
            if (chan_out) chan_out[pos] = c;
        }
        double s1 = wave_sum(wv), s2 = wave_sum(wv * wv);
        double nz = wave_sum((active && wv == 0.0) ? 1.0 : 0.0);
        double mx = wave_max(active ? wv : 0.0);
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

// Reduce the tiles of each channel in order and add to the accumulators
// stats[c] = (sum w, sum w^2, n, n(w == 0), max w).
__global__ __launch_bounds__(kBlock) void k_stats_final(SampleCall call, const double* __restrict__ tile_stats,
                                                        double* __restrict__ stats) {
    const int c = blockIdx.x;
    __shared__ double red[4][kWaves];
    const int64_t t0 = call.tile_start[c], t1 = call.tile_start[c + 1];
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
        st[2] += (double)(call.ev_start[c + 1] - call.ev_start[c]);
        st[3] += s2;
        st[4] = fmax(st[4], mx);
    }
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
// Breit-Wigner, 2 everything.
int kind_class(int kinds) {
    if ((kinds & ~KIND_POW_INT) == 0) return 0;
    if ((kinds & ~(KIND_POW_INT | KIND_BW)) == 0) return 1;
    return 2;
}

// One launch per (register class, kind class) instantiation.
#define MSX_DISPATCH(RC, KC, LAUNCH)                                       \
    do {                                                                   \
        constexpr int K0 = KIND_POW_INT, K1 = KIND_POW_INT | KIND_BW, K2 = KINDS_ALL; \
        const int rc_ = (RC), kc_ = (KC);                                  \
        if (rc_ == 0) {                                                    \
            if (kc_ == 0) LAUNCH(6, 4, K0);                                \
            else if (kc_ == 1) LAUNCH(6, 4, K1);                           \
            else LAUNCH(6, 4, K2);                                         \
        } else if (rc_ == 1) {                                             \
            if (kc_ == 0) LAUNCH(10, 8, K0);                               \
            else if (kc_ == 1) LAUNCH(10, 8, K1);                          \
            else LAUNCH(10, 8, K2);                                        \
        } else {                                                           \
            if (kc_ == 0) LAUNCH(14, 8, K0);                               \
            else if (kc_ == 1) LAUNCH(14, 8, K1);                          \
            else LAUNCH(14, 8, K2);                                        \
        }                                                                  \
    } while (0)

int grid_for(int64_t n, int cap) {
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g > cap) g = cap;
    return (int)std::max<int64_t>(g, 1);
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

hipError_t launch_uniform(uint64_t seed, uint64_t sid, uint64_t e0, int64_t n, int d, double* y, hipStream_t s) {
    if (n == 0) return hipSuccess;
    int64_t g = (n + kBlock - 1) / kBlock;
    k_uniform<<<dim3((unsigned)g), dim3(kBlock), 0, s>>>(seed, sid, e0, n, d, y);
    return hipGetLastError();
}

hipError_t launch_map(const ChannelTab* ct, const ProcessTab* pt, const double* grid, int nb, int dims, int n_slots,
                      int n_inv, int kinds, double s_lab, int np, int64_t n, const double* y, double* p,
                      double* x1x2, double* jac, double* w, int cu_count, hipStream_t s) {
    if (n == 0) return hipSuccess;
    size_t lds = sizeof(double) * (size_t)dims * (nb + 1);
    int g = grid_for(n, cu_count * 8);
#define MSX_MAP(NS, NI, K) k_map<NS, NI, K><<<g, kBlock, lds, s>>>(ct, pt, grid, nb, s_lab, np, n, y, p, x1x2, jac, w)
    MSX_DISPATCH(reg_class(n_slots, n_inv), kind_class(kinds), MSX_MAP);
#undef MSX_MAP
    return hipGetLastError();
}

hipError_t launch_weight(const ChannelTab* ct, const ProcessTab* pt, int np, int64_t n, const double* p,
                         const double* x1x2, const double* jac, double* w, double* alpha, hipStream_t s) {
    if (n == 0) return hipSuccess;
    int64_t g = (n + kBlock - 1) / kBlock;
    k_weight<<<dim3((unsigned)g), dim3(kBlock), 0, s>>>(ct, pt, np, n, p, x1x2, jac, w, alpha);
    return hipGetLastError();
}

hipError_t launch_sample(const ChannelTab* cts, const ProcessTab* pts, const double* grids, const int64_t* grid_off,
                         const int32_t* chan_nb, const SampleCall& call, int max_slots, int max_inv, int kinds,
                         size_t lds_bytes,
                         uint64_t seed, uint64_t sid, uint64_t ctr_off, int np, int64_t N, double* p, double* x1x2,
                         double* w, int32_t* chan, double* tile_stats, double* stats, int grid, hipStream_t s) {
    if (call.n_tiles == 0) return hipSuccess;
    int g = (int)std::min<int64_t>(call.n_tiles, grid);
#define MSX_SAMPLE(NS, NI, K)                                                                                \
    k_sample<NS, NI, K><<<g, kBlock, lds_bytes, s>>>(cts, pts, grids, grid_off, chan_nb, call, seed, sid, ctr_off, \
                                                     0.0, np, N, p, x1x2, w, chan, tile_stats)
    MSX_DISPATCH(reg_class(max_slots, max_inv), kind_class(kinds), MSX_SAMPLE);
#undef MSX_SAMPLE
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    k_stats_final<<<call.n_chan, kBlock, 0, s>>>(call, tile_stats, stats);
    return hipGetLastError();
}

int sample_tile_size() { return kBlock; }

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

__global__ __launch_bounds__(256) void k_unw_hist(int64_t n, const double* __restrict__ w, int shift, int width,
                                                  uint64_t prefix, int first, double* __restrict__ counts,
                                                  double* __restrict__ sums) {
    __shared__ unsigned int c_l[kUnwBuckets];
    __shared__ double s_l[kUnwBuckets];
    const int nbk = 1 << width;
    for (int i = threadIdx.x; i < nbk; i += blockDim.x) {
        c_l[i] = 0u;
        s_l[i] = 0.0;
    }
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        double v = w[e];
        if (!(v > 0.0)) continue;  // zero weights carry no excess
        uint64_t bits = (uint64_t)__double_as_longlong(v);
        if (!first && (bits >> (shift + width)) != prefix) continue;
        int b = (int)((bits >> shift) & (uint64_t)(nbk - 1));
        atomicAdd(&c_l[b], 1u);
        atomicAdd(&s_l[b], v);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nbk; i += blockDim.x) {
        if (c_l[i]) {
            atomicAdd(&counts[i], (double)c_l[i]);
            atomicAdd(&sums[i], s_l[i]);
        }
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

}  // namespace

hipError_t launch_unw_pass(int64_t n, const double* w, int shift, int width, uint64_t prefix, int first,
                           double* counts, double* sums, int cu_count, hipStream_t s) {
    int g = grid_for(n, cu_count * 4);
    k_unw_hist<<<g, 256, 0, s>>>(n, w, shift, width, prefix, first, counts, sums);
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
