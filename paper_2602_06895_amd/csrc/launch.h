// Host-side launchers of the gfx950 kernels (defined in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tables.h"

namespace msx {

// Arguments of one mapping-chain launch (single-channel map or fused sample).
struct ChainLaunch {
    bool sample;
    bool inverse;  // k_inverse: p_in, x1x2_in -> y_out, jac (FP64 units only)
    size_t lds;
    int grid;
    hipStream_t stream;
    const ChannelTab* cts;
    const ProcessTab* pts;
    const double* grids;
    // map
    int nb;
    double s_lab;
    const double* y;
    double* jac;
    // sample
    const int64_t* grid_off;
    const int32_t* chan_nb;
    const SampleCall* call;  // device memory
    uint64_t seed, sid, ctr_off;
    const uint64_t* ctr_dev;  // device counter offset (overrides ctr_off) or NULL
    int32_t* chan;
    double* tile_stats;
    double* vpart;  // per-tile VEGAS histograms [tiles][vstride], NULL: no accumulation
    int vstride;
    // both
    int np;
    int64_t n;  // map: events; sample: row stride of the outputs
    double* p;
    double* x1x2;
    double* w;
    // inverse
    const double* p_in;
    const double* x1x2_in;
    double* y_out;
};

// One register class (NS slots, NI invariants) at one precision; defined in
// the chain_*.hip instantiation units.
template <int NS, int NI, bool MIX>
hipError_t launch_chain_class(int kind_class, const ChainLaunch& a);
// The inverse map of one register class (FP64); the inverse_*.hip units.
template <int NS, int NI>
hipError_t launch_inverse_class(int kind_class, const ChainLaunch& a);

hipError_t launch_uniform(uint64_t seed, uint64_t sid, uint64_t e0, int64_t n, int d, double* y, hipStream_t s);

hipError_t launch_map(const ChannelTab* ct, const ProcessTab* pt, const double* grid, int nb, int dims, int n_slots,
                      int n_inv, int kinds, int mixed, double s_lab, int np, int64_t n, const double* y, double* p,
                      double* x1x2, double* jac, double* w, int cu_count, hipStream_t s);

hipError_t launch_inverse(const ChannelTab* ct, const double* grid, int nb, int dims, int n_slots, int n_inv, int kinds,
                          double s_lab, int np, int64_t n, const double* p, const double* x1x2, double* y, double* jac,
                          int cu_count, hipStream_t s);

// Observables of lab-frame events: spec = k x (kind, set, rank, 0) int32;
// out [k][n].  k <= 8.
hipError_t launch_observables(const double* p, int np, int64_t n, const int32_t* spec, int k, double* out,
                              hipStream_t s);
// w[e] = 0 unless lo[j] <= x[j][e] < hi[j] for all j < k (k <= 8).
hipError_t launch_cut(const double* x, int k, int64_t n, const double* lo, const double* hi, double* w, hipStream_t s);
// Weighted histogram of x: out [2][nb] = (sum w, sum w^2) per bin of [lo, hi);
// part: scratch of histogram_blocks(n) x 2 nb doubles.
int64_t histogram_blocks(int64_t n);
hipError_t launch_histogram(const double* x, const double* w, int64_t n, int nb, double lo, double hi, double* part,
                            double* out, hipStream_t s);

// Hit-or-miss unweighting: kept indices (increasing) to keep, unit weights
// max(1, w / w_max) to uw (optional), the number kept to count (device);
// blk: scratch of unweight_blocks(n) (at least 1) int64.
int64_t unweight_blocks(int64_t n);
hipError_t launch_unweight(const double* w, int64_t n, double w_max, uint64_t seed, uint64_t sid, uint64_t e0,
                           int64_t* blk, int64_t* keep, double* uw, int64_t* count, hipStream_t s);

// g = alpha / jac (first) or g += alpha / jac; jac = 0 adds nothing.
hipError_t launch_density_add(double* g, const double* jac, double alpha, int64_t n, bool first, hipStream_t s);

hipError_t launch_weight(const ChannelTab* ct, const ProcessTab* pt, int mixed, int np, int64_t n, const double* p,
                         const double* x1x2, const double* jac, double* w, double* alpha, hipStream_t s);

// A fused-sample kernel compiled at run time for one context's channels,
// with their channel and process tables as compile-time constants (jit.cpp);
// it takes k_sample's arguments.  rows: height of its LDS staging column.
struct JitSample {
    hipModule_t module = nullptr;
    hipFunction_t fn = nullptr;
    int rows = 0;
    int waves = 0;    // waves per SIMD it was compiled for (0: the compiler's choice)
    int scratch = 0;  // its scratch bytes per lane
    int c0 = 0, c1 = 0;  // the channels it samples
};
// The kernels compiled for a context: consecutive channel groups, launched
// one after the other (each runs only its channels' tiles).
constexpr int kMaxJitGroups = kMaxChannels;
struct JitSampleSet {
    int n = 0;
    JitSample k[kMaxJitGroups];
};

// Fused multichannel sample.  `call` is the device copy of the call table;
// `max_tiles` bounds its n_tiles (for the per-channel statistics pass);
// `ld` is the row stride of the outputs (>= the events of the call).
// With vpart != NULL the kernel also accumulates every channel's VEGAS
// histogram (sum w^2 per bin of every dimension) into per-tile partials
// vpart [tiles][vstride] (vstride >= dims x bins of every channel), and a
// second kernel adds them, tiles in order, to hist at hist_off[c] (device
// array, per channel).  With jit != NULL (and jit->n > 0) the launch runs
// those kernels instead of the register / kind class kernel of
// (max_slots, max_inv, kinds).
hipError_t launch_sample(const ChannelTab* cts, const ProcessTab* pts, const double* grids, const int64_t* grid_off,
                         const int32_t* chan_nb, const SampleCall* call, int n_chan, int max_slots, int max_inv,
                         int kinds, int mixed, size_t lds_bytes, uint64_t seed, uint64_t sid, const uint64_t* ctr_dev,
                         uint64_t ctr_off, int np, int64_t ld, double* p, double* x1x2, double* w, int32_t* chan,
                         double* tile_stats, double* stats, int grid, hipStream_t s, double* vpart = nullptr,
                         int vstride = 0, const int64_t* hist_off = nullptr, int64_t hist_total = 0,
                         double* hist = nullptr, const JitSampleSet* jit = nullptr);
// Dynamic LDS bytes of a sample launch with VEGAS accumulation (grid area
// lds_bytes, vstride doubles per wave histogram) for the register class of
// (max_slots, max_inv).
size_t sample_lds_bytes(int max_slots, int max_inv, size_t lds_bytes, int vstride);

// Device copy of a host-built call table (stream ordered).
hipError_t launch_set_call(const SampleCall& host, SampleCall* dev, hipStream_t s);

// Call table from device-resident counts: prefix sums over n_chan channels,
// tiles of kBlock * ept events.  If a count is negative or the total exceeds
// `capacity`, n_tiles = 0 and *status = 1 (else 0).
hipError_t launch_plan(const int64_t* counts, int n_chan, int64_t capacity, int ept, SampleCall* dev,
                       int32_t* status, hipStream_t s);

int sample_block();  // threads per workgroup of the sample kernel

// Adds the moments (sum w, sum w^2, n, n(w == 0), max w) of w [n] to out[5]
// (device; the first four summed, the last a maximum); part: scratch of
// 4 moments_blocks() doubles.  Deterministic.
int64_t moments_blocks();
hipError_t launch_moments_add(const double* w, int64_t n, double* part, double* out, hipStream_t s);
hipError_t launch_fill_i32(int32_t* x, int64_t n, int32_t v, hipStream_t s);
// *ctr += the events of the call table (device-count launches that advance
// their counter offset).
hipError_t launch_advance_counter(const SampleCall* call, uint64_t* ctr, hipStream_t s);

// The allocation-free sample entry point's fixed device scratch: room for the
// tile statistics of kNoAllocTiles tiles, one copy per GPU (devices
// 0 .. kMaxScratchDevices - 1).  *out = its device address on `device`, looked
// up on the first call for that device and kept.
constexpr int64_t kNoAllocTiles = 1 << 17;
constexpr int kMaxScratchDevices = 64;
hipError_t noalloc_scratch(int device, double** out);

hipError_t launch_vegas_accumulate(int64_t n, int dims, int nb, const double* y, const double* w, double* part,
                                   int64_t nchunk, int64_t chunk, double* hist, hipStream_t s);

hipError_t launch_vegas_refine(int n_rows, const int32_t* row_nb, const int64_t* row_grid, const int64_t* row_hist,
                               double alpha, double* grids, double* hist, hipStream_t s);

}  // namespace msx

namespace msx {

// Unweighting-efficiency search (the largest weight W whose excess
// sum_i max(0, w_i - W) reaches overweight x the total tot[0]), refined over
// the bit patterns of the weights, which order non-negative doubles like
// their values: six passes, each a histogram over bucket = (bits >> shift) &
// (2^width - 1) of the positive weights whose higher bits equal the prefix
// found so far (counts, and the bucket's significand sum as the sums of
// m >> 26 and m & (2^26 - 1), the weight being m 2^(e - 1075); integer
// atomics only), then a one-thread scan for the crossing bucket.  On return
// (stream order) st holds the crossing value's bit pattern in prefix and the
// sums above it.  st must start at zero, the bucket arrays (kUnwMaxBuckets
// words each) too; they are zero again afterwards.  No host round trip.
constexpr int kUnwMaxBuckets = 4096;
struct UnwState {
    uint64_t prefix;
    double S_up, N_up;
};
hipError_t launch_unw_search(int64_t n, const double* w, double overweight, const double* tot, UnwState* st,
                             uint64_t* counts, uint64_t* sum_hi, uint64_t* sum_lo, int cu_count, hipStream_t s);
// total sum and max of w (two doubles at out)
hipError_t launch_sum_max(int64_t n, const double* w, double* out, double* part, int nblk, hipStream_t s);

}  // namespace msx
