// Host-side launchers of the gfx950 kernels (defined in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tables.h"

namespace msx {

hipError_t launch_uniform(uint64_t seed, uint64_t sid, uint64_t e0, int64_t n, int d, double* y, hipStream_t s);

hipError_t launch_map(const ChannelTab* ct, const ProcessTab* pt, const double* grid, int nb, int dims, int n_slots,
                      int n_inv, int kinds, double s_lab, int np, int64_t n, const double* y, double* p,
                      double* x1x2, double* jac, double* w, int cu_count, hipStream_t s);

hipError_t launch_weight(const ChannelTab* ct, const ProcessTab* pt, int np, int64_t n, const double* p,
                         const double* x1x2, const double* jac, double* w, double* alpha, hipStream_t s);

hipError_t launch_sample(const ChannelTab* cts, const ProcessTab* pts, const double* grids, const int64_t* grid_off,
                         const int32_t* chan_nb, const SampleCall& call, int max_slots, int max_inv, int kinds,
                         size_t lds_bytes,
                         uint64_t seed, uint64_t sid, uint64_t ctr_off, int np, int64_t N, double* p, double* x1x2,
                         double* w, int32_t* chan, double* tile_stats, double* stats, int grid, hipStream_t s);

int sample_tile_size();

hipError_t launch_vegas_accumulate(int64_t n, int dims, int nb, const double* y, const double* w, double* part,
                                   int64_t nchunk, int64_t chunk, double* hist, hipStream_t s);

hipError_t launch_vegas_refine(int n_rows, const int32_t* row_nb, const int64_t* row_grid, const int64_t* row_hist,
                               double alpha, double* grids, double* hist, hipStream_t s);

}  // namespace msx

namespace msx {

// Unweighting-efficiency search, one refinement pass: histogram (count, sum)
// over bucket = (bits >> shift) & (2^width - 1) of every weight whose bit
// pattern above shift + width equals `prefix` (all weights when first).
hipError_t launch_unw_pass(int64_t n, const double* w, int shift, int width, uint64_t prefix, int first,
                           double* counts, double* sums, int cu_count, hipStream_t s);
// total sum and max of w (two doubles at out)
hipError_t launch_sum_max(int64_t n, const double* w, double* out, double* part, int nblk, hipStream_t s);

}  // namespace msx
