// C ABI of the phase-space library (declared in include/msx.h).
#include "../../include/msx.h"
#include "../../include/msx_flow.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "compiler.h"
#include "jit.h"
#include "json.h"
#include "launch.h"
#include "tables.h"

using namespace msx;

struct msx_ctx {
    int device = 0;
    int cu_count = 256;
    int mixed = 0;  // MSX_MIXED: FP32 transcendentals in the mapping chain
    Compiled comp;
    std::string err;
    // device tables
    ChannelTab* d_chans = nullptr;
    ProcessTab* d_procs = nullptr;
    double* d_grids = nullptr;      // all channels' edges, [dims][nb+1] each
    double* d_hist = nullptr;       // all channels' sum w^2 per bin, [dims][nb] each
    double* d_stats = nullptr;      // [C][5]
    int64_t* d_grid_off = nullptr;  // per channel offset into d_grids
    int32_t* d_chan_nb = nullptr;   // per channel bins
    int32_t* d_row_nb = nullptr;    // per (channel, dim) row: bins, grid offset, hist offset
    int64_t* d_row_grid = nullptr;
    int64_t* d_row_hist = nullptr;
    std::vector<int64_t> grid_off, hist_off;
    int64_t grid_total = 0, hist_total = 0;
    int n_rows = 0;
    int max_np = 0;
    // scratch, grown on demand
    double* d_tile = nullptr;
    int64_t tile_cap = 0;
    double* d_vpart = nullptr;
    double* d_obs_hist = nullptr;  // observable histogram partials
    int64_t obs_hist_cap = 0;
    int64_t* d_ublk = nullptr;  // unweighting block offsets
    int64_t ublk_cap = 0;
    double* d_inv = nullptr;  // multichannel density scratch: y [max dims][n] then jac [n]
    int64_t inv_cap = 0;      // doubles
    int64_t vpart_cap = 0;
    double* d_unw = nullptr;  // 3 * 4096 bucket words + 2 * 1024 partials + 2 + the search state (3)
    // VEGAS accumulation inside the fused sample: per-channel histogram
    // offsets (device), the per-tile partial stride and the partials
    int64_t* d_hist_off = nullptr;
    int vstride = 0;
    double* d_vtiles = nullptr;
    int64_t vtiles_cap = 0;  // tiles
    // device address of the library's fixed scratch on this device
    // (msx_sample_noalloc); not owned by the context
    double* d_noalloc = nullptr;
    // next event id of MSX_COUNTER_AUTO sample calls
    uint64_t next_counter = 0;
    // learned samplers attached per channel (not owned) and whether the
    // attach check enabled them
    std::vector<msx_flow*> flow;
    std::vector<int> flow_on;
    // MSX_SAMPLE_USE_FLOW scratch of one flow channel's events, and moment partials
    int64_t fs_cap = 0;
    float* fs_y = nullptr;
    float* fs_logq = nullptr;
    double* fs_p = nullptr;
    double* fs_x = nullptr;
    double* fs_wfj = nullptr;
    double* fs_w = nullptr;
    double* d_mom = nullptr;
    size_t lds_max = 0;
    SampleCall* d_call = nullptr;  // call table of the last sample launch
    // launch shape of the fused sample kernel (events per thread per tile,
    // workgroups of the persistent grid; 0 = 8 per compute unit)
    int ept = 1;
    int grid = 0;
    // register / kind class covering every channel (device-count launches)
    int all_slots = 0, all_inv = 0, all_kinds = 0;
    bool any_hadronic = false;
    // the fused sample compiled for these channels (msx_specialize); kept
    // loaded until msx_destroy once built, since captured graphs may use it
    JitSampleSet jit;
    bool jit_on = false;
};

struct msx_graph {
    int device = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // the graph's own call table and tile scratch (the context's may be
    // reallocated by later calls)
    SampleCall* d_call = nullptr;
    double* d_tile = nullptr;
    double* d_vtiles = nullptr;  // VEGAS tile partials (graphs that accumulate)
};

namespace {

thread_local std::string g_err;

msx_status fail(msx_ctx* ctx, msx_status st, const std::string& msg) {
    if (ctx) ctx->err = msg;
    else g_err = msg;
    return st;
}

msx_status dev_fail(msx_ctx* ctx, hipError_t e, const char* what) {
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(ctx, e == hipErrorOutOfMemory ? MSX_ERR_OOM : MSX_ERR_DEVICE, m);
}

#define MSX_HIP(ctx, call, what)                          \
    do {                                                  \
        hipError_t _e = (call);                           \
        if (_e != hipSuccess) return dev_fail(ctx, _e, what); \
    } while (0)

template <class T>
hipError_t dmalloc(T** p, size_t count) {
    return hipMalloc((void**)p, std::max<size_t>(count, 1) * sizeof(T));
}

void free_all(msx_ctx* c) {
    void* ptrs[] = {c->d_chans, c->d_procs, c->d_grids, c->d_hist, c->d_stats, c->d_grid_off, c->d_chan_nb,
                    c->d_row_nb, c->d_row_grid, c->d_row_hist, c->d_tile, c->d_vpart, c->d_unw, c->d_call,
                    c->d_inv, c->d_ublk, c->d_obs_hist, c->d_hist_off, c->d_vtiles, c->fs_y, c->fs_logq, c->fs_p,
                    c->fs_x, c->fs_wfj, c->fs_w, c->d_mom};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
}

bool bad_ctx(const msx_ctx* ctx) { return ctx == nullptr; }

const JitSampleSet* jit_of(const msx_ctx* ctx) { return ctx->jit_on ? &ctx->jit : nullptr; }

msx_status set_device(msx_ctx* ctx) {
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return dev_fail(ctx, e, "hipSetDevice");
    return MSX_OK;
}

msx_status ensure_tiles(msx_ctx* ctx, int64_t tiles) {
    if (tiles <= ctx->tile_cap) return MSX_OK;
    if (ctx->d_tile) MSX_HIP(ctx, hipFree(ctx->d_tile), "hipFree");
    ctx->d_tile = nullptr;
    ctx->tile_cap = 0;
    MSX_HIP(ctx, dmalloc(&ctx->d_tile, 4 * tiles), "tile scratch");
    ctx->tile_cap = tiles;
    return MSX_OK;
}

int sample_grid(const msx_ctx* ctx) { return ctx->grid > 0 ? ctx->grid : ctx->cu_count * 8; }

// Per-tile VEGAS histogram partials for `tiles` tiles (grown on demand).
msx_status ensure_vtiles(msx_ctx* ctx, int64_t tiles) {
    if (tiles <= ctx->vtiles_cap) return MSX_OK;
    if (ctx->d_vtiles) MSX_HIP(ctx, hipFree(ctx->d_vtiles), "hipFree");
    ctx->d_vtiles = nullptr;
    ctx->vtiles_cap = 0;
    MSX_HIP(ctx, dmalloc(&ctx->d_vtiles, (size_t)ctx->vstride * tiles), "VEGAS tile partials");
    ctx->vtiles_cap = tiles;
    return MSX_OK;
}

constexpr size_t kLdsPerWorkgroup = 160 * 1024;  // gfx950: 160 KiB of LDS per compute unit

// Checks the flags of a sample call; with MSX_SAMPLE_ACCUMULATE_VEGAS also
// that the kernel's LDS (staging column, grid, wave histograms) fits.
msx_status check_sample_flags(msx_ctx* ctx, int32_t flags, int max_slots, int max_inv) {
    if (flags & ~(MSX_SAMPLE_ACCUMULATE_VEGAS | MSX_SAMPLE_USE_FLOW | MSX_SAMPLE_ADVANCE_COUNTER))
        return fail(ctx, MSX_ERR_ARG, "unknown sample flags");
    if ((flags & MSX_SAMPLE_ACCUMULATE_VEGAS) &&
        sample_lds_bytes(max_slots, max_inv, ctx->lds_max, ctx->vstride) > kLdsPerWorkgroup)
        return fail(ctx, MSX_ERR_UNSUPPORTED,
                    "VEGAS accumulation in the fused sample needs more than 160 KiB of LDS for these channels "
                    "(dims x bins too large); use msx_vegas_accumulate");
    return MSX_OK;
}

// Device-count sample: plan kernel, then the fused launch with the register
// class of all channels.  Enqueues only (safe to capture).
int64_t device_max_tiles(const msx_ctx* ctx, int64_t capacity) {
    const int64_t T = (int64_t)sample_block() * ctx->ept;
    return (capacity + T - 1) / T + (int64_t)ctx->comp.chans.size();
}

// Device-count sample: plan kernel, then the fused launch with the register
// class of all channels.  Enqueues only (safe to capture).  d_tile must hold
// 4 * device_max_tiles(capacity) doubles.
msx_status sample_device(msx_ctx* ctx, const int64_t* counts, uint64_t seed, uint64_t stream_id,
                         const uint64_t* counter_offset, int64_t capacity, double* p, double* x1x2, double* w,
                         int32_t* chan, int32_t* status, SampleCall* d_call, double* d_tile, double* d_vtiles,
                         bool advance, hipStream_t s) {
    const int C = (int)ctx->comp.chans.size();
    const int64_t max_tiles = device_max_tiles(ctx, capacity);
    MSX_HIP(ctx, launch_plan(counts, C, capacity, ctx->ept, d_call, status, s), "sample plan");
    const int grid = (int)std::min<int64_t>(max_tiles, sample_grid(ctx));
    MSX_HIP(ctx,
            launch_sample(ctx->d_chans, ctx->d_procs, ctx->d_grids, ctx->d_grid_off, ctx->d_chan_nb, d_call, C,
                          ctx->all_slots, ctx->all_inv, ctx->all_kinds, ctx->mixed, ctx->lds_max, seed, stream_id,
                          counter_offset, 0, ctx->max_np, capacity, p, x1x2, w, chan, d_tile, ctx->d_stats, grid, s,
                          d_vtiles, ctx->vstride, ctx->d_hist_off, ctx->hist_total, ctx->d_hist, jit_of(ctx)),
            "sample launch");
    if (advance) MSX_HIP(ctx, launch_advance_counter(d_call, const_cast<uint64_t*>(counter_offset), s), "counter");
    return MSX_OK;
}

msx_status sample_with_flows(msx_ctx* ctx, const int64_t* counts, uint64_t seed, uint64_t stream_id,
                             uint64_t counter_offset, int32_t flags, double* p, double* x1x2, double* w, int32_t* chan,
                             void* stream);

msx_status check_channel(msx_ctx* ctx, int32_t channel) {
    if (channel < 0 || channel >= (int32_t)ctx->comp.chans.size())
        return fail(ctx, MSX_ERR_ARG, "channel index out of range");
    return MSX_OK;
}

}  // namespace

extern "C" {

const char* msx_last_error(const msx_ctx* ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

msx_status msx_create_channels(const char* process_json, int32_t precision, int32_t device, msx_ctx** out) {
    if (!out) return fail(nullptr, MSX_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!process_json) return fail(nullptr, MSX_ERR_ARG, "process_json is NULL");
    if (precision != MSX_FP64 && precision != MSX_MIXED)
        return fail(nullptr, MSX_ERR_ARG, "precision must be MSX_FP64 or MSX_MIXED");
    JValue root;
    std::string err;
    if (!parse_json(process_json, root, err)) return fail(nullptr, MSX_ERR_ARG, "JSON: " + err);
    msx_ctx* c = new msx_ctx();
    c->mixed = precision == MSX_MIXED ? 1 : 0;
    if (!compile_processes(root, c->comp, err)) {
        delete c;
        return fail(nullptr, MSX_ERR_ARG, "process description: " + err);
    }
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || device < 0 || device >= ndev) {
        delete c;
        return fail(nullptr, MSX_ERR_DEVICE, "no such HIP device");
    }
    c->device = device;
    if ((e = hipSetDevice(device)) != hipSuccess) {
        delete c;
        return fail(nullptr, MSX_ERR_DEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
        c->cu_count = cus;
    const int C = (int)c->comp.chans.size();
    std::vector<double> grids, hist_init;
    std::vector<int32_t> chan_nb(C), row_nb;
    std::vector<int64_t> row_grid, row_hist;
    for (int ch = 0; ch < C; ++ch) {
        const ChannelMeta& m = c->comp.meta[ch];
        c->grid_off.push_back((int64_t)grids.size());
        c->hist_off.push_back(c->hist_total);
        chan_nb[ch] = m.nbins;
        for (int k = 0; k < m.dims; ++k) {
            row_nb.push_back(m.nbins);
            row_grid.push_back((int64_t)grids.size());
            row_hist.push_back(c->hist_total + (int64_t)k * m.nbins);
            for (int i = 0; i <= m.nbins; ++i) grids.push_back((double)i / m.nbins);
        }
        c->hist_total += (int64_t)m.dims * m.nbins;
        c->max_np = std::max(c->max_np, m.n_momenta);
        c->lds_max = std::max(c->lds_max, sizeof(double) * (size_t)m.dims * (m.nbins + 1));
        c->all_slots = std::max(c->all_slots, c->comp.chans[ch].n_slots);
        c->all_inv = std::max(c->all_inv, c->comp.chans[ch].n_inv);
        c->all_kinds |= c->comp.chans[ch].kinds;
        c->any_hadronic = c->any_hadronic || m.hadronic;
    }
    c->grid_total = (int64_t)grids.size();
    c->n_rows = (int)row_nb.size();
    for (int ch = 0; ch < C; ++ch)
        c->vstride = std::max(c->vstride, c->comp.meta[ch].dims * c->comp.meta[ch].nbins);
    c->flow.assign(C, nullptr);
    c->flow_on.assign(C, 0);
    auto up = [&](void* dst, const void* src, size_t bytes) { return hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice); };
    if ((e = dmalloc(&c->d_chans, C)) != hipSuccess || (e = dmalloc(&c->d_procs, c->comp.procs.size())) != hipSuccess ||
        (e = dmalloc(&c->d_grids, grids.size())) != hipSuccess || (e = dmalloc(&c->d_hist, c->hist_total)) != hipSuccess ||
        (e = dmalloc(&c->d_stats, 5 * C)) != hipSuccess || (e = dmalloc(&c->d_grid_off, C)) != hipSuccess ||
        (e = dmalloc(&c->d_chan_nb, C)) != hipSuccess || (e = dmalloc(&c->d_row_nb, row_nb.size())) != hipSuccess ||
        (e = dmalloc(&c->d_row_grid, row_grid.size())) != hipSuccess ||
        (e = dmalloc(&c->d_row_hist, row_hist.size())) != hipSuccess ||
        (e = dmalloc(&c->d_unw, 3 * 4096 + 2 * 1024 + 2 + 3)) != hipSuccess || (e = dmalloc(&c->d_call, 1)) != hipSuccess ||
        (e = dmalloc(&c->d_hist_off, C)) != hipSuccess || (e = dmalloc(&c->d_mom, 4 * moments_blocks())) != hipSuccess ||
        (e = up(c->d_hist_off, c->hist_off.data(), sizeof(int64_t) * C)) != hipSuccess ||
        (e = up(c->d_chans, c->comp.chans.data(), sizeof(ChannelTab) * C)) != hipSuccess ||
        (e = up(c->d_procs, c->comp.procs.data(), sizeof(ProcessTab) * c->comp.procs.size())) != hipSuccess ||
        (e = up(c->d_grids, grids.data(), sizeof(double) * grids.size())) != hipSuccess ||
        (e = up(c->d_grid_off, c->grid_off.data(), sizeof(int64_t) * C)) != hipSuccess ||
        (e = up(c->d_chan_nb, chan_nb.data(), sizeof(int32_t) * C)) != hipSuccess ||
        (e = up(c->d_row_nb, row_nb.data(), sizeof(int32_t) * row_nb.size())) != hipSuccess ||
        (e = up(c->d_row_grid, row_grid.data(), sizeof(int64_t) * row_grid.size())) != hipSuccess ||
        (e = up(c->d_row_hist, row_hist.data(), sizeof(int64_t) * row_hist.size())) != hipSuccess ||
        (e = hipMemset(c->d_hist, 0, sizeof(double) * std::max<int64_t>(c->hist_total, 1))) != hipSuccess ||
        (e = hipMemset(c->d_stats, 0, sizeof(double) * 5 * C)) != hipSuccess ||
        (e = noalloc_scratch(device, &c->d_noalloc)) != hipSuccess) {
        std::string m = std::string("device setup: ") + hipGetErrorString(e);
        msx_status st = e == hipErrorOutOfMemory ? MSX_ERR_OOM : MSX_ERR_DEVICE;
        free_all(c);
        delete c;
        return fail(nullptr, st, m);
    }
    *out = c;
    return MSX_OK;
}

msx_status msx_destroy(msx_ctx* ctx) {
    if (!ctx) return MSX_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    free_all(ctx);
    jit_release(ctx->jit);
    delete ctx;
    return MSX_OK;
}

msx_status msx_specialize(msx_ctx* ctx, int32_t on) {
    if (bad_ctx(ctx)) return fail(nullptr, MSX_ERR_ARG, "ctx is NULL");
    if (!on) {
        ctx->jit_on = false;
        return MSX_OK;
    }
    if (ctx->jit.n == 0) {
        if (msx_status st = set_device(ctx)) return st;
        std::string err;
        bool spills = false;
        if (!jit_build_sample(ctx->comp, ctx->mixed, ctx->device, ctx->jit, err, spills))
            return fail(ctx, spills ? MSX_ERR_UNSUPPORTED : MSX_ERR_DEVICE, "specialised sample kernel: " + err);
    }
    ctx->jit_on = true;
    return MSX_OK;
}

msx_status msx_get_meta(const msx_ctx* ctx, int32_t key, int32_t index, int64_t* value) {
    msx_ctx* c = const_cast<msx_ctx*>(ctx);
    if (bad_ctx(ctx)) return fail(nullptr, MSX_ERR_ARG, "ctx is NULL");
    if (!value) return fail(c, MSX_ERR_ARG, "value is NULL");
    const int C = (int)ctx->comp.chans.size();
    auto chan = [&](int64_t v) -> msx_status {
        if (index < 0 || index >= C) return fail(c, MSX_ERR_ARG, "channel index out of range");
        *value = v;
        return MSX_OK;
    };
    switch (key) {
        case MSX_META_N_CHANNELS: *value = C; return MSX_OK;
        case MSX_META_MAX_MOMENTA: *value = ctx->max_np; return MSX_OK;
        case MSX_META_DEVICE: *value = ctx->device; return MSX_OK;
        case MSX_META_PRECISION: *value = ctx->mixed ? MSX_MIXED : MSX_FP64; return MSX_OK;
        case MSX_META_EVENTS_PER_THREAD: *value = ctx->ept; return MSX_OK;
        case MSX_META_GRID: *value = sample_grid(ctx); return MSX_OK;
        case MSX_META_COUNTER: *value = (int64_t)ctx->next_counter; return MSX_OK;
        case MSX_META_SPECIALIZED: *value = ctx->jit_on ? ctx->jit.n : 0; return MSX_OK;
        case MSX_META_FLOW:
            return chan(index >= 0 && index < C ? (ctx->flow[index] ? 1 + ctx->flow_on[index] : 0) : 0);
        case MSX_META_DIMS: return chan(index >= 0 && index < C ? ctx->comp.meta[index].dims : 0);
        case MSX_META_N_MOMENTA: return chan(index >= 0 && index < C ? ctx->comp.meta[index].n_momenta : 0);
        case MSX_META_HADRONIC: return chan(index >= 0 && index < C ? ctx->comp.meta[index].hadronic : 0);
        case MSX_META_VEGAS_BINS: return chan(index >= 0 && index < C ? ctx->comp.meta[index].nbins : 0);
        case MSX_META_PROCESS: return chan(index >= 0 && index < C ? ctx->comp.meta[index].process : 0);
        default: return fail(c, MSX_ERR_ARG, "unknown metadata key");
    }
}

msx_status msx_uniform(msx_ctx* ctx, uint64_t seed, uint64_t stream_id, uint64_t e0, int64_t n, int32_t d, double* y,
                       void* stream) {
    if (bad_ctx(ctx)) return fail(nullptr, MSX_ERR_ARG, "ctx is NULL");
    if (n < 0 || d < 1 || d > 64) return fail(ctx, MSX_ERR_ARG, "need n >= 0 and 1 <= d <= 64");
    if (n > 0 && !y) return fail(ctx, MSX_ERR_ARG, "y is NULL");
    if (n > 0 && e0 > UINT64_MAX - (uint64_t)n) return fail(ctx, MSX_ERR_ARG, "event ids overflow the counter");
    if (msx_status st = set_device(ctx)) return st;
    MSX_HIP(ctx, launch_uniform(seed, stream_id, e0, n, d, y, (hipStream_t)stream), "uniform launch");
    return MSX_OK;
}

msx_status msx_map(msx_ctx* ctx, int32_t channel, int64_t n, const double* y, double* p, double* x1x2, double* jac,
                   double* w, void* stream) {
    if (bad_ctx(ctx)) return fail(nullptr, MSX_ERR_ARG, "ctx is NULL");
    if (msx_status st = check_channel(ctx, channel)) return st;
    if (n < 0) return fail(ctx, MSX_ERR_ARG, "n < 0");
    const ChannelMeta& m = ctx->comp.meta[channel];
    if (n > 0 && (!y || !p || !jac)) return fail(ctx, MSX_ERR_ARG, "y, p and jac are required");
    if (m.hadronic && n > 0 && !x1x2) return fail(ctx, MSX_ERR_ARG, "x1x2 is required for hadronic beams");
    if (!m.hadronic && x1x2) return fail(ctx, MSX_ERR_ARG, "x1x2 must be NULL for fixed beams");
    if (n == 0) return MSX_OK;
    if (msx_status st = set_device(ctx)) return st;
    const ChannelTab& t = ctx->comp.chans[channel];
    const ProcessTab& pt = ctx->comp.procs[m.process];
    MSX_HIP(ctx,
            launch_map(ctx->d_chans + channel, ctx->d_procs + m.process, ctx->d_grids + ctx->grid_off[channel], m.nbins,
                       m.dims, t.n_slots, t.n_inv, t.kinds, ctx->mixed, pt.s_lab, m.n_momenta, n, y, p, x1x2, jac, w,
                       ctx->cu_count,
                       (hipStream_t)stream),
            "map launch");
    return MSX_OK;
}

msx_status msx_inverse_map(msx_ctx* ctx, int32_t channel, int64_t n, const double* p, const double* x1x2, double* y,
                           double* jac, void* stream) {
    if (bad_ctx(ctx)) return fail(nullptr, MSX_ERR_ARG, "ctx is NULL");
    if (msx_status st = check_channel(ctx, channel)) return st;
    if (n < 0) return fail(ctx, MSX_ERR_ARG, "n < 0");
    const ChannelMeta& m = ctx->comp.meta[channel];
    if (n > 0 && (!p || !y)) return fail(ctx, MSX_ERR_ARG, "p and y are required");
    if (m.hadronic && n > 0 && !x1x2) return fail(ctx, MSX_ERR_ARG, "x1x2 is required for hadronic beams");
    if (!m.hadronic && x1x2) return fail(ctx, MSX_ERR_ARG, "x1x2 must be NULL for fixed beams");
    if (n == 0) return MSX_OK;
    if (msx_status st = set_device(ctx)) return st;
    const ChannelTab& t = ctx->comp.chans[channel];
    const ProcessTab& pt = ctx->comp.procs[m.process];
    MSX_HIP(ctx,
            launch_inverse(ctx->d_chans + channel, ctx->d_grids + ctx->grid_off[channel], m.nbins, m.dims, t.n_slots,
                           t.n_inv, t.kinds, pt.s_lab, m.n_momenta, n, p, x1x2, y, jac, ctx->cu_count,
                           (hipStream_t)stream),
            "inverse launch");
    return MSX_OK;
}

msx_status msx_multichannel_density(msx_ctx* ctx, int32_t process, int64_t n, const double* p, const double* x1x2,
                                    const double* alpha, double* g, void* stream) {
    if (bad_ctx(ctx)) return fail(nullptr, MSX_ERR_ARG, "ctx is NULL");
    if (process < 0 || process >= (int32_t)ctx->comp.procs.size())
        return fail(ctx, MSX_ERR_ARG, "process index out of range");
    if (n < 0) return fail(ctx, MSX_ERR_ARG, "n < 0");
    if (n > 0 && (!p || !g || !alpha)) return fail(ctx, MSX_ERR_ARG, "p, alpha and g are required");
    std::vector<int> chans;
    int dmax = 0;
    for (int c = 0; c < (int)ctx->comp.meta.size(); ++c)
        if (ctx->comp.meta[c].process == process) {
            chans.push_back(c);
            dmax = std::max(dmax, ctx->comp.meta[c].dims);
        }
    const ChannelMeta& m0 = ctx->comp.meta[chans[0]];
    if (m0.hadronic && n > 0 && !x1x2) return fail(ctx, MSX_ERR_ARG, "x1x2 is required for hadronic beams");
    if (!m0.hadronic && x1x2) return fail(ctx, MSX_ERR_ARG, "x1x2 must be NULL for fixed beams");
    for (size_t i = 0; i < chans.size(); ++i)
        if (!(alpha[i] >= 0.0)) return fail(ctx, MSX_ERR_ARG, "alpha must be >= 0");
    if (n == 0) return MSX_OK;
    if (msx_status st = set_device(ctx)) return st;
    const int64_t need = (int64_t)(dmax + 1) * n;
    if (need > ctx->inv_cap) {
        // the previous scratch may still be read by work in flight
        MSX_HIP(ctx, hipDeviceSynchronize(), "synchronize");
        if (ctx->d_inv) MSX_HIP(ctx, hipFree(ctx->d_inv), "hipFree");
        ctx->d_inv = nullptr;
        ctx->inv_cap = 0;
        MSX_HIP(ctx, dmalloc(&ctx->d_inv, need), "density scratch");
        ctx->inv_cap = need;
    }
    double* y = ctx->d_inv;
    double* jac = ctx->d_inv + (int64_t)dmax * n;
    hipStream_t s = (hipStream_t)stream;
    for (size_t i = 0; i < chans.size(); ++i) {
        const int c = chans[i];
        const ChannelMeta& m = ctx->comp.meta[c];
        const ChannelTab& t = ctx->comp.chans[c];
        const ProcessTab& pt = ctx->comp.procs[m.process];
        MSX_HIP(ctx,
                launch_inverse(ctx->d_chans + c, ctx->d_grids + ctx->grid_off[c], m.nbins, m.dims, t.n_slots, t.n_inv,
                               t.kinds, pt.s_lab, m.n_momenta, n, p, x1x2, y, jac, ctx->cu_count, s),
                "inverse launch");
        MSX_HIP(ctx, launch_density_add(g, jac, alpha[i], n, i == 0, s), "density launch");
    }
    return MSX_OK;
}

msx_status msx_weight(msx_ctx* ctx, int32_t channel, int64_t n, const double* p, const double* x1x2,
                      const double* jac, double* w, double* alpha, void* stream) {
    if (bad_ctx(ctx)) return fail(nullptr, MSX_ERR_ARG, "ctx is NULL");
    if (msx_status st = check_channel(ctx, channel)) return st;
    if (n < 0) return fail(ctx, MSX_ERR_ARG, "n < 0");
    const ChannelMeta& m = ctx->comp.meta[channel];
    if (n > 0 && (!p || !jac || !w)) return fail(ctx, MSX_ERR_ARG, "p, jac and w are required");
    if (m.hadronic && n > 0 && !x1x2) return fail(ctx, MSX_ERR_ARG, "x1x2 is required for hadronic beams");
    if (n == 0) return MSX_OK;
    if (msx_status st = set_device(ctx)) return st;
    MSX_HIP(ctx,
            launch_weight(ctx->d_chans + channel, ctx->d_procs + m.process, ctx->mixed, m.n_momenta, n, p, x1x2, jac, w, alpha,
                          (hipStream_t)stream),
            "weight launch");
    return MSX_OK;
}

namespace {

// msx_sample and msx_sample_noalloc: with noalloc, the tile statistics go to
// the library's fixed device scratch (no allocation; flags must be 0).
msx_status sample_host(msx_ctx* ctx, const int64_t* counts, uint64_t seed, uint64_t stream_id,
                       uint64_t counter_offset, int32_t flags, double* p, double* x1x2, double* w, int32_t* chan,
                       void* stream, bool noalloc) {
    if (bad_ctx(ctx)) return fail(nullptr, MSX_ERR_ARG, "ctx is NULL");
    if (!counts) return fail(ctx, MSX_ERR_ARG, "counts is NULL");
    if (noalloc && flags != 0) return fail(ctx, MSX_ERR_UNSUPPORTED, "msx_sample_noalloc takes no flags");
    if (flags & MSX_SAMPLE_ADVANCE_COUNTER)
        return fail(ctx, MSX_ERR_ARG, "MSX_SAMPLE_ADVANCE_COUNTER is for device-count launches (MSX_COUNTER_AUTO here)");
    if (counter_offset == MSX_COUNTER_AUTO) {
        // the context's running event counter: resolve it, then advance it
        // by the events of this call once the call is accepted
        int64_t total = 0;
        for (int c = 0; c < (int)ctx->comp.chans.size(); ++c) {
            if (counts[c] < 0) return fail(ctx, MSX_ERR_ARG, "negative event count");
            if (counts[c] > INT64_MAX / 4 - total) return fail(ctx, MSX_ERR_ARG, "event count overflow");
            total += counts[c];
        }
        const uint64_t start = ctx->next_counter;
        if (start == MSX_COUNTER_AUTO || start > MSX_COUNTER_AUTO - 1 - (uint64_t)total)
            return fail(ctx, MSX_ERR_ARG, "the context's event counter is exhausted");
        msx_status st = sample_host(ctx, counts, seed, stream_id, start, flags, p, x1x2, w, chan, stream, noalloc);
        if (st == MSX_OK) ctx->next_counter = start + (uint64_t)total;
        return st;
    }
    if (flags & MSX_SAMPLE_USE_FLOW) return sample_with_flows(ctx, counts, seed, stream_id, counter_offset, flags, p,
                                                              x1x2, w, chan, stream);
    const int C = (int)ctx->comp.chans.size();
    SampleCall call;
    std::memset(&call, 0, sizeof call);
    call.n_chan = C;
    call.ept = ctx->ept;
    const int64_t T = (int64_t)sample_block() * ctx->ept;
    int64_t N = 0, tiles = 0;
    bool any_hadronic = false;
    int max_slots = 0, max_inv = 0, kinds = 0;
    for (int c = 0; c < C; ++c) {
        if (counts[c] < 0) return fail(ctx, MSX_ERR_ARG, "negative event count");
        call.ev_start[c] = N;
        call.tile_start[c] = tiles;
        if (counts[c] > INT64_MAX / 4 - N) return fail(ctx, MSX_ERR_ARG, "event count overflow");
        N += counts[c];
        tiles += (counts[c] + T - 1) / T;
        if (counts[c] > 0) {
            any_hadronic = any_hadronic || ctx->comp.meta[c].hadronic;
            max_slots = std::max(max_slots, ctx->comp.chans[c].n_slots);
            max_inv = std::max(max_inv, ctx->comp.chans[c].n_inv);
            kinds |= ctx->comp.chans[c].kinds;
        }
    }
    call.ev_start[C] = N;
    call.tile_start[C] = tiles;
    call.n_tiles = tiles;
    if (N == 0) return MSX_OK;
    if (counter_offset > UINT64_MAX - (uint64_t)N) return fail(ctx, MSX_ERR_ARG, "event ids overflow the counter");
    if (!p || !w) return fail(ctx, MSX_ERR_ARG, "p and w are required");
    if (any_hadronic && !x1x2) return fail(ctx, MSX_ERR_ARG, "x1x2 is required when a sampled channel is hadronic");
    if (msx_status st = check_sample_flags(ctx, flags, max_slots, max_inv)) return st;
    const bool acc = (flags & MSX_SAMPLE_ACCUMULATE_VEGAS) != 0;
    if (noalloc && tiles > kNoAllocTiles)
        return fail(ctx, MSX_ERR_ARG,
                    "msx_sample_noalloc: " + std::to_string(tiles) + " tiles of " + std::to_string(T) +
                        " events exceed the fixed scratch of " + std::to_string(kNoAllocTiles) + " tiles");
    if (msx_status st = set_device(ctx)) return st;
    if (!noalloc)
        if (msx_status st = ensure_tiles(ctx, tiles)) return st;
    if (acc)
        if (msx_status st = ensure_vtiles(ctx, tiles)) return st;
    hipStream_t s = (hipStream_t)stream;
    MSX_HIP(ctx, launch_set_call(call, ctx->d_call, s), "sample call table");
    const int grid = (int)std::min<int64_t>(tiles, sample_grid(ctx));
    MSX_HIP(ctx,
            launch_sample(ctx->d_chans, ctx->d_procs, ctx->d_grids, ctx->d_grid_off, ctx->d_chan_nb, ctx->d_call, C,
                          max_slots, max_inv, kinds, ctx->mixed, ctx->lds_max, seed, stream_id, nullptr,
                          counter_offset, ctx->max_np, N, p, x1x2, w, chan, noalloc ? ctx->d_noalloc : ctx->d_tile,
                          ctx->d_stats, grid, s, acc ? ctx->d_vtiles : nullptr, ctx->vstride, ctx->d_hist_off,
                          ctx->hist_total, ctx->d_hist, jit_of(ctx)),
            "sample launch");
    return MSX_OK;
}

}  // namespace

msx_status msx_sample(msx_ctx* ctx, const int64_t* counts, uint64_t seed, uint64_t stream_id, uint64_t counter_offset,
                      int32_t flags, double* p, double* x1x2, double* w, int32_t* chan, void* stream) {
    return sample_host(ctx, counts, seed, stream_id, counter_offset, flags, p, x1x2, w, chan, stream, false);
}

msx_status msx_sample_noalloc(msx_ctx* ctx, const int64_t* counts, uint64_t seed, uint64_t stream_id,
                              uint64_t counter_offset, double* p, double* x1x2, double* w, int32_t* chan,
                              void* stream) {
    return sample_host(ctx, counts, seed, stream_id, counter_offset, 0, p, x1x2, w, chan, stream, true);
}

msx_status msx_sample_device(msx_ctx* ctx, const int64_t* counts, uint64_t seed, uint64_t stream_id,
                             const uint64_t* counter_offset, int64_t capacity, int32_t flags, double* p, double* x1x2,
                             double* w, int32_t* chan, int32_t* status, void* stream) {
    if (bad_ctx(ctx)) return fail(nullptr, MSX_ERR_ARG, "ctx is NULL");
    if (!counts || !counter_offset) return fail(ctx, MSX_ERR_ARG, "counts and counter_offset are required");
    if (capacity <= 0) return fail(ctx, MSX_ERR_ARG, "capacity must be positive");
    if (!p || !w) return fail(ctx, MSX_ERR_ARG, "p and w are required");
    if (ctx->any_hadronic && !x1x2) return fail(ctx, MSX_ERR_ARG, "x1x2 is required (the context has hadronic channels)");
    if (flags & MSX_SAMPLE_USE_FLOW) return fail(ctx, MSX_ERR_UNSUPPORTED, "MSX_SAMPLE_USE_FLOW needs host counts");
    if (msx_status st = check_sample_flags(ctx, flags, ctx->all_slots, ctx->all_inv)) return st;
    const bool acc = (flags & MSX_SAMPLE_ACCUMULATE_VEGAS) != 0;
    if (msx_status st = set_device(ctx)) return st;
    const int64_t max_tiles = device_max_tiles(ctx, capacity);
    if (msx_status st = ensure_tiles(ctx, max_tiles)) return st;
    if (acc)
        if (msx_status st = ensure_vtiles(ctx, max_tiles)) return st;
    return sample_device(ctx, counts, seed, stream_id, counter_offset, capacity, p, x1x2, w, chan, status,
                         ctx->d_call, ctx->d_tile, acc ? ctx->d_vtiles : nullptr,
                         (flags & MSX_SAMPLE_ADVANCE_COUNTER) != 0, (hipStream_t)stream);
}

msx_status msx_sample_graph_create(msx_ctx* ctx, const int64_t* counts, uint64_t seed, uint64_t stream_id,
                                   const uint64_t* counter_offset, int64_t capacity, int32_t flags, double* p,
                                   double* x1x2, double* w, int32_t* chan, int32_t* status, msx_graph** out) {
    if (!out) return fail(ctx, MSX_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (bad_ctx(ctx)) return fail(nullptr, MSX_ERR_ARG, "ctx is NULL");
    if (!counts || !counter_offset) return fail(ctx, MSX_ERR_ARG, "counts and counter_offset are required");
    if (capacity <= 0) return fail(ctx, MSX_ERR_ARG, "capacity must be positive");
    if (!p || !w) return fail(ctx, MSX_ERR_ARG, "p and w are required");
    if (ctx->any_hadronic && !x1x2) return fail(ctx, MSX_ERR_ARG, "x1x2 is required (the context has hadronic channels)");
    if (flags & MSX_SAMPLE_USE_FLOW) return fail(ctx, MSX_ERR_UNSUPPORTED, "MSX_SAMPLE_USE_FLOW needs host counts");
    if (msx_status st = check_sample_flags(ctx, flags, ctx->all_slots, ctx->all_inv)) return st;
    const bool acc = (flags & MSX_SAMPLE_ACCUMULATE_VEGAS) != 0;
    if (msx_status st = set_device(ctx)) return st;
    // everything the launches need is allocated before the capture
    msx_graph* g = new msx_graph();
    g->device = ctx->device;
    auto drop = [&](msx_graph* q) {
        if (q->exec) (void)hipGraphExecDestroy(q->exec);
        if (q->graph) (void)hipGraphDestroy(q->graph);
        if (q->d_call) (void)hipFree(q->d_call);
        if (q->d_tile) (void)hipFree(q->d_tile);
        if (q->d_vtiles) (void)hipFree(q->d_vtiles);
        delete q;
    };
    hipError_t e = dmalloc(&g->d_call, 1);
    if (e == hipSuccess) e = dmalloc(&g->d_tile, (size_t)4 * device_max_tiles(ctx, capacity));
    if (e == hipSuccess && acc) e = dmalloc(&g->d_vtiles, (size_t)ctx->vstride * device_max_tiles(ctx, capacity));
    if (e != hipSuccess) {
        drop(g);
        return dev_fail(ctx, e, "graph scratch");
    }
    hipStream_t s = nullptr;
    if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess) {
        drop(g);
        return dev_fail(ctx, e, "capture stream");
    }
    e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    msx_status st = MSX_OK;
    if (e == hipSuccess) {
        st = sample_device(ctx, counts, seed, stream_id, counter_offset, capacity, p, x1x2, w, chan, status, g->d_call,
                           g->d_tile, g->d_vtiles, (flags & MSX_SAMPLE_ADVANCE_COUNTER) != 0, s);
        hipError_t e2 = hipStreamEndCapture(s, &g->graph);
        if (st == MSX_OK && e2 != hipSuccess) e = e2;
    }
    if (e == hipSuccess && st == MSX_OK) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(s);
    if (e != hipSuccess || st != MSX_OK) {
        drop(g);
        return st != MSX_OK ? st : dev_fail(ctx, e, "graph capture");
    }
    *out = g;
    return MSX_OK;
}

msx_status msx_graph_launch(msx_graph* g, void* stream) {
    if (!g) return fail(nullptr, MSX_ERR_ARG, "graph is NULL");
    hipError_t e = hipSetDevice(g->device);
    if (e == hipSuccess) e = hipGraphLaunch(g->exec, (hipStream_t)stream);
    if (e != hipSuccess) return dev_fail(nullptr, e, "graph launch");
    return MSX_OK;
}

msx_status msx_graph_destroy(msx_graph* g) {
    if (!g) return MSX_OK;
    (void)hipSetDevice(g->device);
    (void)hipDeviceSynchronize();
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->d_call) (void)hipFree(g->d_call);
    if (g->d_tile) (void)hipFree(g->d_tile);
    if (g->d_vtiles) (void)hipFree(g->d_vtiles);
    delete g;
    return MSX_OK;
}

msx_status msx_set_launch(msx_ctx* ctx, int32_t events_per_thread, int32_t grid) {
    if (bad_ctx(ctx)) return fail(nullptr, MSX_ERR_ARG, "ctx is NULL");
    if (events_per_thread < 1 || events_per_thread > 64) return fail(ctx, MSX_ERR_ARG, "events_per_thread must be 1..64");
    if (grid < 0 || grid > (1 << 20)) return fail(ctx, MSX_ERR_ARG, "grid must be 0..2^20");
    ctx->ept = events_per_thread;
    ctx->grid = grid;
    return MSX_OK;
}

msx_status msx_autotune(msx_ctx* ctx, const int64_t* counts, uint64_t seed, int32_t reps, double* best_ms) {
    if (bad_ctx(ctx)) return fail(nullptr, MSX_ERR_ARG, "ctx is NULL");
    if (!counts) return fail(ctx, MSX_ERR_ARG, "counts is NULL");
    if (reps < 1 || reps > 1000) return fail(ctx, MSX_ERR_ARG, "reps must be 1..1000");
    const int C = (int)ctx->comp.chans.size();
    int64_t N = 0;
    for (int c = 0; c < C; ++c) {
        if (counts[c] < 0 || counts[c] > INT64_MAX / 4 - N) return fail(ctx, MSX_ERR_ARG, "bad event count");
        N += counts[c];
    }
    if (N == 0) return fail(ctx, MSX_ERR_ARG, "no events to time");
    if (msx_status st = set_device(ctx)) return st;
    // scratch outputs for the trial launches
    double *p = nullptr, *x1x2 = nullptr, *w = nullptr, *stats_save = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&]() {
        if (p) (void)hipFree(p);
        if (x1x2) (void)hipFree(x1x2);
        if (w) (void)hipFree(w);
        if (stats_save) (void)hipFree(stats_save);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (s) (void)hipStreamDestroy(s);
    };
    hipError_t e;
    if ((e = dmalloc(&p, (size_t)4 * ctx->max_np * N)) != hipSuccess || (e = dmalloc(&x1x2, (size_t)2 * N)) != hipSuccess ||
        (e = dmalloc(&w, (size_t)N)) != hipSuccess || (e = dmalloc(&stats_save, (size_t)5 * C)) != hipSuccess ||
        (e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess ||
        (e = hipMemcpy(stats_save, ctx->d_stats, sizeof(double) * 5 * C, hipMemcpyDeviceToDevice)) != hipSuccess) {
        cleanup();
        return dev_fail(ctx, e, "autotune setup");
    }
    const int ept_c[] = {1, 2, 4};
    const int mult_c[] = {2, 4, 8, 16};
    double best = 1e300;
    int best_ept = 1, best_grid = 0;
    const int save_ept = ctx->ept, save_grid = ctx->grid;
    msx_status st = MSX_OK;
    for (int ept : ept_c) {
        for (int mult : mult_c) {
            ctx->ept = ept;
            ctx->grid = ctx->cu_count * mult;
            // one untimed launch, then reps timed ones
            st = msx_sample(ctx, counts, seed, 0, 0, 0, p, x1x2, w, nullptr, s);
            for (int r = 0; st == MSX_OK && r < reps; ++r) {
                if (r == 0) (void)hipEventRecord(e0, s);
                st = msx_sample(ctx, counts, seed, 0, 0, 0, p, x1x2, w, nullptr, s);
            }
            if (st != MSX_OK) break;
            (void)hipEventRecord(e1, s);
            if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            const double per = ms / reps;
            if (per < best) {
                best = per;
                best_ept = ept;
                best_grid = ctx->grid;
            }
        }
        if (st != MSX_OK || e != hipSuccess) break;
    }
    ctx->ept = save_ept;
    ctx->grid = save_grid;
    if (st == MSX_OK && e == hipSuccess) {
        // the trial launches accumulated statistics: restore them
        e = hipMemcpy(ctx->d_stats, stats_save, sizeof(double) * 5 * C, hipMemcpyDeviceToDevice);
        if (e == hipSuccess) e = hipDeviceSynchronize();
    }
    cleanup();
    if (st != MSX_OK) return st;
    if (e != hipSuccess) return dev_fail(ctx, e, "autotune");
    ctx->ept = best_ept;
    ctx->grid = best_grid;
    if (best_ms) *best_ms = best;
    return MSX_OK;
}

msx_status msx_stats(msx_ctx* ctx, double* out, void* stream) {
    if (bad_ctx(ctx)) return fail(nullptr, MSX_ERR_ARG, "ctx is NULL");
    if (!out) return fail(ctx, MSX_ERR_ARG, "out is NULL");
    if (msx_status st = set_device(ctx)) return st;
    const int C = (int)ctx->comp.chans.size();
    MSX_HIP(ctx, hipMemcpyAsync(out, ctx->d_stats, sizeof(double) * 5 * C, hipMemcpyDeviceToHost, (hipStream_t)stream),
            "stats copy");
    MSX_HIP(ctx, hipStreamSynchronize((hipStream_t)stream), "stats sync");
    return MSX_OK;
}

msx_status msx_reset_stats(msx_ctx* ctx, void* stream) {
    if (bad_ctx(ctx)) return fail(nullptr, MSX_ERR_ARG, "ctx is NULL");
    if (msx_status st = set_device(ctx)) return st;
    const int C = (int)ctx->comp.chans.size();
    MSX_HIP(ctx, hipMemsetAsync(ctx->d_stats, 0, sizeof(double) * 5 * C, (hipStream_t)stream), "stats reset");
    return MSX_OK;
}

msx_status msx_vegas_accumulate(msx_ctx* ctx, int32_t channel, int64_t n, const double* y, const double* w,
                                void* stream) {
    if (bad_ctx(ctx)) return fail(nullptr, MSX_ERR_ARG, "ctx is NULL");
    if (msx_status st = check_channel(ctx, channel)) return st;
    if (n < 0) return fail(ctx, MSX_ERR_ARG, "n < 0");
    if (n == 0) return MSX_OK;
    if (!y || !w) return fail(ctx, MSX_ERR_ARG, "y and w are required");
    if (msx_status st = set_device(ctx)) return st;
    const ChannelMeta& m = ctx->comp.meta[channel];
    const int64_t chunk_min = 4096;
    int64_t nchunk = std::min<int64_t>(1024, (n + chunk_min - 1) / chunk_min);
    int64_t chunk = (n + nchunk - 1) / nchunk;
    int64_t need = nchunk * m.dims * m.nbins;
    if (need > ctx->vpart_cap) {
        if (ctx->d_vpart) MSX_HIP(ctx, hipFree(ctx->d_vpart), "hipFree");
        ctx->d_vpart = nullptr;
        ctx->vpart_cap = 0;
        MSX_HIP(ctx, dmalloc(&ctx->d_vpart, need), "histogram scratch");
        ctx->vpart_cap = need;
    }
    MSX_HIP(ctx,
            launch_vegas_accumulate(n, m.dims, m.nbins, y, w, ctx->d_vpart, nchunk, chunk,
                                    ctx->d_hist + ctx->hist_off[channel], (hipStream_t)stream),
            "histogram launch");
    return MSX_OK;
}

msx_status msx_vegas_update(msx_ctx* ctx, double alpha, void* stream) {
    if (bad_ctx(ctx)) return fail(nullptr, MSX_ERR_ARG, "ctx is NULL");
    if (!(alpha > 0.0) || !std::isfinite(alpha)) return fail(ctx, MSX_ERR_ARG, "alpha must be finite and > 0");
    if (msx_status st = set_device(ctx)) return st;
    MSX_HIP(ctx,
            launch_vegas_refine(ctx->n_rows, ctx->d_row_nb, ctx->d_row_grid, ctx->d_row_hist, alpha, ctx->d_grids,
                                ctx->d_hist, (hipStream_t)stream),
            "refine launch");
    return MSX_OK;
}

msx_status msx_vegas_adapt(msx_ctx* ctx, int64_t n_per_channel, int32_t iterations, double alpha, uint64_t seed,
                           uint64_t stream_id, uint64_t counter_offset, double* stats_out, void* stream) {
    if (bad_ctx(ctx)) return fail(nullptr, MSX_ERR_ARG, "ctx is NULL");
    if (n_per_channel < 1 || iterations < 1) return fail(ctx, MSX_ERR_ARG, "need n_per_channel >= 1 and iterations >= 1");
    if (!(alpha > 0.0) || !std::isfinite(alpha)) return fail(ctx, MSX_ERR_ARG, "alpha must be finite and > 0");
    const int C = (int)ctx->comp.chans.size();
    if (n_per_channel > INT64_MAX / 8 / C / iterations) return fail(ctx, MSX_ERR_ARG, "too many events");
    const int64_t N = n_per_channel * C;
    if (counter_offset > UINT64_MAX - (uint64_t)(N * iterations))
        return fail(ctx, MSX_ERR_ARG, "event ids overflow the counter");
    if (msx_status st = set_device(ctx)) return st;
    hipStream_t s = (hipStream_t)stream;
    double *p = nullptr, *x1x2 = nullptr, *w = nullptr;
    auto cleanup = [&]() {
        if (p) (void)hipFree(p);
        if (x1x2) (void)hipFree(x1x2);
        if (w) (void)hipFree(w);
    };
    hipError_t e;
    if ((e = dmalloc(&p, (size_t)4 * ctx->max_np * N)) != hipSuccess ||
        (ctx->any_hadronic && (e = dmalloc(&x1x2, (size_t)2 * N)) != hipSuccess) ||
        (e = dmalloc(&w, (size_t)N)) != hipSuccess) {
        cleanup();
        return dev_fail(ctx, e, "adaptation buffers");
    }
    std::vector<int64_t> counts(C, n_per_channel);
    msx_status st = MSX_OK;
    for (int it = 0; it < iterations && st == MSX_OK; ++it) {
        st = msx_reset_stats(ctx, stream);
        if (st == MSX_OK)
            st = msx_sample(ctx, counts.data(), seed, stream_id, counter_offset + (uint64_t)it * (uint64_t)N,
                            MSX_SAMPLE_ACCUMULATE_VEGAS, p, x1x2, w, nullptr, stream);
        if (st == MSX_OK && stats_out && it == iterations - 1) st = msx_stats(ctx, stats_out, stream);
        if (st == MSX_OK) st = msx_vegas_update(ctx, alpha, stream);
    }
    if (st == MSX_OK) st = msx_reset_stats(ctx, stream);
    if (st == MSX_OK && (e = hipStreamSynchronize(s)) != hipSuccess) st = dev_fail(ctx, e, "adaptation sync");
    cleanup();
    return st;
}

msx_status msx_allocate_counts(int32_t n_channels, const double* stats, int64_t total, double floor_frac,
                               int64_t* counts) {
    if (n_channels < 1 || !stats || !counts) return fail(nullptr, MSX_ERR_ARG, "need n_channels >= 1, stats and counts");
    if (total < 0) return fail(nullptr, MSX_ERR_ARG, "total < 0");
    if (!(floor_frac >= 0.0) || floor_frac * n_channels > 1.0)
        return fail(nullptr, MSX_ERR_ARG, "floor_frac must lie in [0, 1 / n_channels]");
    const int C = n_channels;
    std::vector<double> sd(C);
    double sum_sd = 0.0;
    for (int c = 0; c < C; ++c) {
        const double* st = stats + 5 * c;
        for (int j = 0; j < 5; ++j)
            if (!std::isfinite(st[j])) return fail(nullptr, MSX_ERR_ARG, "statistics must be finite");
        const double n = std::max(st[2], 1.0);
        const double mean = st[0] / n;
        sd[c] = std::sqrt(std::max(st[1] / n - mean * mean, 0.0));
        sum_sd += sd[c];
    }
    const int64_t floor_n = (int64_t)(floor_frac * (double)total);
    const int64_t rest = total - floor_n * C;
    int64_t assigned = 0;
    int arg = 0;
    double best = -1.0;
    for (int c = 0; c < C; ++c) {
        const double share = sum_sd > 0.0 ? sd[c] / sum_sd : 1.0 / C;
        counts[c] = floor_n + (int64_t)std::floor(share * (double)rest);
        assigned += counts[c];
        if (share > best) {
            best = share;
            arg = c;
        }
    }
    counts[arg] += total - assigned;
    return MSX_OK;
}

msx_status msx_get_grid(msx_ctx* ctx, int32_t channel, double* edges) {
    if (bad_ctx(ctx)) return fail(nullptr, MSX_ERR_ARG, "ctx is NULL");
    if (msx_status st = check_channel(ctx, channel)) return st;
    if (!edges) return fail(ctx, MSX_ERR_ARG, "edges is NULL");
    if (msx_status st = set_device(ctx)) return st;
    const ChannelMeta& m = ctx->comp.meta[channel];
    MSX_HIP(ctx, hipDeviceSynchronize(), "sync");
    MSX_HIP(ctx,
            hipMemcpy(edges, ctx->d_grids + ctx->grid_off[channel], sizeof(double) * m.dims * (m.nbins + 1),
                      hipMemcpyDeviceToHost),
            "grid copy");
    return MSX_OK;
}

msx_status msx_set_grid(msx_ctx* ctx, int32_t channel, const double* edges) {
    if (bad_ctx(ctx)) return fail(nullptr, MSX_ERR_ARG, "ctx is NULL");
    if (msx_status st = check_channel(ctx, channel)) return st;
    if (!edges) return fail(ctx, MSX_ERR_ARG, "edges is NULL");
    const ChannelMeta& m = ctx->comp.meta[channel];
    for (int k = 0; k < m.dims; ++k) {
        const double* e = edges + (size_t)k * (m.nbins + 1);
        if (e[0] != 0.0 || e[m.nbins] != 1.0) return fail(ctx, MSX_ERR_ARG, "grid edges must run from 0 to 1");
        for (int i = 0; i < m.nbins; ++i)
            if (!(e[i + 1] > e[i])) return fail(ctx, MSX_ERR_ARG, "grid edges must increase strictly");
    }
    if (msx_status st = set_device(ctx)) return st;
    MSX_HIP(ctx, hipDeviceSynchronize(), "sync");
    MSX_HIP(ctx,
            hipMemcpy(ctx->d_grids + ctx->grid_off[channel], edges, sizeof(double) * m.dims * (m.nbins + 1),
                      hipMemcpyHostToDevice),
            "grid copy");
    return MSX_OK;
}

msx_status msx_observables(msx_ctx* ctx, int32_t process, int64_t n, const double* p, const int32_t* spec, int32_t k,
                           double* out, void* stream) {
    if (bad_ctx(ctx)) return fail(nullptr, MSX_ERR_ARG, "ctx is NULL");
    if (process < 0 || process >= (int32_t)ctx->comp.procs.size())
        return fail(ctx, MSX_ERR_ARG, "process index out of range");
    if (n < 0) return fail(ctx, MSX_ERR_ARG, "n < 0");
    if (k < 1 || k > 8 || !spec) return fail(ctx, MSX_ERR_ARG, "1 to 8 observables are required");
    const int nf = ctx->comp.procs[process].n_final;
    for (int j = 0; j < k; ++j) {
        const int kind = spec[4 * j];
        const uint32_t set = (uint32_t)spec[4 * j + 1];
        if (kind < MSX_OBS_E || kind > MSX_OBS_DR_HARDEST) return fail(ctx, MSX_ERR_ARG, "unknown observable kind");
        if (set == 0 || (nf < 32 && (set >> nf) != 0)) return fail(ctx, MSX_ERR_ARG, "observable particle set out of range");
        if (kind == MSX_OBS_PT_RANK && (spec[4 * j + 2] < 0 || spec[4 * j + 2] >= nf))
            return fail(ctx, MSX_ERR_ARG, "rank out of range");
    }
    if (n > 0 && (!p || !out)) return fail(ctx, MSX_ERR_ARG, "p and out are required");
    if (n == 0) return MSX_OK;
    if (msx_status st = set_device(ctx)) return st;
    MSX_HIP(ctx, launch_observables(p, nf + 2, n, spec, k, out, (hipStream_t)stream), "observables launch");
    return MSX_OK;
}

msx_status msx_cut(msx_ctx* ctx, int64_t n, const double* x, int32_t k, const double* lo, const double* hi, double* w,
                   void* stream) {
    if (bad_ctx(ctx)) return fail(nullptr, MSX_ERR_ARG, "ctx is NULL");
    if (n < 0) return fail(ctx, MSX_ERR_ARG, "n < 0");
    if (k < 1 || k > 8 || !lo || !hi) return fail(ctx, MSX_ERR_ARG, "1 to 8 cut ranges are required");
    if (n > 0 && (!x || !w)) return fail(ctx, MSX_ERR_ARG, "x and w are required");
    if (n == 0) return MSX_OK;
    if (msx_status st = set_device(ctx)) return st;
    MSX_HIP(ctx, launch_cut(x, k, n, lo, hi, w, (hipStream_t)stream), "cut launch");
    return MSX_OK;
}

msx_status msx_histogram(msx_ctx* ctx, int64_t n, const double* x, const double* w, int32_t bins, double lo, double hi,
                         double* hist, void* stream) {
    if (bad_ctx(ctx)) return fail(nullptr, MSX_ERR_ARG, "ctx is NULL");
    if (n < 0) return fail(ctx, MSX_ERR_ARG, "n < 0");
    if (bins < 1 || bins > 4096) return fail(ctx, MSX_ERR_ARG, "bins must be 1..4096");
    if (!(hi > lo) || !std::isfinite(lo) || !std::isfinite(hi)) return fail(ctx, MSX_ERR_ARG, "need finite lo < hi");
    if (!hist || (n > 0 && (!x || !w))) return fail(ctx, MSX_ERR_ARG, "x, w and hist are required");
    if (msx_status st = set_device(ctx)) return st;
    const int64_t need = histogram_blocks(n) * 2 * (int64_t)bins;
    if (need > ctx->obs_hist_cap) {
        // the previous scratch may still be read by work in flight
        MSX_HIP(ctx, hipDeviceSynchronize(), "synchronize");
        if (ctx->d_obs_hist) MSX_HIP(ctx, hipFree(ctx->d_obs_hist), "hipFree");
        ctx->d_obs_hist = nullptr;
        ctx->obs_hist_cap = 0;
        MSX_HIP(ctx, dmalloc(&ctx->d_obs_hist, need), "histogram scratch");
        ctx->obs_hist_cap = need;
    }
    MSX_HIP(ctx, launch_histogram(x, w, n, bins, lo, hi, ctx->d_obs_hist, hist, (hipStream_t)stream), "histogram launch");
    return MSX_OK;
}

msx_status msx_unweight(msx_ctx* ctx, const double* w, int64_t n, double w_max, uint64_t seed, uint64_t stream_id,
                        uint64_t counter_offset, int64_t* keep, double* uw, int64_t* count, void* stream) {
    if (bad_ctx(ctx)) return fail(nullptr, MSX_ERR_ARG, "ctx is NULL");
    if (n < 0) return fail(ctx, MSX_ERR_ARG, "n < 0");
    if (!count) return fail(ctx, MSX_ERR_ARG, "count is required");
    if (n > 0 && (!w || !keep)) return fail(ctx, MSX_ERR_ARG, "w and keep are required");
    if (!(w_max > 0.0) || !std::isfinite(w_max)) return fail(ctx, MSX_ERR_ARG, "w_max must be finite and > 0");
    if (msx_status st = set_device(ctx)) return st;
    const int64_t nb = std::max<int64_t>(1, unweight_blocks(n));
    if (nb > ctx->ublk_cap) {
        // the previous scratch may still be read by work in flight
        MSX_HIP(ctx, hipDeviceSynchronize(), "synchronize");
        if (ctx->d_ublk) MSX_HIP(ctx, hipFree(ctx->d_ublk), "hipFree");
        ctx->d_ublk = nullptr;
        ctx->ublk_cap = 0;
        MSX_HIP(ctx, dmalloc(&ctx->d_ublk, nb), "unweighting scratch");
        ctx->ublk_cap = nb;
    }
    MSX_HIP(ctx,
            launch_unweight(w, n, w_max, seed, stream_id, counter_offset, ctx->d_ublk, keep, uw, count,
                            (hipStream_t)stream),
            "unweighting launch");
    return MSX_OK;
}

msx_status msx_unweight_eff(msx_ctx* ctx, const double* w, int64_t n, double overweight, double* eff, double* w_max,
                            void* stream) {
    if (bad_ctx(ctx)) return fail(nullptr, MSX_ERR_ARG, "ctx is NULL");
    if (n <= 0 || !w) return fail(ctx, MSX_ERR_ARG, "need n > 0 weights");
    if (!eff || !w_max) return fail(ctx, MSX_ERR_ARG, "eff and w_max are required");
    if (!(overweight > 0.0 && overweight < 1.0)) return fail(ctx, MSX_ERR_ARG, "overweight must be in (0, 1)");
    if (msx_status st = set_device(ctx)) return st;
    hipStream_t s = (hipStream_t)stream;
    uint64_t* counts = (uint64_t*)ctx->d_unw;
    uint64_t* sum_hi = counts + kUnwMaxBuckets;
    uint64_t* sum_lo = counts + 2 * kUnwMaxBuckets;
    double* part = ctx->d_unw + 3 * kUnwMaxBuckets;
    double* tot = part + 2 * 1024;
    UnwState* st = (UnwState*)(tot + 2);
    if (n >= (int64_t(1) << 36)) return fail(ctx, MSX_ERR_ARG, "at most 2^36 weights");
    const int nblk = (int)std::min<int64_t>(1024, (n + 255) / 256);
    MSX_HIP(ctx, hipMemsetAsync(ctx->d_unw, 0, sizeof(uint64_t) * 3 * kUnwMaxBuckets, s), "memset");
    MSX_HIP(ctx, hipMemsetAsync(st, 0, sizeof(UnwState), s), "memset");
    MSX_HIP(ctx, launch_sum_max(n, w, tot, part, nblk, s), "sum launch");
    MSX_HIP(ctx, launch_unw_search(n, w, overweight, tot, st, counts, sum_hi, sum_lo, ctx->cu_count, s), "search");
    double hs[2];
    UnwState hst;
    MSX_HIP(ctx, hipMemcpyAsync(hs, tot, sizeof hs, hipMemcpyDeviceToHost, s), "copy");
    MSX_HIP(ctx, hipMemcpyAsync(&hst, st, sizeof hst, hipMemcpyDeviceToHost, s), "copy");
    MSX_HIP(ctx, hipStreamSynchronize(s), "sync");
    const double total = hs[0];
    if (!(total > 0.0) || !std::isfinite(total)) return fail(ctx, MSX_ERR_ARG, "weights must be finite with a positive sum");
    const double target = overweight * total;
    const uint64_t prefix = hst.prefix;
    const double S_up = hst.S_up, N_up = hst.N_up;
    // the crossing bucket is now the single value v; for W in [v, next) the
    // weights above W are exactly those counted in S_up / N_up
    double v;
    std::memcpy(&v, &prefix, sizeof v);
    double W = N_up > 0.0 ? (S_up - target) / N_up : v;
    if (W < v) W = v;
    *w_max = W;
    *eff = W > 0.0 ? (total / (double)n) / W : 0.0;
    return MSX_OK;
}

}  // extern "C"

namespace {

msx_status ensure_flow_scratch(msx_ctx* ctx, int64_t n, int dims) {
    if (n <= ctx->fs_cap) return MSX_OK;
    void** ptrs[] = {(void**)&ctx->fs_y, (void**)&ctx->fs_logq, (void**)&ctx->fs_p, (void**)&ctx->fs_x,
                     (void**)&ctx->fs_wfj, (void**)&ctx->fs_w};
    for (void** q : ptrs) {
        if (*q) MSX_HIP(ctx, hipFree(*q), "hipFree");
        *q = nullptr;
    }
    ctx->fs_cap = 0;
    int max_dims = dims;
    for (const ChannelMeta& m : ctx->comp.meta) max_dims = std::max(max_dims, m.dims);
    MSX_HIP(ctx, dmalloc(&ctx->fs_y, (size_t)max_dims * n), "flow sample scratch");
    MSX_HIP(ctx, dmalloc(&ctx->fs_logq, (size_t)n), "flow sample scratch");
    MSX_HIP(ctx, dmalloc(&ctx->fs_p, (size_t)4 * ctx->max_np * n), "flow sample scratch");
    MSX_HIP(ctx, dmalloc(&ctx->fs_x, (size_t)2 * n), "flow sample scratch");
    MSX_HIP(ctx, dmalloc(&ctx->fs_wfj, (size_t)n), "flow sample scratch");
    MSX_HIP(ctx, dmalloc(&ctx->fs_w, (size_t)n), "flow sample scratch");
    ctx->fs_cap = n;
    return MSX_OK;
}

// MSX_SAMPLE_USE_FLOW: the fused kernel runs every channel without an
// enabled flow (the call table skips the flow channels' output ranges and
// statistics); each flow channel then samples through msx_flow_sample into
// the context's scratch, whose rows are copied into the caller's layout, and
// its statistics are added by the moments kernel.
msx_status sample_with_flows(msx_ctx* ctx, const int64_t* counts, uint64_t seed, uint64_t stream_id,
                             uint64_t counter_offset, int32_t flags, double* p, double* x1x2, double* w, int32_t* chan,
                             void* stream) {
    const int C = (int)ctx->comp.chans.size();
    SampleCall call;
    std::memset(&call, 0, sizeof call);
    call.n_chan = C;
    call.ept = ctx->ept;
    const int64_t T = (int64_t)sample_block() * ctx->ept;
    int64_t N = 0, tiles = 0;
    bool any_hadronic = false;
    int max_slots = 0, max_inv = 0, kinds = 0;
    for (int c = 0; c < C; ++c) {
        if (counts[c] < 0) return fail(ctx, MSX_ERR_ARG, "negative event count");
        if (counts[c] > INT64_MAX / 4 - N) return fail(ctx, MSX_ERR_ARG, "event count overflow");
        const bool by_flow = ctx->flow[c] && ctx->flow_on[c];
        call.ev_start[c] = N;
        call.tile_start[c] = tiles;
        N += counts[c];
        if (counts[c] > 0) any_hadronic = any_hadronic || ctx->comp.meta[c].hadronic;
        if (by_flow) {
            call.skip_mask |= 1ull << c;
        } else {
            tiles += (counts[c] + T - 1) / T;
            if (counts[c] > 0) {
                max_slots = std::max(max_slots, ctx->comp.chans[c].n_slots);
                max_inv = std::max(max_inv, ctx->comp.chans[c].n_inv);
                kinds |= ctx->comp.chans[c].kinds;
            }
        }
    }
    call.ev_start[C] = N;
    call.tile_start[C] = tiles;
    call.n_tiles = tiles;
    if (N == 0) return MSX_OK;
    if (counter_offset > UINT64_MAX - (uint64_t)N) return fail(ctx, MSX_ERR_ARG, "event ids overflow the counter");
    if (!p || !w) return fail(ctx, MSX_ERR_ARG, "p and w are required");
    if (any_hadronic && !x1x2) return fail(ctx, MSX_ERR_ARG, "x1x2 is required when a sampled channel is hadronic");
    if (msx_status st = check_sample_flags(ctx, flags, max_slots, max_inv)) return st;
    bool any_flow = false;
    for (int c = 0; c < C; ++c) any_flow = any_flow || (counts[c] > 0 && (call.skip_mask >> c & 1));
    if (!any_flow) return fail(ctx, MSX_ERR_STATE, "MSX_SAMPLE_USE_FLOW: no sampled channel has an enabled flow");
    const bool acc = (flags & MSX_SAMPLE_ACCUMULATE_VEGAS) != 0;
    if (msx_status st = set_device(ctx)) return st;
    hipStream_t s = (hipStream_t)stream;
    if (tiles > 0) {
        if (msx_status st = ensure_tiles(ctx, tiles)) return st;
        if (acc)
            if (msx_status st = ensure_vtiles(ctx, tiles)) return st;
        MSX_HIP(ctx, launch_set_call(call, ctx->d_call, s), "sample call table");
        const int grid = (int)std::min<int64_t>(tiles, sample_grid(ctx));
        MSX_HIP(ctx,
                launch_sample(ctx->d_chans, ctx->d_procs, ctx->d_grids, ctx->d_grid_off, ctx->d_chan_nb, ctx->d_call,
                              C, max_slots, max_inv, kinds, ctx->mixed, ctx->lds_max, seed, stream_id, nullptr,
                              counter_offset, ctx->max_np, N, p, x1x2, w, chan, ctx->d_tile, ctx->d_stats, grid, s,
                              acc ? ctx->d_vtiles : nullptr, ctx->vstride, ctx->d_hist_off, ctx->hist_total,
                              ctx->d_hist, jit_of(ctx)),
                "sample launch");
    }
    for (int c = 0; c < C; ++c) {
        const int64_t n = counts[c];
        if (n == 0 || !(call.skip_mask >> c & 1)) continue;
        const ChannelMeta& m = ctx->comp.meta[c];
        const int64_t off = call.ev_start[c];
        if (msx_status st = ensure_flow_scratch(ctx, n, m.dims)) return st;
        if (msx_flow_sample(ctx->flow[c], ctx, c, n, seed, stream_id, counter_offset + (uint64_t)off, ctx->fs_y,
                            ctx->fs_logq, ctx->fs_p, m.hadronic ? ctx->fs_x : nullptr, ctx->fs_wfj, ctx->fs_w,
                            stream) != MSX_OK)
            return fail(ctx, MSX_ERR_DEVICE, std::string("flow sample: ") + msx_flow_last_error(ctx->flow[c]));
        const size_t row = sizeof(double) * (size_t)n;
        for (int comp = 0; comp < 4; ++comp)
            MSX_HIP(ctx,
                    hipMemcpy2DAsync(p + ((size_t)comp * ctx->max_np) * N + off, sizeof(double) * N,
                                     ctx->fs_p + (size_t)comp * m.n_momenta * n, row, row, m.n_momenta,
                                     hipMemcpyDeviceToDevice, s),
                    "flow event copy");
        if (m.hadronic)
            MSX_HIP(ctx,
                    hipMemcpy2DAsync(x1x2 + off, sizeof(double) * N, ctx->fs_x, row, row, 2, hipMemcpyDeviceToDevice,
                                     s),
                    "flow event copy");
        MSX_HIP(ctx, hipMemcpyAsync(w + off, ctx->fs_w, row, hipMemcpyDeviceToDevice, s), "flow event copy");
        if (chan) MSX_HIP(ctx, launch_fill_i32(chan + off, n, c, s), "channel ids");
        MSX_HIP(ctx, launch_moments_add(ctx->fs_w, n, ctx->d_mom, ctx->d_stats + 5 * c, s), "flow statistics");
    }
    return MSX_OK;
}

// Philox stream tags of the attach check's samples.
constexpr uint64_t kCheckStreamVegas = 0x4d53584356ull, kCheckStreamFlow = 0x4d53584346ull;

// Relative variance var(w) / mean(w)^2 of n weights on the device (host result).
msx_status rel_variance(msx_ctx* ctx, const double* w, int64_t n, double* d_out, double* out, hipStream_t s) {
    MSX_HIP(ctx, hipMemsetAsync(d_out, 0, sizeof(double) * 5, s), "moments clear");
    MSX_HIP(ctx, launch_moments_add(w, n, ctx->d_mom, d_out, s), "moments");
    double h[5];
    MSX_HIP(ctx, hipMemcpyAsync(h, d_out, sizeof h, hipMemcpyDeviceToHost, s), "moments copy");
    MSX_HIP(ctx, hipStreamSynchronize(s), "moments sync");
    const double mean = h[0] / n;
    *out = mean != 0.0 ? std::max(h[1] / n - mean * mean, 0.0) / (mean * mean) : INFINITY;
    return MSX_OK;
}

// Serialised context state: this header, dims[C] and bins[C] (int32), the
// grids (grid_total doubles), the VEGAS histograms (hist_total), the
// statistics (5 C), then per attached flow (int32 channel, int32 enabled,
// int64 bytes, the flow's own state).
struct CtxStateHeader {
    char magic[8];  // "MSXSTAT1"
    int32_t n_channels, ept, grid, n_flows;
    int64_t grid_total, hist_total;
    uint64_t next_counter;
    int64_t pad;
};
constexpr char kCtxMagic[8] = {'M', 'S', 'X', 'S', 'T', 'A', 'T', '1'};

}  // namespace

extern "C" {

msx_status msx_get_state(msx_ctx* ctx, void* buf, size_t* size) {
    if (bad_ctx(ctx)) return fail(nullptr, MSX_ERR_ARG, "ctx is NULL");
    if (!size) return fail(ctx, MSX_ERR_ARG, "size is NULL");
    const int C = (int)ctx->comp.chans.size();
    size_t need = sizeof(CtxStateHeader) + sizeof(int32_t) * 2 * C +
                  sizeof(double) * (size_t)(ctx->grid_total + ctx->hist_total + 5 * C);
    std::vector<size_t> fbytes(C, 0);
    int n_flows = 0;
    for (int c = 0; c < C; ++c) {
        if (!ctx->flow[c]) continue;
        if (msx_flow_get_state(ctx->flow[c], nullptr, &fbytes[c]) != MSX_OK)
            return fail(ctx, MSX_ERR_ARG, std::string("flow state: ") + msx_flow_last_error(ctx->flow[c]));
        need += 2 * sizeof(int32_t) + sizeof(int64_t) + fbytes[c];
        ++n_flows;
    }
    if (!buf) {
        *size = need;
        return MSX_OK;
    }
    if (*size < need) return fail(ctx, MSX_ERR_ARG, "state buffer too small");
    if (msx_status st = set_device(ctx)) return st;
    MSX_HIP(ctx, hipDeviceSynchronize(), "sync");
    char* b = (char*)buf;
    CtxStateHeader h{};
    std::memcpy(h.magic, kCtxMagic, 8);
    h.n_channels = C;
    h.ept = ctx->ept;
    h.grid = ctx->grid;
    h.n_flows = n_flows;
    h.grid_total = ctx->grid_total;
    h.hist_total = ctx->hist_total;
    h.next_counter = ctx->next_counter;
    std::memcpy(b, &h, sizeof h);
    b += sizeof h;
    for (int c = 0; c < C; ++c) {
        const int32_t v[2] = {ctx->comp.meta[c].dims, ctx->comp.meta[c].nbins};
        std::memcpy(b + sizeof(int32_t) * c, &v[0], sizeof(int32_t));
        std::memcpy(b + sizeof(int32_t) * (C + c), &v[1], sizeof(int32_t));
    }
    b += sizeof(int32_t) * 2 * C;
    MSX_HIP(ctx, hipMemcpy(b, ctx->d_grids, sizeof(double) * ctx->grid_total, hipMemcpyDeviceToHost), "state copy");
    b += sizeof(double) * ctx->grid_total;
    MSX_HIP(ctx, hipMemcpy(b, ctx->d_hist, sizeof(double) * ctx->hist_total, hipMemcpyDeviceToHost), "state copy");
    b += sizeof(double) * ctx->hist_total;
    MSX_HIP(ctx, hipMemcpy(b, ctx->d_stats, sizeof(double) * 5 * C, hipMemcpyDeviceToHost), "state copy");
    b += sizeof(double) * 5 * C;
    for (int c = 0; c < C; ++c) {
        if (!ctx->flow[c]) continue;
        const int32_t hc[2] = {c, ctx->flow_on[c]};
        const int64_t nb = (int64_t)fbytes[c];
        std::memcpy(b, hc, sizeof hc);
        b += sizeof hc;
        std::memcpy(b, &nb, sizeof nb);
        b += sizeof nb;
        size_t got = fbytes[c];
        if (msx_flow_get_state(ctx->flow[c], b, &got) != MSX_OK)
            return fail(ctx, MSX_ERR_DEVICE, std::string("flow state: ") + msx_flow_last_error(ctx->flow[c]));
        b += fbytes[c];
    }
    *size = need;
    return MSX_OK;
}

msx_status msx_set_state(msx_ctx* ctx, const void* buf, size_t size) {
    if (bad_ctx(ctx)) return fail(nullptr, MSX_ERR_ARG, "ctx is NULL");
    if (!buf || size < sizeof(CtxStateHeader)) return fail(ctx, MSX_ERR_ARG, "state buffer too small");
    const int C = (int)ctx->comp.chans.size();
    const char* b = (const char*)buf;
    const char* end = b + size;
    CtxStateHeader h;
    std::memcpy(&h, b, sizeof h);
    b += sizeof h;
    if (std::memcmp(h.magic, kCtxMagic, 8) != 0) return fail(ctx, MSX_ERR_STATE, "not a context state");
    if (h.n_channels != C || h.grid_total != ctx->grid_total || h.hist_total != ctx->hist_total)
        return fail(ctx, MSX_ERR_STATE, "state of a different process description");
    if (h.ept < 1 || h.ept > 64 || h.grid < 0 || h.grid > (1 << 20) || h.n_flows < 0 || h.n_flows > C)
        return fail(ctx, MSX_ERR_STATE, "corrupt state header");
    const size_t fixed = sizeof(int32_t) * 2 * C + sizeof(double) * (size_t)(h.grid_total + h.hist_total + 5 * C);
    if ((size_t)(end - b) < fixed) return fail(ctx, MSX_ERR_STATE, "truncated state");
    for (int c = 0; c < C; ++c) {
        int32_t d, nb;
        std::memcpy(&d, b + sizeof(int32_t) * c, sizeof d);
        std::memcpy(&nb, b + sizeof(int32_t) * (C + c), sizeof nb);
        if (d != ctx->comp.meta[c].dims || nb != ctx->comp.meta[c].nbins)
            return fail(ctx, MSX_ERR_STATE, "state of a different process description");
    }
    b += sizeof(int32_t) * 2 * C;
    const double* grids = (const double*)b;
    std::vector<double> g(grids, grids + h.grid_total);
    for (int c = 0; c < C; ++c) {
        const ChannelMeta& m = ctx->comp.meta[c];
        for (int k = 0; k < m.dims; ++k) {
            const double* e = g.data() + ctx->grid_off[c] + (size_t)k * (m.nbins + 1);
            if (e[0] != 0.0 || e[m.nbins] != 1.0) return fail(ctx, MSX_ERR_STATE, "grid edges must run from 0 to 1");
            for (int i = 0; i < m.nbins; ++i)
                if (!(e[i + 1] > e[i])) return fail(ctx, MSX_ERR_STATE, "grid edges must increase strictly");
        }
    }
    b += sizeof(double) * h.grid_total;
    const char* hist = b;
    b += sizeof(double) * h.hist_total;
    const char* stats = b;
    b += sizeof(double) * 5 * C;
    // flows: each must be attached to the same channel of this context
    struct FlowRec {
        int c, on;
        const char* blob;
        size_t bytes;
    };
    std::vector<FlowRec> fr;
    for (int i = 0; i < h.n_flows; ++i) {
        if ((size_t)(end - b) < 2 * sizeof(int32_t) + sizeof(int64_t)) return fail(ctx, MSX_ERR_STATE, "truncated state");
        int32_t hc[2];
        int64_t nb;
        std::memcpy(hc, b, sizeof hc);
        b += sizeof hc;
        std::memcpy(&nb, b, sizeof nb);
        b += sizeof nb;
        if (hc[0] < 0 || hc[0] >= C || nb < 0 || (size_t)(end - b) < (size_t)nb)
            return fail(ctx, MSX_ERR_STATE, "corrupt flow record");
        if (!ctx->flow[hc[0]]) return fail(ctx, MSX_ERR_STATE, "the state holds a flow for a channel without one");
        fr.push_back({hc[0], hc[1] ? 1 : 0, b, (size_t)nb});
        b += nb;
    }
    if (b != end) return fail(ctx, MSX_ERR_STATE, "state size mismatch");
    if (msx_status st = set_device(ctx)) return st;
    MSX_HIP(ctx, hipDeviceSynchronize(), "sync");
    for (const FlowRec& f : fr)
        if (msx_flow_set_state(ctx->flow[f.c], f.blob, f.bytes) != MSX_OK)
            return fail(ctx, MSX_ERR_STATE, std::string("flow state: ") + msx_flow_last_error(ctx->flow[f.c]));
    MSX_HIP(ctx, hipMemcpy(ctx->d_grids, g.data(), sizeof(double) * h.grid_total, hipMemcpyHostToDevice), "state copy");
    MSX_HIP(ctx, hipMemcpy(ctx->d_hist, hist, sizeof(double) * h.hist_total, hipMemcpyHostToDevice), "state copy");
    MSX_HIP(ctx, hipMemcpy(ctx->d_stats, stats, sizeof(double) * 5 * C, hipMemcpyHostToDevice), "state copy");
    for (const FlowRec& f : fr) ctx->flow_on[f.c] = f.on;
    ctx->ept = h.ept;
    ctx->grid = h.grid;
    ctx->next_counter = h.next_counter;
    return MSX_OK;
}

msx_status msx_attach_flow(msx_ctx* ctx, int32_t channel, msx_flow* flow, int64_t n_check, uint64_t seed,
                           int32_t* enabled, double* rel_var) {
    if (bad_ctx(ctx)) return fail(nullptr, MSX_ERR_ARG, "ctx is NULL");
    if (msx_status st = check_channel(ctx, channel)) return st;
    if (enabled) *enabled = 0;
    if (!flow) {
        ctx->flow[channel] = nullptr;
        ctx->flow_on[channel] = 0;
        return MSX_OK;
    }
    const ChannelMeta& m = ctx->comp.meta[channel];
    int32_t fd = 0;
    if (msx_flow_dims(flow, &fd) != MSX_OK || fd != m.dims)
        return fail(ctx, MSX_ERR_ARG, "the flow's dimension differs from the channel's");
    if (n_check < 0) return fail(ctx, MSX_ERR_ARG, "n_check < 0");
    int on = 1;
    double rv[2] = {NAN, NAN};
    if (n_check > 0) {
        // the fallback decision: relative weight variance of n_check events
        // drawn through the VEGAS grid alone and through the flow (same
        // channel, fixed stream tags); the flow is enabled only if lower
        if (msx_status st = set_device(ctx)) return st;
        if (msx_status st = ensure_flow_scratch(ctx, n_check, m.dims)) return st;
        hipStream_t s = nullptr;
        MSX_HIP(ctx, hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "check stream");
        double *d_out = nullptr, *y = nullptr;
        msx_status st = MSX_OK;
        hipError_t e = dmalloc(&d_out, 5);
        if (e == hipSuccess) e = dmalloc(&y, (size_t)m.dims * n_check);
        if (e != hipSuccess) st = dev_fail(ctx, e, "check buffers");
        if (st == MSX_OK) st = msx_uniform(ctx, seed, kCheckStreamVegas, 0, n_check, m.dims, y, s);
        if (st == MSX_OK)
            st = msx_map(ctx, channel, n_check, y, ctx->fs_p, m.hadronic ? ctx->fs_x : nullptr, ctx->fs_wfj,
                         ctx->fs_w, s);
        if (st == MSX_OK) st = rel_variance(ctx, ctx->fs_w, n_check, d_out, &rv[0], s);
        if (st == MSX_OK &&
            msx_flow_sample(flow, ctx, channel, n_check, seed, kCheckStreamFlow, 0, ctx->fs_y, ctx->fs_logq,
                            ctx->fs_p, m.hadronic ? ctx->fs_x : nullptr, ctx->fs_wfj, ctx->fs_w, s) != MSX_OK)
            st = fail(ctx, MSX_ERR_DEVICE, std::string("flow sample: ") + msx_flow_last_error(flow));
        if (st == MSX_OK) st = rel_variance(ctx, ctx->fs_w, n_check, d_out, &rv[1], s);
        if (d_out) (void)hipFree(d_out);
        if (y) (void)hipFree(y);
        (void)hipStreamDestroy(s);
        if (st != MSX_OK) return st;
        on = rv[1] < rv[0] ? 1 : 0;
    }
    ctx->flow[channel] = flow;
    ctx->flow_on[channel] = on;
    if (enabled) *enabled = on;
    if (rel_var) {
        rel_var[0] = rv[0];
        rel_var[1] = rv[1];
    }
    return MSX_OK;
}

}  // extern "C"
