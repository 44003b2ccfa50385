/*
 * msx.h -- C ABI of the MI355X (gfx950) phase-space sampling library.
 *
 * The library turns batches of uniform random numbers into collider-event
 * momenta and importance weights, following the phase-space generator of
 * Heimel, Mattelaer and Winterhalder, "MadSpace -- Event Generation for the
 * Era of GPUs and ML" (arXiv:2602.06895):
 *
 *   VEGAS grid lookup -> multichannel selection -> chain of phase-space
 *   mappings (section 2.2) -> Jacobian product -> integrand x channel weight.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every function returns an msx_status and never throws or aborts.
 *    Argument and shape errors return MSX_ERR_ARG synchronously, before any
 *    work is enqueued; msx_last_error() then holds a message.
 *  - Event buffers are DEVICE pointers owned by the caller (the paper's
 *    zero-copy tensor sharing, section 3.2.7); the context owns its channel
 *    tables, VEGAS grids, statistics and scratch, and msx_destroy frees them.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream) and
 *    the call returns without waiting, except where a function says it
 *    synchronises.  A context is not thread-safe; use one per host thread.
 *  - Layout is structure-of-arrays with the event index fastest:
 *      y     [d][n]               uniforms in (0,1), before VEGAS
 *      p     [4][np][n]           (E, px, py, pz) of np = n_final + 2 momenta:
 *                                 incoming a, b first, then final-state
 *                                 particles by label; lab frame
 *      x1x2  [2][n]               momentum fractions (hadronic beams only)
 *      jac / w / alpha [n]        double
 *      chan  [n]                  int32 channel index (msx_sample)
 *  - Per-event physics failures are not errors: such events get weight 0
 *    (the paper's technical cut, operation cut_unphysical).
 *
 * Process description (msx_create_channels): a JSON object, or an object
 * {"processes": [...]} holding several, each with
 *   "sqrt_s"      collider energy in GeV
 *   "beams"       "hadronic" (s-hat sampled, PDF convolution, section 2.2.2)
 *                 or "fixed" (s-hat = sqrt_s^2, no x1/x2)
 *   "shat_min"    lower bound of s-hat in GeV^2 (hadronic)
 *   "masses"      outgoing masses; particles are labelled 1..n
 *   "nu"          default power-law exponent (section 2.2.1), "regulator" a
 *                 (auxiliary mass^2 -a used for massless structures)
 *   "vegas_bins"  bins per VEGAS dimension
 *   "integrand"   toy integrand: "pdf": [a, b] for x^a (1-x)^b on both
 *                 momentum fractions; "pt_min"; "ang": k for 1 + cos^2 of
 *                 particle k (fixed beams); "props": list of
 *                 {"t": bool, "particles": [...], "bw": bool, "m", "w", "mu"}
 *                 factors 1/(|q^2| + mu^2) or 1/((q^2 - m^2)^2 + m^2 w^2)
 *                 with q = p_a - sum p_k (t) or sum p_k (s)
 *   "alpha_mu"    present: local multichannel weights alpha_c(x) from the
 *                 channels' propagator denominators (section 2.1.1); absent:
 *                 alpha = 1
 *   "channels"    diagram topologies:
 *                   {"t_chain": [leg...], "t_order": "AB.."}  legs along the
 *                   t-channel spine from incoming a to b, and for each of the
 *                   first kappa-1 generation steps whether the next leg is
 *                   peeled from the A or the B side (section 2.2.8);
 *                   with "st": true every block after the first is the
 *                   (s~, t) double-invariant block (section 2.2.5): its
 *                   r_phi gives s~ = (p1 + the leg the previous block
 *                   peeled)^2, uniform between its bounds, on the half of
 *                   the azimuth its half of [0, 1) selects;
 *                   {"s": cluster}  pure s-channel;
 *                   {"chili": true}  a Chili channel (section 2.4, hadronic
 *                   beams only): per particle but the last p_T (1/p_T^2
 *                   above the integrand's "pt_min", else the regulated map
 *                   with lambda = its mass or 1), rapidity and azimuth in
 *                   the lab frame, then the last one's rapidity: 3 n - 2
 *                   dimensions in that order; x1, x2 follow from the
 *                   momenta.  It has no propagators: under "alpha_mu" it
 *                   takes the constant weight 1 / (channels of the
 *                   process); msx_inverse_map recovers its uniforms from
 *                   the lab-frame p_T, rapidities and relative azimuths.
 *                 A leg is a particle label or a cluster
 *                 {"d": [child, child], "m", "w", "nu", "order", "rambo"};
 *                 "d" with three children makes a 1 -> 3 decay (section
 *                 2.2.6: dimensions E1, E2, phi, theta, beta);
 *                 "rambo": true samples the cluster's mass with the
 *                 FastRambo map of its particle count (section 2.2.9).
 * Random-number dimensions of a tree channel, in order: s-hat (hadronic), the
 * cluster invariants in sampling order, the kappa-1 t-channel invariants,
 * x1 (hadronic), (r_phi, r_t) per 2->2 block, (r_phi, r_theta) per decay
 * (five numbers per 1 -> 3 decay) in depth-first order -- the order of the paper's compute-graph example
 * (section 3.2.1).
 */
#ifndef MSX_H
#define MSX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MSX_OK = 0,
    MSX_ERR_ARG = 1,         /* invalid argument, size or description */
    MSX_ERR_DEVICE = 2,      /* a HIP runtime call failed */
    MSX_ERR_OOM = 3,         /* device allocation failed */
    MSX_ERR_UNSUPPORTED = 4, /* valid request beyond this build's limits */
    MSX_ERR_STATE = 5        /* call not valid in the context's state */
} msx_status;

typedef struct msx_ctx msx_ctx;

/* Arithmetic of the mapping chain (msx_create_channels `precision`).
 *  MSX_FP64:  every step in FP64.
 *  MSX_MIXED: the well-conditioned transcendentals of the chain -- the power
 *             laws of the G_nu maps (eq. prop_stable_nu; their endpoint
 *             difference through log1p / expm1 of the FP64 range ratio), the
 *             exp/log of the log maps, the azimuth sines and cosines of the
 *             2->2 blocks and decays, the toy-PDF powers -- in FP32.  Kallen
 *             functions, x - m^2, the t range, the s-channel mass bounds,
 *             square roots of invariants, the momentum fractions x1, x2 (eq.
 *             pdf_sampling; the PDFs take 1 - x), the Breit-Wigner map (eq.
 *             prop_massive), every boost and the Jacobian product stay FP64.
 *             Output layout and types are the same as for MSX_FP64. */
enum { MSX_FP64 = 0, MSX_MIXED = 1 };

/* Metadata keys for msx_get_meta (integer keys, in the spirit of the UMAMI
 * interface of section 3.3). `index` selects a channel where noted. */
enum {
    MSX_META_N_CHANNELS = 0,   /* number of channels (all processes) */
    MSX_META_DIMS = 1,         /* random dimensions of channel `index` */
    MSX_META_N_MOMENTA = 2,    /* np = n_final + 2 of channel `index` */
    MSX_META_HADRONIC = 3,     /* 1 if channel `index` has x1/x2 */
    MSX_META_VEGAS_BINS = 4,   /* bins per dimension of channel `index` */
    MSX_META_MAX_MOMENTA = 5,  /* largest np over all channels */
    MSX_META_PROCESS = 6,      /* process index of channel `index` */
    MSX_META_DEVICE = 7,       /* HIP device ordinal of the context */
    MSX_META_PRECISION = 8,    /* MSX_FP64 or MSX_MIXED */
    MSX_META_EVENTS_PER_THREAD = 9, /* sample launch shape: events per thread per tile */
    MSX_META_GRID = 10,        /* sample launch shape: workgroups of the persistent grid */
    MSX_META_COUNTER = 11,     /* next event id of MSX_COUNTER_AUTO sample calls */
    MSX_META_FLOW = 12,        /* channel `index`: 0 no flow attached, 1 attached but VEGAS kept
                                  (the attach check found the flow no better), 2 flow enabled */
    MSX_META_SPECIALIZED = 13  /* kernels msx_specialize built that sample launches use (0: none) */
};

/* Text of the last error on this context (or of the last failed create when
 * ctx is NULL).  Owned by the library; valid until the next call. */
const char* msx_last_error(const msx_ctx* ctx);

/* Parse the process description, compile every channel into its device
 * table (section 2.2: recursive decomposition, s- and t-channel orders),
 * upload tables and uniform VEGAS grids to device `device`.  `precision`
 * is MSX_FP64 or MSX_MIXED (else MSX_ERR_ARG).  On success *out owns all
 * device state. */
msx_status msx_create_channels(const char* process_json, int32_t precision, int32_t device,
                               msx_ctx** out);

/* Free every device and host resource of ctx (NULL is allowed). */
msx_status msx_destroy(msx_ctx* ctx);

msx_status msx_get_meta(const msx_ctx* ctx, int32_t key, int32_t index, int64_t* value);

/* Uniforms of the library's counter-based generator: Philox4x64-10 (Salmon
 * et al., SC'11) with key (seed, stream_id) and counter (e, k/4, 0, 0);
 * y[k][i] for event id e = e0 + i is ((word_{k mod 4} >> 11) + 0.5) 2^-53.
 * msx_sample draws exactly these numbers for event id = counter_offset +
 * output position.  y: device [d][n]; 1 <= d <= 64. */
msx_status msx_uniform(msx_ctx* ctx, uint64_t seed, uint64_t stream_id, uint64_t e0, int64_t n,
                       int32_t d, double* y, void* stream);

/* Forward map of one channel (the parity entry point): y [d][n] uniforms are
 * pushed through the channel's current VEGAS grid and mapping chain.
 * Outputs p [4][np][n] (required), x1x2 [2][n] (required for hadronic
 * beams, must be NULL otherwise), jac [n] (required; 0 for unphysical
 * events), w [n] (optional: also evaluate alpha_c * f * jac, as msx_weight
 * would).  n = 0 is a no-op. */
msx_status msx_map(msx_ctx* ctx, int32_t channel, int64_t n, const double* y, double* p,
                   double* x1x2, double* jac, double* w, void* stream);

/* Inverse map of one channel (section 2.1: every mapping of the chain is
 * invertible): from lab-frame momenta p [4][np][n] (incoming partons first,
 * as msx_map writes them) and x1x2 [2][n] (required for hadronic beams, NULL
 * otherwise), the uniforms y [d][n] (required) that the channel's mapping
 * chain and current VEGAS grid send to them, and jac [n] (optional) = the
 * forward Jacobian at y, so that the channel's density at the event is
 * 1/jac (0 for an event the forward chain would cut).  Steps: the beam boost
 * undone; s-hat = x1 x2 s_lab and x1 = tau^r; each invariant from the
 * momenta of its cluster; per 2->2 block |t| = -(p_A - p_1)^2 and the
 * azimuth of p_1 about p_A in the rest frame of p_A + p_B; per decay the
 * angles of the first child in its parent's rest frame; then each map and
 * the VEGAS grid inverted.  FP64 in both precision modes.  An event that is
 * not in the channel's image (a recovered uniform more than 1e-6 outside
 * [0, 1], e.g. a jet below a Chili channel's p_T cut) gets y = NaN in every
 * dimension and jac = 0: its density in this channel is 0.  n = 0 is a
 * no-op. */
msx_status msx_inverse_map(msx_ctx* ctx, int32_t channel, int64_t n, const double* p, const double* x1x2, double* y,
                           double* jac, void* stream);

/* Global multichannel density of the channels of process `process` (the
 * Kleiss-Pittau form of the multichannel method, section 2.1):
 *   g(p) = sum_c alpha[c] / J_c(y_c(p)),
 * with y_c(p) the channel's inverse map and J_c its forward Jacobian there
 * (msx_inverse_map), over the process's channels in context order; alpha
 * (host, one entry >= 0 per channel of the process) are the a-priori channel
 * weights.  An event that channel c's chain cuts contributes 0.  The
 * multichannel weight of an event is then f(p) / g(p).  p [4][np][n],
 * x1x2 [2][n] (hadronic) and g [n] are device arrays.  Uses a context-owned
 * scratch of (max dims + 1) n doubles (grown on demand: a call that grows it
 * synchronizes the device).  n = 0 is a no-op. */
msx_status msx_multichannel_density(msx_ctx* ctx, int32_t process, int64_t n, const double* p, const double* x1x2,
                                    const double* alpha, double* g, void* stream);

/* Event weight w = alpha_c(x) f(x) jac from momenta p [4][np][n] (lab frame,
 * as written by msx_map), x1x2 (hadronic) and jac; alpha [n] optional. */
msx_status msx_weight(msx_ctx* ctx, int32_t channel, int64_t n, const double* p,
                      const double* x1x2, const double* jac, double* w, double* alpha,
                      void* stream);

/* counter_offset value of msx_sample / msx_sample_noalloc that takes the
 * context's running event counter (MSX_META_COUNTER, saved by msx_get_state)
 * as the first event id and advances it by the events of the call, so that
 * successive calls draw disjoint events without the caller tracking ids. */
#define MSX_COUNTER_AUTO UINT64_MAX

/* Flags of the sample calls.
 *  MSX_SAMPLE_ACCUMULATE_VEGAS: the fused kernel also adds, per channel,
 *    sum w^2 per VEGAS bin of every dimension (bin of the event's uniform
 *    under the current grid) into the context's histograms, which
 *    msx_vegas_update consumes (the adaptation phase of section 4.2: adapt
 *    the grids, then freeze them).  Each wave keeps a private histogram in
 *    LDS, every tile writes the sum of its waves' histograms, and a second
 *    kernel adds the tiles in order, so the sums are deterministic for a
 *    given events-per-thread setting.  Needs (4 dims bins + 1024) doubles of
 *    LDS beside the kernel's own; MSX_ERR_UNSUPPORTED beyond 160 KiB (then
 *    use msx_vegas_accumulate).
 *  MSX_SAMPLE_USE_FLOW: channels with a flow attached (msx_attach_flow) draw
 *    their uniforms from the flow (msx_flow_sample) instead of the VEGAS grid
 *    alone; the other channels run the fused kernel.  Host counts only
 *    (msx_sample); those channels' events are not VEGAS-accumulated.
 *  MSX_SAMPLE_ADVANCE_COUNTER: device-count launches only
 *    (msx_sample_device, msx_sample_graph_create): after the sample the
 *    library adds the call's total event count to *counter_offset (which it
 *    then writes, despite the const), so that every replay of a captured
 *    graph draws new events. */
enum { MSX_SAMPLE_ACCUMULATE_VEGAS = 1, MSX_SAMPLE_USE_FLOW = 2, MSX_SAMPLE_ADVANCE_COUNTER = 4 };

/* Fused production path, all channels in one launch: for channel c,
 * counts[c] events (host array of n_channels entries) are generated at
 * output positions [off_c, off_c + counts[c]) with off_c = sum of earlier
 * counts: Philox uniforms -> VEGAS -> mapping chain -> weight.  Outputs:
 * p [4][npmax][N] (rows beyond a channel's np untouched), x1x2 [2][N] (or
 * NULL when no channel is hadronic), w [N], chan [N] (optional), with
 * N = sum counts.  Per-channel statistics are added to the context's
 * accumulators (msx_stats).  Results do not depend on launch shapes.
 * flags: MSX_SAMPLE_* (0 for a plain sample). */
msx_status msx_sample(msx_ctx* ctx, const int64_t* counts, uint64_t seed, uint64_t stream_id,
                      uint64_t counter_offset, int32_t flags, double* p, double* x1x2, double* w,
                      int32_t* chan, void* stream);

/* msx_sample for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same events, weights, channel ids and statistics as msx_sample with flags 0
 * (bit-identical for the same launch shape), but the per-tile statistics of
 * the launch live in a fixed device array of the library (4 doubles x 2^17
 * tiles = 4 MiB, one copy per GPU, held until the process ends) instead of
 * context scratch grown on demand, and the call allocates nothing.  The
 * tiles of a call (sum over channels of ceil(counts[c] / (256 x events per
 * thread))) must not exceed 2^17: larger calls fail with MSX_ERR_ARG before
 * any launch.  All contexts on one GPU share the array: calls that overlap in
 * time on one GPU (different streams, or different host threads) race on it
 * and give wrong statistics; calls ordered on one stream do not. */
msx_status msx_sample_noalloc(msx_ctx* ctx, const int64_t* counts, uint64_t seed, uint64_t stream_id,
                              uint64_t counter_offset, double* p, double* x1x2, double* w, int32_t* chan,
                              void* stream);

/* msx_sample with its parameters in device memory, for launches captured in
 * a HIP graph and replayed with new values: counts [n_channels] (int64) and
 * counter_offset (one uint64) are read by the device when the launch runs.
 * Outputs have room for `capacity` events: p [4][max_np][capacity], x1x2
 * [2][capacity] (required if any channel is hadronic), w, chan [capacity];
 * events fill positions 0 .. sum(counts) - 1.  If a count is negative or the
 * total exceeds capacity, nothing is sampled and *status (device int32,
 * optional) is set to 1, else 0.  The channel lookup and register class cover
 * all channels of the context.  Statistics accumulate as for msx_sample.  The
 * first call allocates scratch sized for `capacity`; capture it only after a
 * call of the same capacity (msx_sample_graph_create does this itself). */
msx_status msx_sample_device(msx_ctx* ctx, const int64_t* counts, uint64_t seed, uint64_t stream_id,
                             const uint64_t* counter_offset, int64_t capacity, int32_t flags, double* p,
                             double* x1x2, double* w, int32_t* chan, int32_t* status, void* stream);

/* A captured, instantiated HIP graph of one msx_sample_device launch (the
 * persistent fused kernel of all channels plus its statistics pass).  Launch
 * it any number of times after writing new counts / counter offset to the
 * device buffers it was created with; those buffers and the context must
 * outlive the graph.  The graph owns its call table and tile scratch; it
 * adds to the context's statistics, so launches that overlap with other
 * sample calls of the same context race on them. */
typedef struct msx_graph msx_graph;
msx_status msx_sample_graph_create(msx_ctx* ctx, const int64_t* counts, uint64_t seed, uint64_t stream_id,
                                   const uint64_t* counter_offset, int64_t capacity, int32_t flags,
                                   double* p, double* x1x2, double* w, int32_t* chan, int32_t* status,
                                   msx_graph** out);
msx_status msx_graph_launch(msx_graph* graph, void* stream);
msx_status msx_graph_destroy(msx_graph* graph);

/* Launch shape of the fused sample kernel: events per thread per tile (1..64)
 * and workgroups of the persistent grid (0: 8 per compute unit).  Per-event
 * results are independent of the shape; per-channel statistics are summed in
 * a shape-dependent order. */
msx_status msx_set_launch(msx_ctx* ctx, int32_t events_per_thread, int32_t grid);

/* Time msx_sample on `counts` (host) for each candidate launch shape
 * (events per thread 1, 2, 4; 2, 4, 8, 16 workgroups per compute unit),
 * `reps` timed launches each, and keep the fastest (msx_set_launch).  Uses
 * its own output scratch; the context's statistics are left unchanged.
 * Synchronises the device.  *best_ms (optional) gets the time per launch. */
msx_status msx_autotune(msx_ctx* ctx, const int64_t* counts, uint64_t seed, int32_t reps, double* best_ms);

/* Channel-specialised fused sample (the per-event chain of section 2.2 with
 * the integrand and channel weight of eq. multi-channel-mg, as msx_sample).
 * on != 0: compiles, with the HIP run-time compiler for the context's
 * device, versions of the fused sample kernel in which this context's
 * channel and process tables are compile-time constants (the map kinds,
 * operation counts and momentum slots of every channel fixed in the code),
 * loads them, and from then on every sample launch of the context uses
 * them: msx_sample, msx_sample_device, msx_sample_noalloc and graphs
 * captured afterwards.  Channels are compiled in groups of at most eight
 * consecutive channels, one kernel each, launched one after the other in
 * the same stream (a group whose kernel would spill registers is split).
 * Results are bit-identical to the default kernel's in MSX_FP64 (same
 * source, no floating-point contraction in either) and differ by FP32
 * roundings in MSX_MIXED; the kernels run fewer instructions with fewer
 * registers.  The first call compiles on the host (0.5 s for one t tbar
 * channel, 4 s for eight pp -> 4 jets channels) and synchronises the device;
 * later calls only switch.  on == 0 switches launches back to the default
 * kernel; the compiled ones stay loaded until msx_destroy (graphs captured
 * with them keep working).  MSX_META_SPECIALIZED gives the number of
 * kernels in use (0: the default kernel).  Errors: MSX_ERR_DEVICE with the
 * compiler's log when the run-time compiler or a module load fails;
 * MSX_ERR_UNSUPPORTED when the kernel of a single channel would spill
 * registers to scratch (it would be slower than the default one).  In both
 * cases the context keeps the default kernel. */
msx_status msx_specialize(msx_ctx* ctx, int32_t on);

/* Copy the accumulated per-channel statistics to host out [n_channels][5]:
 * (sum w, sum w^2, n, n with w == 0, max w).  Synchronises `stream`. */
msx_status msx_stats(msx_ctx* ctx, double* out, void* stream);
msx_status msx_reset_stats(msx_ctx* ctx, void* stream);

/* Add sum w^2 per VEGAS bin of channel `channel` from uniforms y [d][n] and
 * weights w [n] into the context's histogram (deterministic order). */
msx_status msx_vegas_accumulate(msx_ctx* ctx, int32_t channel, int64_t n, const double* y,
                                const double* w, void* stream);

/* VEGAS adaptation phase, run by the library: `iterations` times, sample
 * n_per_channel events of every channel with MSX_SAMPLE_ACCUMULATE_VEGAS
 * (seed, stream_id; iteration i uses event ids counter_offset +
 * i n_per_channel n_channels + output position), then msx_vegas_update
 * (alpha).  stats_out [n_channels][5] (host, optional) receives the
 * statistics of the last iteration, whose events were drawn from the grids
 * before the last refinement.  The context's statistics are left reset.
 * Allocates the event buffers of one iteration for the duration of the call;
 * synchronises `stream`. */
msx_status msx_vegas_adapt(msx_ctx* ctx, int64_t n_per_channel, int32_t iterations, double alpha, uint64_t seed,
                           uint64_t stream_id, uint64_t counter_offset, double* stats_out, void* stream);

/* Events per channel for a multichannel sample of `total` events (the
 * allocation of section 3.4.1's per-channel jobs): with sd_c the standard
 * deviation of channel c's weights from stats [n_channels][5] (host, as
 * msx_stats returns them), counts[c] = floor(floor_frac total) +
 * floor(share_c (total - n_channels floor(floor_frac total))), share_c =
 * sd_c / sum sd (equal shares when every sd is 0), and the remainder goes to
 * the channel with the largest share; counts sum to total.  Minimises the
 * variance of sum_c <w>_c (Neyman allocation) above the floor.  Host only
 * (no device work); MSX_ERR_ARG when total < 0, floor_frac outside [0, 1 /
 * n_channels] or a statistic is not finite. */
msx_status msx_allocate_counts(int32_t n_channels, const double* stats, int64_t total, double floor_frac,
                               int64_t* counts);

/* Refine every channel's grid from its accumulated histogram (smoothing,
 * damping exponent `alpha` > 0, equal-share redistribution; VEGAS as cited
 * by the paper for its adaptive grids), then clear the histograms.  Channels
 * with an empty histogram keep their grid. */
msx_status msx_vegas_update(msx_ctx* ctx, double alpha, void* stream);

/* The context's adaptive state as one host blob (checkpoint / resume; the
 * explicit state that section 3.3's interface conventions ask of a
 * component): every channel's VEGAS grid and accumulated histogram, the
 * per-channel statistics, the sample launch shape, the running event counter
 * (MSX_COUNTER_AUTO) and, for every channel with an attached flow, whether it
 * is enabled and the flow's own state (msx_flow_get_state: FP32 parameters,
 * Adam moments and step count).  get: buf NULL sets *size to the bytes
 * needed; otherwise *size must be at least that, and receives it.  set:
 * restores a blob taken from a context of the same process description (same
 * channels, dimensions and bins) whose flows are attached to the same
 * channels, with shapes equal (else MSX_ERR_STATE, nothing changed); grids
 * are validated as msx_set_grid does.  Both synchronise the device.  The
 * layout is host-endian and versioned by its leading 8 bytes ("MSXSTAT1"). */
msx_status msx_get_state(msx_ctx* ctx, void* buf, size_t* size);
msx_status msx_set_state(msx_ctx* ctx, const void* buf, size_t size);

/* Host copies of a channel's grid edges [d][bins+1] (checkpoint/resume and
 * tests).  Both synchronise. set_grid validates monotone edges from 0 to 1. */
msx_status msx_get_grid(msx_ctx* ctx, int32_t channel, double* edges);
msx_status msx_set_grid(msx_ctx* ctx, int32_t channel, const double* edges);

/* Unweighting efficiency of weights w [n] >= 0 (device): the smallest W with
 * sum max(0, w_i - W) <= overweight * sum w_i, and eff = mean(w) / W -- the
 * on-the-fly maximum weight with an overweight allowance of section 3.4.1.
 * Found on the device by six refinement passes over the weights' bit
 * patterns with exact integer bucket sums (the same bits on every call).
 * Results on host; synchronises `stream` once.  Errors: MSX_ERR_ARG for
 * n <= 0, n >= 2^36, a missing pointer, overweight outside (0, 1), or
 * weights without a finite positive sum. */
msx_status msx_unweight_eff(msx_ctx* ctx, const double* w, int64_t n, double overweight,
                            double* eff, double* w_max, void* stream);

/* Observables of lab-frame events (the distributions of the paper's section
 * 4.2: a partonic invariant mass, the transverse momentum of the hardest jet,
 * the separation of the two hardest jets).  An observable is four int32:
 * (kind, set, rank, 0), set a bitmask of final-state particle labels (bit i =
 * particle i, p index i + 2).  Kinds on the summed momentum of the set:
 * MSX_OBS_E energy, MSX_OBS_PT transverse momentum, MSX_OBS_ETA
 * pseudorapidity asinh(p_z / p_T), MSX_OBS_PHI azimuth atan2(p_y, p_x),
 * MSX_OBS_M invariant mass sqrt(max(E^2 - p^2, 0)); on the members of the
 * set ordered by p_T (descending, lower label first on ties):
 * MSX_OBS_PT_RANK the p_T of the rank-th hardest (0 = hardest),
 * MSX_OBS_DR_HARDEST the separation sqrt(d_eta^2 + d_phi^2) of the two
 * hardest (d_phi wrapped into [0, pi]).  */
enum {
    MSX_OBS_E = 0,
    MSX_OBS_PT = 1,
    MSX_OBS_ETA = 2,
    MSX_OBS_PHI = 3,
    MSX_OBS_M = 4,
    MSX_OBS_PT_RANK = 5,
    MSX_OBS_DR_HARDEST = 6
};

/* k (1..8) observables of n events of process `process`: spec [4 k] int32
 * (host), p [4][np][n] (device, lab frame as msx_map / msx_sample write it),
 * out [k][n] (device).  n = 0 is a no-op. */
msx_status msx_observables(msx_ctx* ctx, int32_t process, int64_t n, const double* p, const int32_t* spec, int32_t k,
                           double* out, void* stream);

/* General cut: w[e] := 0 unless lo[j] <= x[j][e] < hi[j] for every j < k
 * (1..8); x [k][n] observables (device, e.g. from msx_observables), lo, hi
 * [k] (host; +-inf for open ends), w [n] (device, in place). */
msx_status msx_cut(msx_ctx* ctx, int64_t n, const double* x, int32_t k, const double* lo, const double* hi, double* w,
                   void* stream);

/* Weighted histogram of x [n] with weights w [n] (device): hist [2][bins]
 * (device) = (sum w, sum w^2) over the events in each of `bins` (1..4096)
 * equal bins of [lo, hi), bin = floor((x - lo) bins / (hi - lo)); events
 * outside [lo, hi) are not counted.  Deterministic (fixed summation order for
 * a given n).  Uses a context-owned scratch of 2 bins ceil(n / 2048) doubles
 * (grown on demand: a call that grows it synchronizes the device). */
msx_status msx_histogram(msx_ctx* ctx, int64_t n, const double* x, const double* w, int32_t bins, double lo, double hi,
                         double* hist, void* stream);

/* Hit-or-miss unweighting of weights w [n] >= 0 (device) against a maximum
 * weight w_max > 0 (section 3.4.1: the channel-wise files are unweighted with
 * the current estimate of the maximum weight, at the end once more with the
 * final one).  Event i is kept when u_i w_max < w_i, with u_i the uniform of
 * event id counter_offset + i under (seed, stream_id) -- dimension 0 of
 * msx_uniform, a stream of its own so that the decision is reproducible.
 * Outputs (device): keep [n] the kept indices in increasing order (first
 * *count entries), uw [n] (optional) their unit weights max(1, w_i / w_max)
 * (above 1 for overweight events), count [1] int64 the number kept.  A
 * second unweighting against a larger final maximum W' takes the effective
 * weights max(w_i, w_max) of the kept events.  Enqueues only (the count stays
 * on the device); a call that grows the context's block scratch synchronizes
 * the device.  n = 0 sets *count = 0. */
msx_status msx_unweight(msx_ctx* ctx, const double* w, int64_t n, double w_max, uint64_t seed, uint64_t stream_id,
                        uint64_t counter_offset, int64_t* keep, double* uw, int64_t* count, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MSX_H */
