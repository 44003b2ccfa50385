"""Throughput of the phase-space hot path on one MI355X.

Headline workload: pp -> t tbar -> b W+ b~ W- -> 6 massless final states at
sqrt(s) = 13 TeV, one channel, 16 random dimensions, Breit-Wigner maps for
the tops (173, 1.5) and Ws (80.4, 2.1), toy PDFs x^-1.2 (1-x)^3, integrand =
the Breit-Wigner propagators, FP64.  VEGAS grids (64 bins x 16 dims) are
adapted first (10 x 1e5 events, inside the fused sample, untimed), then
frozen.  One step = one replay of a captured HIP graph of the fused sample of
1e8 events (in-kernel Philox uniforms -> VEGAS -> mapping chain -> integrand
-> SoA stores and statistics; the graph advances its own event counter, so
every replay draws new events), with inputs (grids, channel tables) already
resident in HBM.  The eight-channel pp -> 4 jets workload (1e7 events per
step) and the other reports are extra keys of the same JSON line.

Prints one JSON line.  --gpus N > 1 is refused: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_EVENTS = 100_000_000
C2_EVENTS = 10_000_000
BYTES_PER_EVENT = 8 * 4 * 8 + 2 * 8 + 8  # pp -> t tbar -> 6: momenta (a, b, 6 final), x1 x2, w
C2_BYTES_PER_EVENT = 6 * 4 * 8 + 2 * 8 + 8 + 4  # momenta (a, b, 4 jets), x1 x2, w, channel id
HBM_PEAK_GBS = 8000.0
# VALU issue: 256 CUs x 4 SIMDs at 2.4 GHz, one wave64 VALU instruction per
# SIMD every 4 cycles (16 lanes per cycle; FP64 FMA is full rate on gfx950)
VALU_PEAK_GINST = 1024 * 2.4 / 4


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(desc, grids, counts, seed, min_seconds=10.0, single_seconds=4.0):
    """The FP64 oracle on the host cores (OpenMP over events), built on this
    host with -O3 -march=native (no FMA contraction, like the reference
    build): every channel in proportion to the GPU counts, repeated until
    min_seconds of wall time on all cores and single_seconds on one core;
    uniform generation is outside the timed region."""
    import tempfile

    import oracle
    import workloads as W

    P = oracle.Process(desc)
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    try:
        tmp = tempfile.mkdtemp(prefix="msx_oracle_")
        variant = oracle.build_timing(tmp)
        build = "-O3 -march=native -ffp-contract=off, built on this host"
    except Exception as exc:  # no compiler on the host: the reference build
        variant, build = "ref", f"-O2 -ffp-contract=off (timing build failed: {exc})"
    frac = counts / counts.sum()
    batch = 200_000
    per = np.maximum(1, np.round(frac * batch)).astype(np.int64)
    ys = [W.philox_uniforms(seed, 0, 0, int(per[c]), P.dims[c]) for c in range(len(per))]

    def run(nt, seconds):
        done, elapsed = 0, 0.0
        while elapsed < seconds:
            t0 = time.perf_counter()
            for c in range(len(per)):
                P.map(c, ys[c], grids[c], nthreads=nt, variant=variant)
            elapsed += time.perf_counter() - t0
            done += int(per.sum())
        return done, elapsed

    done, elapsed = run(threads, min_seconds)
    d1, e1 = run(1, single_seconds)
    return {"value": done / elapsed, "unit": "events/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} events of the same workload ({int(per.sum())} per pass, channels in the "
                      f"GPU's proportions, frozen grids), {elapsed:.1f} s on {threads} threads",
            "single_thread_events_per_s": d1 / e1, "cpu_model": _cpu_model(), "build": build}


# sources of the fused sample kernel (a change invalidates the committed counter figures)
KERNEL_SOURCES = ["paper_2602_06895_amd/csrc/" + f for f in
                  ("chain_kernels.h", "chain.h", "device_util.h", "tables.h", "chain_f64_s.hip", "chain_f64_m.hip",
                   "jit.cpp")] + ["paper_2602_06895_amd/build.py"]
# the fused sample kernel the library compiles for the context's channels
# (msx_specialize); --no-specialize times the class kernel k_sample instead
SPECIALIZE = True
PROFILE = os.path.join(ROOT, "profiles", "msx_jit_sample_ttbar6_1e8.txt")
PROFILE_C2 = os.path.join(ROOT, "profiles", "msx_jit_sample_pp4j_1e7.txt")
PROFILE_CLASS = os.path.join(ROOT, "profiles", "k_sample_ttbar6_1e8.txt")


def make_context(desc, **kw):
    """A context whose sample launches use the specialised kernel (unless
    --no-specialize); returns (context, seconds the run-time compile took)."""
    from paper_2602_06895_amd import Context

    ctx = Context(desc, **kw)
    t0 = time.perf_counter()
    if SPECIALIZE:
        ctx.specialize()
    return ctx, time.perf_counter() - t0


def kernel_source_hash() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled(path=None):
    """Figures of a committed counter summary ('key: value' lines): HBM bytes
    per launch and VALU instructions per event, or None where the kernel
    sources changed since the counters were taken."""
    path = path or PROFILE
    out = {"hbm_bytes_per_event": None, "valu_per_event": None}
    if not os.path.exists(path):
        return out
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != kernel_source_hash():
        return out
    for k in out:
        try:
            out[k] = float(vals[k])
        except (KeyError, ValueError):
            pass
    return out



def roofline(events, bytes_per_event, launch_s, prof):
    """Both roofs of a fused sample launch: HBM (algorithmic bytes / launch
    time against 8 TB/s) and VALU issue (the counted VALU instructions per
    event / launch time against 1024 SIMDs x 2.4 GHz / 4 cycles); `bound`
    names the roof at the larger fraction, whose figures fill the top level."""
    hbm = events * bytes_per_event / launch_s / 1e9
    roofs = {"hbm": {"achieved": hbm, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": hbm / HBM_PEAK_GBS,
                     "bytes_per_event": bytes_per_event}}
    if prof.get("valu_per_event"):
        inst = prof["valu_per_event"] / 64.0 * events / launch_s / 1e9
        roofs["alu"] = {"achieved": inst, "peak": VALU_PEAK_GINST, "unit": "Ginst/s",
                        "frac": inst / VALU_PEAK_GINST, "valu_per_event": prof["valu_per_event"],
                        "note": "wave64 VALU instructions issued per second (SQ_INSTS_VALU)"}
    bound = max(roofs, key=lambda k: roofs[k]["frac"])
    top = roofs[bound]
    tr = prof.get("hbm_bytes_per_event")
    return {"bound": bound, "achieved": top["achieved"], "peak": top["peak"], "unit": top["unit"],
            "frac": top["frac"], "traffic": tr * events if tr is not None else None, "roofs": roofs,
            "avg_launch_ms": launch_s * 1e3}

def graph_steps(ctx, counts, seed, steps, warmup, flags_extra=0, want_chan=False, stream_id=0):
    """Capture the fused sample of `counts` (device counts, a device event
    counter the graph advances itself) and replay it: `warmup` untimed
    replays, then `steps` timed ones bracketed by synchronisations; every
    replay is also bracketed by HIP events on the launch stream.  Statistics
    are reset before the timed replays.  Returns (buffers, wall seconds,
    per-replay milliseconds)."""
    import torch

    from paper_2602_06895_amd import SAMPLE_ADVANCE_COUNTER

    N = int(np.sum(counts))
    buf = ctx.sample_buffers(N, want_chan=want_chan)
    dc = torch.from_numpy(np.asarray(counts, dtype=np.int64)).to(ctx.device)
    off = torch.zeros(1, dtype=torch.int64, device=ctx.device)
    g = ctx.sample_graph(dc, seed, stream_id, off, buf, flags=SAMPLE_ADVANCE_COUNTER | flags_extra)
    stream = torch.cuda.current_stream(ctx.device)
    for _ in range(warmup):
        g.launch()
    ctx.reset_stats()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        ev[i][0].record(stream)
        g.launch()
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = [a.elapsed_time(b) for a, b in ev]
    g.close()
    return buf, wall, ms


def integral_of(stats, steps):
    """Multichannel integral over the timed replays and the relative error
    that one replay's events reach."""
    I, var = 0.0, 0.0
    for s1, s2, n, nz, mx in stats:
        if n <= 1:
            continue
        mean = s1 / n
        I += mean
        var += max(s2 / n - mean * mean, 0.0) / (n - 1)
    return I, (math.sqrt(var * steps) / I if I > 0 else float("nan"))

def _timed(fn, reps):
    """Average milliseconds of fn() over reps launches (HIP events on the
    current stream, after one untimed call)."""
    import torch

    fn()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def mixed_report(n=100_000_000, steps=10, n_err=10_000_000):
    """pp -> t tbar -> 6 (16 dims, Breit-Wigner t and W): FP64 and mixed
    precision fused samples of n events (graph replays, same grids, each
    precision at its own autotuned launch shape), and the
    per-quantity error of mixed results against FP64 ones on the same n_err
    events."""
    import torch

    import workloads as W
    from paper_2602_06895_amd import MIXED, Context, adapt_vegas
    from paper_2602_06895_amd.report import precision_error

    c64, _ = make_context(W.c3_ttbar6())
    adapt_vegas(c64, n_per_channel=100_000, iterations=10, seed=3, stream_id=1)
    grid = c64.get_grid(0)
    counts = np.array([n])
    c64.autotune(counts, seed=1, reps=3)
    _, wall64, ms64 = graph_steps(c64, counts, 77, steps, 2)
    torch.cuda.empty_cache()
    cmx, _ = make_context(W.c3_ttbar6(), precision=MIXED)
    cmx.set_grid(0, grid)
    cmx.autotune(counts, seed=1, reps=3)
    _, wallmx, msmx = graph_steps(cmx, counts, 77, steps, 2)
    torch.cuda.empty_cache()
    ce = np.array([n_err])
    o64 = c64.sample(ce, seed=78, stream_id=0)
    omx = cmx.sample(ce, seed=78, stream_id=0)
    err = precision_error(omx["p"], omx["w"], o64["p"], o64["w"], c64.max_momenta)
    t64, tmx = float(np.median(ms64)), float(np.median(msmx))
    c64.close()
    cmx.close()
    return {"workload": f"pp->ttbar->6 13 TeV, BW t/W, 16 dims, {n} events per graph replay",
            "fp64_events_per_s": n / (t64 / 1e3), "mixed_events_per_s": n / (tmx / 1e3), "speedup": t64 / tmx,
            "median_replay_ms": {"fp64": t64, "mixed": tmx},
            "mixed_error_vs_fp64": dict(err, events=n_err)}

def flow_report(train_steps=400, batch=65536, n_eval=1_000_000, lr=1e-3, workload="c3", channel=0):
    """Learned sampler on one channel: VEGAS adapted and frozen, then an
    8-layer rational-quadratic coupling flow (16 bins, MLP 3 x 128, BF16
    matrix cores) trained on weights the sampler generates; unweighting
    efficiency and relative error of the same number of events with and
    without the flow.  The flow is kept only if its weight variance is below
    VEGAS's.  workload "c3": the pp -> t tbar -> 6 integrand (16 dims);
    "c2": one channel of pp -> 4 jets (10 dims)."""
    import torch

    import workloads as W
    from paper_2602_06895_amd import FLOW_BF16, Context, Flow, adapt_vegas

    desc = W.c3_ttbar6() if workload == "c3" else W.c2_pp4j()
    ctx, _ = make_context(desc)
    adapt_vegas(ctx, n_per_channel=100_000, iterations=10, seed=3, stream_id=1)
    d = ctx.dims[channel]
    counts = np.zeros(ctx.n_channels, dtype=np.int64)
    counts[channel] = n_eval
    ov = ctx.sample(counts, seed=9, stream_id=4)
    wv = ov["w"]
    eff_v, _ = ctx.unweight_eff(wv, 1e-3)
    rel_v = float(wv.std() / wv.mean()) / math.sqrt(n_eval)
    flow = Flow(d, 8, 16, 128, mlp=FLOW_BF16)
    flow.set_params(W.flow_params(31, d, 8, 16, 128))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = []
    for s in range(train_steps):
        o = flow.sample(ctx, channel, batch, seed=10, stream_id=5, counter_offset=s * batch)
        losses.append(flow.train_step(o["y"], o["wfj"], o["logq"], lr))
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    of = flow.sample(ctx, channel, n_eval, seed=11, stream_id=6)
    wf = of["w"]
    eff_f, _ = ctx.unweight_eff(wf, 1e-3)
    rel_f = float(wf.std() / wf.mean()) / math.sqrt(n_eval)
    # matrix-core throughput of the conditioner: one forward pass of 2^20 events
    nf = 1 << 20
    u = torch.rand(d, nf, device="cuda", dtype=torch.float32) * 0.999 + 5e-4
    ms = _timed(lambda: flow.forward(u), 3)
    nh = d // 2
    no = nh * 49
    flops = 2.0 * 8 * (nh * 128 + 2 * 128 * 128 + 128 * no) * nf
    # HBM bytes per event and layer of the fused forward pass (BF16, hidden
    # 128, 16 bins): z read (d floats), the transformed coordinates written,
    # the log-determinant read and written; weights come from L2
    fused = True
    bytes_layer = d * 4 + nh * 4 + 8
    hbm_gbs = 8 * bytes_layer * nf / (ms / 1e3) / 1e9
    # the library's fallback decision (msx_attach_flow): relative weight
    # variances of n_eval events through VEGAS alone and through the flow
    use_flow, (rv_v, rv_f) = ctx.attach_flow(channel, flow, n_check=n_eval, seed=12)
    # time to the relative error VEGAS reaches with the headline's event
    # count: the flow needs target_n rv_f / rv_v events for the same error
    target_n = N_EVENTS
    target = math.sqrt(rv_v / target_n)
    cv = np.zeros(ctx.n_channels, dtype=np.int64)
    cv[channel] = 10_000_000
    ov2 = ctx.sample(cv, seed=13, stream_id=4)
    t_v = _timed(lambda: ctx.sample(cv, seed=13, stream_id=4, out=ov2), 3)
    t_f = _timed(lambda: flow.sample(ctx, channel, n_eval, seed=14, stream_id=7), 3)
    vegas_eps, flow_eps = cv[channel] / (t_v / 1e3), n_eval / (t_f / 1e3)
    n_flow = target_n * rv_f / rv_v
    ttt = {"target_rel_error": target, "target_from": f"VEGAS with {target_n:.0e} events",
           "vegas": {"events": target_n, "events_per_s": vegas_eps, "seconds": target_n / vegas_eps},
           "flow": {"events": n_flow, "events_per_s": flow_eps, "seconds": n_flow / flow_eps},
           "rel_variance": {"vegas": rv_v, "flow": rv_f}}
    del ov2
    ctx.attach_flow(channel, None)
    name = "pp->ttbar->6 integrand" if workload == "c3" else f"pp->4j channel {channel}"
    res = {"workload": f"{name}, {d} dims, VEGAS 10x1e5 then flow {train_steps} x {batch} BF16",
           "vegas": {"unweighting_eff": eff_v, "rel_error": rel_v, "integral": float(wv.mean())},
           "flow": {"unweighting_eff": eff_f, "rel_error": rel_f, "integral": float(wf.mean())},
           "events": n_eval, "eff_ratio_flow_over_vegas": eff_f / eff_v,
           "rel_error_ratio_vegas_over_flow": rel_v / rel_f, "sampler_kept": "flow" if use_flow else "vegas",
           "sampler_decision": "msx_attach_flow (relative weight variance, library side)",
           "time_to_target": ttt,
           "train_seconds": train_s, "loss_first": float(losses[0].cpu()[0]), "loss_last": float(losses[-1].cpu()[0]),
           "flow_forward_2e20": {"ms": ms, "mlp_tflops": flops / (ms / 1e3) / 1e12, "peak_tflops": 2500.0,
                                 "frac": flops / (ms / 1e3) / 1e12 / 2500.0,
                                 "fused_layers": fused, "bound": "mfma" if fused else "hbm",
                                 "algorithmic_bytes_per_event": 8 * bytes_layer, "hbm_gbs": hbm_gbs,
                                 "hbm_frac": hbm_gbs / HBM_PEAK_GBS}}
    flow.close()
    ctx.close()
    return res


def graph_report(steps=20):
    """24-channel batch (C1 and C2 topologies, power-law counts) as one
    persistent launch replayed from a HIP graph after the autotuner, in FP64
    and in mixed precision, through the class kernel and the kernels compiled
    for the 24 channels (groups of at most eight channels, one launch each);
    median of `steps` replays, eager launches beside."""
    import torch

    import workloads as W
    from paper_2602_06895_amd import MIXED, Context, MsxError

    desc, counts = W.c4_context()
    N = int(counts.sum())
    out = {"workload": f"24 channels (6 processes), {N} events, counts power-law 1e3..1e6"}
    for name, prec in (("fp64", 0), ("mixed", MIXED)):
        for kernel in ("class", "specialized"):
            ctx = Context(desc, precision=prec)
            t0 = time.perf_counter()
            if kernel == "specialized":
                try:
                    ctx.specialize()
                except MsxError as e:
                    # a channel whose specialised kernel would spill is refused
                    out[f"{name}_{kernel}"] = {"refused": str(e)}
                    ctx.close()
                    continue
            spec_s = time.perf_counter() - t0
            eager_ms = _timed(lambda: ctx.sample(counts, seed=4, stream_id=8), steps)
            best = ctx.autotune(counts, seed=4, reps=3)
            ept, grid = ctx.launch_shape()
            _, wall, ms = graph_steps(ctx, counts, 4, steps, 3, want_chan=True, stream_id=8)
            med = float(np.median(ms))
            out[f"{name}_{kernel}"] = {"eager_ms": eager_ms, "graph_median_ms": med,
                                       "graph_ms_range": [min(ms), max(ms)], "graph_events_per_s": N / (med / 1e3),
                                       "autotuned": {"events_per_thread": ept, "grid": grid, "ms": best}}
            if kernel == "specialized":
                out[f"{name}_{kernel}"]["specialize_seconds"] = spec_s
                out[f"{name}_{kernel}"]["kernels"] = ctx.specialized_kernels
            ctx.close()
            torch.cuda.empty_cache()
    return out


def inverse_report(n=10_000_000, reps=5, channel=0):
    """Inverse map (momenta -> uniforms and the channel density) of n
    pp -> 4 jets events of one channel: the momenta come from the forward map
    of seeded uniforms (untimed); the timed call is msx_inverse_map (the
    inverse kernel and the store-free Jacobian pass).  Algorithmic bytes per
    event: momenta 6 x 4 x 8 + x1x2 16 read, y 10 x 8 + jac 8 written, y read
    back by the Jacobian pass = 376 B."""
    import torch

    import workloads as W
    from paper_2602_06895_amd import Context

    ctx = Context(W.c2_pp4j())
    d = ctx.dims[channel]
    y = ctx.uniform(7, 9, 0, n, d)
    fwd = ctx.map(channel, y)
    ms = _timed(lambda: ctx.inverse_map(channel, fwd["p"], fwd["x1x2"]), reps)
    inv = ctx.inverse_map(channel, fwd["p"], fwd["x1x2"])
    torch.cuda.synchronize()
    ok = fwd["jac"] > 0
    err = (inv["y"] - y).abs().amax(dim=0)[ok]
    sub = err[:1_000_000].double()
    q = torch.quantile(sub, torch.tensor([0.5, 0.99], dtype=torch.float64, device="cuda")).tolist()
    bpe = 6 * 4 * 8 + 16 + 2 * d * 8 + 8
    ach = n * bpe / (ms / 1e3) / 1e9
    # global multichannel density over all 8 channels (8 inverse maps)
    alpha = np.full(ctx.n_channels, 1.0 / ctx.n_channels)
    ms_g = _timed(lambda: ctx.multichannel_density(0, fwd["p"], fwd["x1x2"], alpha), 2)
    out = {"workload": f"pp->4j channel {channel}, {n} events, momenta -> uniforms + density",
           "events_per_s": n / (ms / 1e3), "ms": ms,
           "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": ach / HBM_PEAK_GBS, "bytes_per_event": bpe},
           "round_trip_err": {"median": q[0], "p99": q[1], "tail_gt_1e-3": float((err > 1e-3).double().mean())},
           "multichannel_density": {"channels": ctx.n_channels, "ms": ms_g, "events_per_s": n / (ms_g / 1e3)}}
    ctx.close()
    return out


def fastrambo_report(n_particles=6, n=10_000_000, reps=5):
    """e+e- -> 6 massless particles at 1 TeV through one FastRambo chain
    (f = 1, so the weights are the phase-space weights): fused sample
    throughput and the spread of the weights around the volume.  Bytes per
    event: momenta 8 x 4 x 8 + weight 8 + channel 4 = 268 B."""
    import math

    import torch

    import workloads as W
    from paper_2602_06895_amd import Context

    ctx, _ = make_context(W.rambo_process(n_particles))
    counts = np.array([n])
    out = ctx.sample(counts, seed=6, stream_id=1)
    ms = _timed(lambda: ctx.sample(counts, seed=6, stream_id=1, out=out), reps)
    w = out["w"]
    torch.cuda.synchronize()
    mean, std = float(w.mean()), float(w.std())
    k = n_particles
    V = (2 * math.pi) ** (4 - 3 * k) * (math.pi / 2) ** (k - 1) * 1e6 ** (k - 2) / (math.gamma(k) * math.gamma(k - 1))
    bpe = (k + 2) * 4 * 8 + 8 + 4
    ach = n * bpe / (ms / 1e3) / 1e9
    ctx.close()
    return {"workload": f"e+e- -> {k} massless, sqrt(s) = 1 TeV, FastRambo, {n} events",
            "events_per_s": n / (ms / 1e3), "ms": ms, "mean_weight_over_volume": mean / V,
            "weight_std_over_mean": std / mean,
            "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": ach / HBM_PEAK_GBS, "bytes_per_event": bpe}}


def chili_report(n=10_000_000, reps=5):
    """pp -> 4 jets (the headline integrand: toy PDFs, t-propagators, p_T >
    20 GeV) through one Chili channel: fused sample throughput, the integral
    and its relative error per event, and the share of events the recoiling
    last jet fails the cut.  Bytes per event as for the headline: momenta 6 x
    4 x 8 + weight 8 + channel 4 = 204 B."""
    import torch

    import workloads as W
    from paper_2602_06895_amd import Context

    desc = W.c2_pp4j()
    desc["channels"] = [{"chili": True}]
    ctx, _ = make_context(desc)
    counts = np.array([n])
    out = ctx.sample(counts, seed=8, stream_id=1)
    ms = _timed(lambda: ctx.sample(counts, seed=8, stream_id=1, out=out), reps)
    w = out["w"]
    torch.cuda.synchronize()
    mean, std = float(w.mean()), float(w.std())
    zero = float((w == 0).double().mean())
    bpe = 6 * 4 * 8 + 8 + 4
    ach = n * bpe / (ms / 1e3) / 1e9
    ctx.close()
    return {"workload": f"pp -> 4 jets, sqrt(s) = 13 TeV, one Chili channel, {n} events",
            "events_per_s": n / (ms / 1e3), "ms": ms, "integral": mean, "rel_std_per_event": std / mean,
            "cut_share": zero,
            "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": ach / HBM_PEAK_GBS, "bytes_per_event": bpe}}


def dec3_report(n=10_000_000, reps=5):
    """pp -> t tbar -> 6 (the t tbar integrand) with each top decaying
    1 -> 3 (E1, E2, angles; no W mapping) instead of through the W: fused
    sample throughput, the integral and the per-event weight spread next to
    the two-step decay chain's.  Bytes per event: momenta 8 x 4 x 8 + x1x2
    16 + weight 8 + channel 4 = 284 B."""
    import torch

    import workloads as W
    from paper_2602_06895_amd import Context

    out_d = {}
    mt, gt = 173.0, 1.5
    for key in ("three_body", "two_body_chain"):
        desc = W.c3_ttbar6()
        if key == "three_body":
            desc["channels"] = [{"s": {"d": [{"d": [1, 2, 3], "m": mt, "w": gt, "order": 1},
                                             {"d": [4, 5, 6], "m": mt, "w": gt, "order": 2}]}}]
        ctx, _ = make_context(desc)
        counts = np.array([n])
        out = ctx.sample(counts, seed=9, stream_id=1)
        ms = _timed(lambda: ctx.sample(counts, seed=9, stream_id=1, out=out), reps)
        w = out["w"]
        torch.cuda.synchronize()
        mean, std = float(w.mean()), float(w.std())
        out_d[key] = {"events_per_s": n / (ms / 1e3), "ms": ms, "integral": mean, "rel_std_per_event": std / mean}
        ctx.close()
    bpe = 8 * 4 * 8 + 16 + 8 + 4
    ach = n * bpe / (out_d["three_body"]["ms"] / 1e3) / 1e9
    return {"workload": f"pp -> t tbar -> 6, 13 TeV, top decays 1 -> 3, {n} events", **out_d,
            "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": ach / HBM_PEAK_GBS, "bytes_per_event": bpe}}


def summarize(d: str, events: int, steps: int = 10, kernel: str = "k_sample", bytes_per_event: int = BYTES_PER_EVENT,
              title: str = "pp -> t tbar -> 6 (one channel, 16 dims, FP64)"):
    """Summary of the rocprofv3 runs under d (rocpd databases of the commands
    recorded in the profile's header): the trace of the timed dispatches
    (the last `steps` of the largest `kernel` launches), their HBM bytes from
    FETCH_SIZE / WRITE_SIZE scaled by a 1 GiB device copy, and their SQ
    instruction counters."""
    import glob
    import sqlite3

    def db(sub):
        f = glob.glob(os.path.join(d, sub, "*_results.db"))
        return sqlite3.connect(f[0]) if f else None

    out = []
    tr = db("trace")
    like = f"%{kernel}%"
    rows = list(tr.execute("select duration, grid_x, workgroup_x, vgpr_count, accum_vgpr_count, sgpr_count, "
                           "scratch_size, lds_size, name from kernels where name like ? order by start", (like,)))
    big = max(r[0] for r in rows)
    timed = [r for r in rows if r[0] > 0.5 * big][-steps:]
    dur = np.array([r[0] for r in timed]) / 1e3
    r0 = timed[0]
    short0 = r0[8].replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "")
    out.append(f"kernel: {short0} on {title}: {len(timed)} timed dispatches of {events} events")
    out.append(f"duration_us: avg {dur.mean():.1f} min {dur.min():.1f} max {dur.max():.1f}")
    out.append(f"launch (as rocprofv3 records it): grid {r0[1]} work-items, workgroup {r0[2]}, vgpr {r0[3]}, "
               f"agpr {r0[4]}, sgpr {r0[5]}, scratch {r0[6]} B/lane, lds {r0[7]} B")
    others = list(tr.execute("select name, count(*), avg(duration) from kernels group by name order by sum(duration) desc"))
    for name, cnt, avg in others[:8]:
        short = name.replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "")
        out.append(f"  kernel {short}: {cnt} dispatches, avg {avg / 1e3:.1f} us")

    def counter(sub, like_, name):
        c = db(sub)
        if c is None:
            return None
        return [r[0] for r in c.execute("select sum(value) from counters_collection where kernel_name like ? and "
                                        "counter_name = ? group by dispatch_id order by dispatch_id", (like_, name))]

    fetch = counter("fetch", like, "FETCH_SIZE")
    write = counter("write", like, "WRITE_SIZE")
    cf = counter("cfetch", "%copyBuffer%", "FETCH_SIZE")
    cw = counter("cwrite", "%copyBuffer%", "WRITE_SIZE")
    if fetch and write and cf and cw:
        copy_kib = 2 ** 30 / 1024
        sf, sw = copy_kib / np.median(cf), copy_kib / np.median(cw)
        f_big, w_big = max(fetch), max(write)
        hbm = f_big * 1024 * sf + w_big * 1024 * sw
        out.append(f"copy calibration (1 GiB device copy): FETCH_SIZE {np.median(cf):.0f} KiB -> read scale {sf:.3f}; "
                   f"WRITE_SIZE {np.median(cw):.0f} KiB -> write scale {sw:.3f}")
        out.append(f"counters per timed dispatch: FETCH_SIZE {f_big:.1f} KiB, WRITE_SIZE {w_big:.1f} KiB")
        out.append(f"hbm_bytes_per_launch: {hbm:.6e}")
        out.append(f"hbm_bytes_per_event: {hbm / events:.2f}")
    sq = {k: counter("sq", like, k) for k in ("SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_SMEM",
                                                "SQ_WAVES", "SQ_ACTIVE_INST_VALU", "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES")}
    if sq["SQ_INSTS_VALU"]:
        k = int(np.argmax(sq["SQ_INSTS_VALU"]))
        v = {n: (a[k] if a else None) for n, a in sq.items()}
        out.append("SQ counters of the largest dispatch: " +
                   ", ".join(f"{n} {x:.4g}" for n, x in v.items() if x is not None))
        out.append(f"valu_per_event: {v['SQ_INSTS_VALU'] * 64 / events:.1f}")
        if v["SQ_INSTS_SALU"] is not None:
            out.append(f"salu_per_wave: {v['SQ_INSTS_SALU'] * 64 / events:.1f}")
    out.append(f"algorithmic_bytes_per_event: {bytes_per_event}")
    out.append(f"kernel_source_sha256: {kernel_source_hash()}")
    print("\n".join(out))

def summarize_flow(d: str):
    """Per-kernel summary of a rocprofv3 kernel trace of `bench.py --flow-only`
    under d/flow (the coupling-flow kernels; GEMMs split by launch grid)."""
    import glob
    import sqlite3

    f = glob.glob(os.path.join(d, "flow", "*_results.db"))
    c = sqlite3.connect(f[0])
    out = ["flow kernels (name: dispatches, avg us, total ms)"]
    for name, cnt, avg, tot in c.execute("select name, count(*), avg(duration), sum(duration) from kernels "
                                         "group by name order by sum(duration) desc"):
        short = name.replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "")
        out.append(f"  {short[:60]}: {cnt}, {avg / 1e3:.1f}, {tot / 1e6:.2f}")
    out.append("k_gemm by grid (x work-items, y, z: dispatches, avg us, vgpr, agpr)")
    for gx, gy, gz, cnt, avg, vg, ag in c.execute(
            "select grid_x, grid_y, grid_z, count(*), avg(duration), max(vgpr_count), max(accum_vgpr_count) "
            "from kernels where name like '%k_gemm%' group by grid_x, grid_y, grid_z order by sum(duration) desc"):
        out.append(f"  {gx} x {gy} x {gz}: {cnt}, {avg / 1e3:.1f}, {vg}, {ag}")
    print("\n".join(out))


def summarize_trace(d: str):
    """Per-kernel summary of any rocprofv3 kernel trace under d: name,
    dispatches, average and total duration, the largest grid, VGPRs and
    scratch bytes per lane."""
    import glob
    import sqlite3

    out = ["kernels (name: dispatches, avg us, total ms, max grid work-items, vgpr, scratch B/lane)"]
    for f in sorted(glob.glob(os.path.join(d, "**", "*_results.db"), recursive=True)):
        c = sqlite3.connect(f)
        for name, cnt, avg, tot, gx, vg, sc in c.execute(
                "select name, count(*), avg(duration), sum(duration), max(grid_x), max(vgpr_count), "
                "max(scratch_size) from kernels group by name order by sum(duration) desc"):
            short = name.replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "")
            out.append(f"  {short[:70]}: {cnt}, {avg / 1e3:.1f}, {tot / 1e6:.2f}, {gx}, {vg}, {sc}")
    print("\n".join(out))


def summarize_counters(d: str):
    """Average value per dispatch of every counter of a rocprofv3 --pmc run
    under d, per kernel of this library."""
    import glob
    import sqlite3

    out = ["counters (kernel: counter = average per dispatch over dispatches)"]
    for f in sorted(glob.glob(os.path.join(d, "**", "*_results.db"), recursive=True)):
        c = sqlite3.connect(f)
        for name, ctr, avg, cnt in c.execute(
                "select kernel_name, counter_name, avg(v), count(*) from (select kernel_name, counter_name, "
                "dispatch_id, sum(value) as v from counters_collection where kernel_name like '%msx%' "
                "group by kernel_name, counter_name, dispatch_id) group by kernel_name, counter_name "
                "order by kernel_name, counter_name"):
            short = name.replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "")
            out.append(f"  {short[:60]}: {ctr} = {avg:.4g} over {cnt}")
    print("\n".join(out))


def headline(args):
    """The N=1 line: pp -> t tbar -> 6 at 1e8 events per graph replay, FP64."""
    import torch

    import workloads as W
    from paper_2602_06895_amd import Context, adapt_vegas

    desc = W.c3_ttbar6()
    ctx, spec_s = make_context(desc, device=0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    adapt_vegas(ctx, n_per_channel=100_000, iterations=10, alpha=0.5, seed=3, stream_id=1)
    torch.cuda.synchronize()
    adapt_s = time.perf_counter() - t0
    N = args.events
    counts = np.array([N], dtype=np.int64)
    if not args.no_autotune:
        ctx.autotune(counts, seed=1, reps=3)
    grids = [ctx.get_grid(0)]
    buf, wall, ms = graph_steps(ctx, counts, 1000, args.steps, args.warmup)
    I, rel = integral_of(ctx.stats(), args.steps)
    stats = ctx.stats()
    pass_frac = 1.0 - stats[:, 3].sum() / stats[:, 2].sum()
    eff, _ = ctx.unweight_eff(buf["w"], 1e-3)
    ms_per_step = wall * 1e3 / args.steps
    launch_s = float(np.mean(ms)) / 1e3
    ept, grid = ctx.launch_shape()
    del buf
    torch.cuda.empty_cache()
    other = None
    if SPECIALIZE:
        # the class kernel on the same workload and launch shape (5 replays)
        ctx.specialize(False)
        b2, _, ms_cls = graph_steps(ctx, counts, 3000, 5, 1)
        del b2
        torch.cuda.empty_cache()
        other = {"kernel": "k_sample (class kernel, tables read from device memory)",
                 "median_replay_ms": float(np.median(ms_cls)), "events_per_s": N / (float(np.median(ms_cls)) / 1e3)}
    result = {
        "metric": "weighted events/sec at fixed integral rel. error; unweighting eff. flow vs VEGAS",
        "value": N / (ms_per_step / 1e3),
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "pp->ttbar->bW+bW-->6 13 TeV, BW t(173,1.5) W(80.4,2.1), toy PDFs, VEGAS 64 bins "
                               f"x 16 dims adapted 10x1e5 then frozen, {N} events per step, FP64",
                   "events_per_step": N, "channels": 1, "sampler": "vegas",
                   "timed_step": "one replay of the captured fused-sample graph (new events every replay)",
                   "launch": {"events_per_thread": ept, "workgroups": grid},
                   "kernel": "msx_jit_sample (compiled for the channel, msx_specialize)" if SPECIALIZE else
                             "k_sample (class kernel)"},
        "integral": I,
        "rel_error_per_step": rel,
        "median_replay_ms": float(np.median(ms)),
        "pass_cut_fraction": pass_frac,
        "passing_events_per_s": N * pass_frac / (ms_per_step / 1e3),
        "unweighting_eff": eff,
        "vegas_adaptation": {"iterations": 10, "events_per_iteration": 100_000, "seconds": adapt_s,
                             "where": "histograms accumulated inside the fused sample (msx_vegas_adapt)"},
        "specialize_seconds": spec_s,
        "roofline": dict(roofline(N, BYTES_PER_EVENT, launch_s, profiled(PROFILE if SPECIALIZE else PROFILE_CLASS)),
                         kernel=("msx_jit_sample" if SPECIALIZE else "k_sample") +
                         " (fused sample, graph replay: plan + sample + statistics + counter kernels between the "
                         "HIP events)"),
    }
    if other:
        result["class_kernel"] = other
    ctx.close()
    return result, desc, grids, counts


def c2_report(steps=20, warmup=3, autotune=True):
    """pp -> 4 jets, eight channels (t, mixed and s topologies) with local
    channel weights, 1e7 events per graph replay, FP64: throughput, both
    roofs, unweighting and the validation distributions of one replay's
    events."""
    import torch

    import workloads as W
    from paper_2602_06895_amd import OBS_DR_HARDEST, OBS_M, OBS_PT_RANK, Context, adapt_vegas, neyman_counts

    ctx, spec_s = make_context(W.c2_pp4j(), device=0)
    st = adapt_vegas(ctx, n_per_channel=100_000, iterations=10, alpha=0.5, seed=1, stream_id=1)
    counts = neyman_counts(st, C2_EVENTS)
    if autotune:
        ctx.autotune(counts, seed=1, reps=5)
    N = int(counts.sum())
    buf, wall, ms = graph_steps(ctx, counts, 2000, steps, warmup, want_chan=True)
    I, rel = integral_of(ctx.stats(), steps)
    stats = ctx.stats()
    pass_frac = 1.0 - stats[:, 3].sum() / stats[:, 2].sum()
    eff_w = buf["w"].clone()
    off = 0
    for c, k in enumerate(counts):
        eff_w[off:off + k] *= N / float(k)
        off += int(k)
    eff, wmax = ctx.unweight_eff(eff_w, 1e-3)
    unw_ms = _timed(lambda: ctx.unweight(eff_w, wmax, seed=3, stream_id=99), 5)
    kept = int(ctx.unweight(eff_w, wmax, seed=3, stream_id=99)["count"].cpu()[0])
    jets = list(range(4))
    spec = [(OBS_M, jets, 0), (OBS_PT_RANK, jets, 0), (OBS_DR_HARDEST, jets, 0)]

    def distributions():
        x = ctx.observables(0, buf["p"], spec)
        wc = ctx.cut(x, [0.0, 50.0, 0.4], [1.3e4, np.inf, np.inf], eff_w.clone())
        return [ctx.histogram(x[j], wc, b, a, c) for j, (b, a, c) in
                enumerate([(50, 0.0, 6500.0), (40, 0.0, 2000.0), (30, 0.0, 6.0)])]

    dist_ms = _timed(distributions, 3)
    ms_per_step = wall * 1e3 / steps
    ept, grid = ctx.launch_shape()
    out = {"workload": f"pp->4j 13 TeV, 8 channels (t/mixed/s), VEGAS 64 bins x 10 dims adapted 10x1e5 per "
                       f"channel then frozen, Neyman counts, {N} events per graph replay, FP64",
           "events_per_s": N / (ms_per_step / 1e3), "ms_per_step": ms_per_step,
           "median_replay_ms": float(np.median(ms)), "integral": I, "rel_error_per_step": rel,
           "pass_cut_fraction": pass_frac, "unweighting_eff": eff,
           "launch": {"events_per_thread": ept, "workgroups": grid},
           "unweighting": {"w_max_overweight": 1e-3, "kept": kept, "ms": unw_ms, "events_per_s": N / (unw_ms / 1e3)},
           "distributions": {"observables": "sqrt(s-hat), hardest-jet pT, dR of the two hardest jets",
                             "cut_and_3_histograms_ms": dist_ms, "events_per_s": N / (dist_ms / 1e3)},
           "kernel": "msx_jit_sample" if SPECIALIZE else "k_sample", "specialize_seconds": spec_s,
           "roofline": roofline(N, C2_BYTES_PER_EVENT, float(np.mean(ms)) / 1e3,
                                profiled(PROFILE_C2) if SPECIALIZE else {})}
    ctx.close()
    del buf
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--events", type=int, default=N_EVENTS)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-autotune", action="store_true", help="default launch shape instead of the autotuned one")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the pp -> 4 jets, mixed-precision, flow, graph and inverse-map reports")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run device-to-device copies of 1 GiB (scale for HBM byte counters)")
    ap.add_argument("--summarize", metavar="DIR", help="summarise rocprofv3 output under DIR and exit")
    ap.add_argument("--summarize-c2", metavar="DIR", help="the same for the pp -> 4 jets report's kernel")
    ap.add_argument("--summarize-flow", metavar="DIR", help="summarise a flow kernel trace under DIR/flow and exit")
    ap.add_argument("--summarize-trace", metavar="DIR", help="per-kernel summary of any kernel trace under DIR")
    ap.add_argument("--summarize-counters", metavar="DIR", help="per-kernel counter averages of a --pmc run under DIR")
    ap.add_argument("--flow-only", action="store_true", help="only the learned-sampler report")
    ap.add_argument("--flow-steps", type=int, default=400, help="training steps of the learned sampler")
    ap.add_argument("--inverse-only", action="store_true", help="only the inverse-map report")
    ap.add_argument("--c2-only", action="store_true", help="only the pp -> 4 jets report")
    ap.add_argument("--no-specialize", action="store_true",
                    help="sample with the class kernels instead of the kernel compiled for the channels")
    ap.add_argument("--kernel", default=None, help="--summarize*: the kernel name to summarise")
    args = ap.parse_args()
    global SPECIALIZE
    SPECIALIZE = not args.no_specialize
    if args.summarize_trace:
        summarize_trace(args.summarize_trace)
        return
    if args.summarize_counters:
        summarize_counters(args.summarize_counters)
        return
    if args.summarize:
        summarize(args.summarize, args.events, kernel=args.kernel or "msx_jit_sample")
        return
    if args.summarize_c2:
        summarize(args.summarize_c2, C2_EVENTS, kernel=args.kernel or "msx_jit_sample",
                  bytes_per_event=C2_BYTES_PER_EVENT, title="pp -> 4 jets (8 channels, 10 dims, FP64)")
        return
    if args.summarize_flow:
        summarize_flow(args.summarize_flow)
        return
    if args.flow_only:
        print(json.dumps({"flow_vs_vegas": flow_report(train_steps=args.flow_steps)}))
        return
    if args.inverse_only:
        print(json.dumps({"inverse_map": inverse_report(), "fastrambo": fastrambo_report(),
                          "chili": chili_report(), "dec3": dec3_report()}))
        return
    if args.c2_only:
        print(json.dumps({"pp4j": c2_report(args.steps, args.warmup, not args.no_autotune)}))
        return
    if args.copy_calibration:
        import torch

        src = torch.ones(2 ** 27, dtype=torch.float64, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 8, "copy_bytes_written": dst.numel() * 8, "copies": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU sharding is "
              "design-only in this build", file=sys.stderr)
        sys.exit(2)

    import torch

    result, desc, grids, counts = headline(args)
    if not args.no_extras:
        result["pp4j"] = c2_report(autotune=not args.no_autotune)
        result["mixed_precision"] = mixed_report()
        torch.cuda.empty_cache()
        result["flow_vs_vegas"] = flow_report(train_steps=args.flow_steps)
        torch.cuda.empty_cache()
        result["flow_vs_vegas_c2_channel0"] = flow_report(train_steps=args.flow_steps, workload="c2", channel=0)
        torch.cuda.empty_cache()
        result["multichannel_graph"] = graph_report()
        torch.cuda.empty_cache()
        result["inverse_map"] = inverse_report()
        torch.cuda.empty_cache()
        result["fastrambo"] = fastrambo_report()
        result["chili"] = chili_report()
        result["decay_1to3"] = dec3_report()
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(desc, grids, counts, seed=1)
    print(json.dumps(result))


if __name__ == "__main__":
    main()
