"""Throughput of the phase-space hot path on one MI355X.

Workload: pp -> 4 massless jets at sqrt(s) = 13 TeV, eight diagram channels
(pure t, mixed and pure s topologies) with local channel weights, toy PDF
x^-1.2 (1-x)^3, t-propagator integrand with mu = 10 GeV and pT > 20 GeV cuts,
VEGAS 64 bins x 10 dims, FP64.  VEGAS grids are adapted first (untimed), then
frozen.  One step = one fused multichannel `sample` of 1e7 events (in-kernel
Philox uniforms -> VEGAS -> mapping chain -> integrand x channel weight ->
SoA stores and per-channel statistics), inputs (the grids and channel
tables) already resident in HBM.

Prints one JSON line (see the keys below).  --gpus N > 1 is refused: this
build runs on one GPU.
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

N_EVENTS = 10_000_000
BYTES_PER_EVENT = 6 * 4 * 8 + 2 * 8 + 8 + 4  # momenta (a, b, 4 jets), x1 x2, w, channel id
HBM_PEAK_GBS = 8000.0


def cpu_baseline(desc, grids, counts, seed, min_seconds=10.0):
    """The FP64 oracle on the host cores (OpenMP over events): every channel in
    proportion to the GPU counts, repeated until min_seconds of wall time have
    been timed; uniform generation is outside the timed region."""
    import oracle
    import workloads as W

    P = oracle.Process(desc)
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    frac = counts / counts.sum()
    batch = 400_000
    per = np.maximum(1, np.round(frac * batch)).astype(np.int64)
    ys = [W.philox_uniforms(seed, 0, 0, int(per[c]), P.dims[c]) for c in range(len(per))]
    done, elapsed = 0, 0.0
    while elapsed < min_seconds:
        t0 = time.perf_counter()
        for c in range(len(per)):
            P.map(c, ys[c], grids[c], nthreads=threads)
        elapsed += time.perf_counter() - t0
        done += int(per.sum())
    return {"value": done / elapsed, "unit": "events/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} events of the same workload ({int(per.sum())} per pass, channels in the "
                      f"GPU's proportions, frozen grids), {elapsed:.1f} s on {threads} threads"}


# sources of the fused sample kernel (a change invalidates the committed counter figures)
KERNEL_SOURCES = ["paper_2602_06895_amd/csrc/" + f for f in
                  ("chain_kernels.h", "chain.h", "device_util.h", "tables.h", "chain_f64_s.hip")]
PROFILE = os.path.join(ROOT, "profiles", "k_sample_pp4j_1e7.txt")


def kernel_source_hash() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_traffic():
    """HBM bytes per launch from the committed counter summary, or None when the
    kernel sources changed since the counters were taken."""
    if not os.path.exists(PROFILE):
        return None
    vals = {}
    for line in open(PROFILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


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


def mixed_report(n=10_000_000, reps=5):
    """pp -> t tbar -> 6 (16 dims, Breit-Wigner t and W): FP64 and mixed
    precision sample throughput on the same events, and the per-quantity error
    of the mixed results against the FP64 ones."""
    import workloads as W
    from paper_2602_06895_amd import MIXED, Context, adapt_vegas
    from paper_2602_06895_amd.report import precision_error

    c64 = Context(W.c3_ttbar6())
    cmx = Context(W.c3_ttbar6(), precision=MIXED)
    adapt_vegas(c64, n_per_channel=100_000, iterations=5, seed=2, stream_id=1)
    cmx.set_grid(0, c64.get_grid(0))
    counts = np.array([n])
    o64 = c64.sample(counts, seed=77, stream_id=0)
    omx = cmx.sample(counts, seed=77, stream_id=0)
    t64 = _timed(lambda: c64.sample(counts, seed=77, stream_id=0, out=o64), reps)
    tmx = _timed(lambda: cmx.sample(counts, seed=77, stream_id=0, out=omx), reps)
    err = precision_error(omx["p"], omx["w"], o64["p"], o64["w"], c64.max_momenta)
    c64.close()
    cmx.close()
    return {"workload": f"pp->ttbar->6 13 TeV, BW t/W, 16 dims, {n} events per launch",
            "fp64_events_per_s": n / (t64 / 1e3), "mixed_events_per_s": n / (tmx / 1e3), "speedup": t64 / tmx,
            "mixed_error_vs_fp64": err}


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
    ctx = Context(desc)
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
    use_flow = rel_f < rel_v
    name = "pp->ttbar->6 integrand" if workload == "c3" else f"pp->4j channel {channel}"
    res = {"workload": f"{name}, {d} dims, VEGAS 10x1e5 then flow {train_steps} x {batch} BF16",
           "vegas": {"unweighting_eff": eff_v, "rel_error": rel_v, "integral": float(wv.mean())},
           "flow": {"unweighting_eff": eff_f, "rel_error": rel_f, "integral": float(wf.mean())},
           "events": n_eval, "eff_ratio_flow_over_vegas": eff_f / eff_v,
           "rel_error_ratio_vegas_over_flow": rel_v / rel_f, "sampler_kept": "flow" if use_flow else "vegas",
           "train_seconds": train_s, "loss_first": float(losses[0].cpu()[0]), "loss_last": float(losses[-1].cpu()[0]),
           "flow_forward_2e20": {"ms": ms, "mlp_tflops": flops / (ms / 1e3) / 1e12, "peak_tflops": 2500.0,
                                 "frac": flops / (ms / 1e3) / 1e12 / 2500.0,
                                 "fused_layers": fused, "bound": "mfma" if fused else "hbm",
                                 "algorithmic_bytes_per_event": 8 * bytes_layer, "hbm_gbs": hbm_gbs,
                                 "hbm_frac": hbm_gbs / HBM_PEAK_GBS}}
    flow.close()
    ctx.close()
    return res


def graph_report(reps=10):
    """24-channel batch (C1 and C2 topologies, power-law counts) as one
    persistent launch replayed from a HIP graph, after the autotuner."""
    import torch

    import workloads as W
    from paper_2602_06895_amd import Context

    desc, counts = W.c4_context()
    ctx = Context(desc)
    N = int(counts.sum())
    eager_ms = _timed(lambda: ctx.sample(counts, seed=4, stream_id=8), reps)
    best = ctx.autotune(counts, seed=4, reps=3)
    ept, grid = ctx.launch_shape()
    buf = ctx.sample_buffers(N, want_chan=True)
    dc = torch.from_numpy(counts.astype(np.int64)).cuda()
    off = torch.zeros(1, dtype=torch.int64, device="cuda")
    g = ctx.sample_graph(dc, 4, 8, off, buf)
    graph_ms = _timed(g.launch, reps)
    g.close()
    ctx.close()
    return {"workload": f"24 channels (6 processes), {N} events, counts power-law 1e3..1e6",
            "eager_ms": eager_ms, "graph_ms": graph_ms, "graph_events_per_s": N / (graph_ms / 1e3),
            "autotuned": {"events_per_thread": ept, "grid": grid, "ms": best}}


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

    ctx = Context(W.rambo_process(n_particles))
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
    ctx = Context(desc)
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
        ctx = Context(desc)
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


def summarize(d: str, events: int, steps: int = 10):
    """Summary of the rocprofv3 runs under d (rocpd databases written by the
    commands printed below) for the last `steps` k_sample dispatches of
    `events` events (the timed steps of the traced run)."""
    import glob
    import sqlite3

    def db(sub):
        f = glob.glob(os.path.join(d, sub, "*_results.db"))
        return sqlite3.connect(f[0]) if f else None

    out = []
    tr = db("trace")
    rows = list(tr.execute("select duration, grid_x, workgroup_x, vgpr_count, accum_vgpr_count, sgpr_count, "
                           "scratch_size, lds_size from kernels where name like '%k_sample%' order by start"))
    # the timed launches are the last `steps` large ones (adaptation launches
    # carry 8e5 events; the autotuner's trial launches come before the timed ones)
    big = max(r[0] for r in rows)
    timed = [r for r in rows if r[0] > 0.5 * big][-steps:]
    dur = np.array([r[0] for r in timed]) / 1e3
    r0 = timed[0]
    out.append(f"kernel: k_sample (fused multichannel sample), {len(timed)} timed dispatches of {events} events")
    out.append(f"duration_us: avg {dur.mean():.1f} min {dur.min():.1f} max {dur.max():.1f}")
    out.append(f"launch: grid {r0[1]} work-items, workgroup {r0[2]}, vgpr {r0[3]}, agpr {r0[4]}, sgpr {r0[5]}, "
               f"scratch {r0[6]} B/lane, lds {r0[7]} B")
    others = list(tr.execute("select name, count(*), avg(duration) from kernels group by name order by sum(duration) desc"))
    for name, cnt, avg in others[:8]:
        short = name.replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "")
        out.append(f"  kernel {short}: {cnt} dispatches, avg {avg / 1e3:.1f} us")

    def counter(sub, like, name):
        c = db(sub)
        if c is None:
            return None
        v = [r[0] for r in c.execute("select value from counters_collection where kernel_name like ? and "
                                     "counter_name = ? order by dispatch_id", (like, name))]
        return v

    fetch = counter("fetch", "%k_sample%", "FETCH_SIZE")
    write = counter("write", "%k_sample%", "WRITE_SIZE")
    cf = counter("cfetch", "%copyBuffer%", "FETCH_SIZE")
    cw = counter("cwrite", "%copyBuffer%", "WRITE_SIZE")
    if fetch and write and cf and cw:
        copy_kib = 2 ** 30 / 1024
        sf, sw = copy_kib / np.median(cf), copy_kib / np.median(cw)
        f_big = max(fetch)
        w_big = max(write)
        hbm = f_big * 1024 * sf + w_big * 1024 * sw
        out.append(f"copy calibration (1 GiB device copy): FETCH_SIZE {np.median(cf):.0f} KiB -> read scale {sf:.3f}; "
                   f"WRITE_SIZE {np.median(cw):.0f} KiB -> write scale {sw:.3f}")
        out.append(f"counters per timed dispatch: FETCH_SIZE {f_big:.1f} KiB, WRITE_SIZE {w_big:.1f} KiB")
        out.append(f"hbm_bytes_per_launch: {hbm:.6e}")
        out.append(f"hbm_bytes_per_event: {hbm / events:.1f}")
    out.append(f"algorithmic_bytes_per_event: {BYTES_PER_EVENT}")
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
                "dispatch_id, sum(value) as v from counters_collection where kernel_name like '%msx::%' "
                "group by kernel_name, counter_name, dispatch_id) group by kernel_name, counter_name "
                "order by kernel_name, counter_name"):
            short = name.replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "")
            out.append(f"  {short[:60]}: {ctr} = {avg:.4g} over {cnt}")
    print("\n".join(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--events", type=int, default=N_EVENTS)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-autotune", action="store_true", help="default launch shape instead of the autotuned one")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the mixed-precision, flow, graph and inverse-map reports")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run device-to-device copies of 1 GiB (scale for HBM byte counters)")
    ap.add_argument("--summarize", metavar="DIR", help="summarise rocprofv3 output under DIR and exit")
    ap.add_argument("--summarize-flow", metavar="DIR", help="summarise a flow kernel trace under DIR/flow and exit")
    ap.add_argument("--summarize-trace", metavar="DIR", help="per-kernel summary of any kernel trace under DIR")
    ap.add_argument("--summarize-counters", metavar="DIR", help="per-kernel counter averages of a --pmc run under DIR")
    ap.add_argument("--flow-only", action="store_true", help="only the learned-sampler report")
    ap.add_argument("--flow-steps", type=int, default=400, help="training steps of the learned sampler")
    ap.add_argument("--inverse-only", action="store_true", help="only the inverse-map report")
    args = ap.parse_args()
    if args.summarize_trace:
        summarize_trace(args.summarize_trace)
        return
    if args.summarize_counters:
        summarize_counters(args.summarize_counters)
        return
    if args.summarize:
        summarize(args.summarize, args.events)
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

    import workloads as W
    from paper_2602_06895_amd import Context, adapt_vegas, neyman_counts

    desc = W.c2_pp4j()
    ctx = Context(desc, device=0)
    # adaptation phase (untimed): 8 iterations x 1e5 events per channel
    st = adapt_vegas(ctx, n_per_channel=100_000, iterations=8, alpha=0.5, seed=1, stream_id=1)
    counts = neyman_counts(st, args.events)
    grids = [ctx.get_grid(c) for c in range(ctx.n_channels)]
    # launch shape of the fused kernel for these counts (untimed setup)
    if not args.no_autotune:
        ctx.autotune(counts, seed=1, reps=2)
    N = int(counts.sum())
    out = {"p": torch.empty((4, ctx.max_momenta, N), dtype=torch.float64, device="cuda"),
           "w": torch.empty(N, dtype=torch.float64, device="cuda"),
           "x1x2": torch.empty((2, N), dtype=torch.float64, device="cuda"),
           "chan": torch.empty(N, dtype=torch.int32, device="cuda")}
    stream = torch.cuda.current_stream()

    def step(i):
        ctx.sample(counts, seed=1000 + i, stream_id=0, counter_offset=0, out=out)

    for i in range(args.warmup):
        step(i)
    ctx.reset_stats()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t_start = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        step(args.warmup + i)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    launch_ms = [a.elapsed_time(b) for a, b in ev]
    ms_per_step = wall * 1e3 / args.steps
    stats = ctx.stats()
    # integral over all timed steps (each step an independent sample)
    I = 0.0
    var = 0.0
    for s1, s2, n, nz, mx in stats:
        mean = s1 / n
        I += mean
        var += max(s2 / n - mean * mean, 0.0) / (n - 1)
    rel_err_step = math.sqrt(var * args.steps) / I  # rel. error reached by one step's events
    pass_frac = 1.0 - stats[:, 3].sum() / stats[:, 2].sum()
    # unweighting efficiency of one step's events (effective weight w * N / n_c)
    eff_w = out["w"].clone()
    off = 0
    for c, k in enumerate(counts):
        eff_w[off:off + k] *= N / float(k)
        off += int(k)
    eff, wmax = ctx.unweight_eff(eff_w, 1e-3)
    # the unweighting step itself on the same events (not in the timed step)
    unw_ms = _timed(lambda: ctx.unweight(eff_w, wmax, seed=3, stream_id=99), 5)
    kept = int(ctx.unweight(eff_w, wmax, seed=3, stream_id=99)["count"].cpu()[0])
    # the validation distributions of the same events: sqrt(s-hat), hardest-jet
    # p_T and the separation of the two hardest jets, a cut on them, three
    # weighted histograms
    from paper_2602_06895_amd import OBS_DR_HARDEST, OBS_M, OBS_PT_RANK

    jets = list(range(4))
    spec = [(OBS_M, jets, 0), (OBS_PT_RANK, jets, 0), (OBS_DR_HARDEST, jets, 0)]

    def distributions():
        x = ctx.observables(0, out["p"], spec)
        wc = ctx.cut(x, [0.0, 50.0, 0.4], [1.3e4, np.inf, np.inf], eff_w.clone())
        return [ctx.histogram(x[j], wc, b, a, c) for j, (b, a, c) in
                enumerate([(50, 0.0, 6500.0), (40, 0.0, 2000.0), (30, 0.0, 6.0)])]

    dist_ms = _timed(distributions, 3)

    avg_launch_s = float(np.mean(launch_ms)) / 1e3
    achieved = BYTES_PER_EVENT * N / avg_launch_s / 1e9
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
        "config": {"workload": "pp->4j 13 TeV, 8 channels (t/mixed/s), VEGAS 64 bins x 10 dims frozen, "
                               f"{N} events per step, FP64", "events_per_step": N, "channels": int(ctx.n_channels),
                   "sampler": "vegas", "launch": {"events_per_thread": ctx.launch_shape()[0],
                                                  "workgroups": ctx.launch_shape()[1]}},
        "integral": I,
        "rel_error_per_step": rel_err_step,
        "pass_cut_fraction": pass_frac,
        "unweighting_eff": eff,
        "passing_events_per_s": N * pass_frac / (ms_per_step / 1e3),
        "unweighting": {"w_max_overweight": 1e-3, "kept": kept, "ms": unw_ms,
                        "events_per_s": N / (unw_ms / 1e3)},
        "distributions": {"observables": "sqrt(s-hat), hardest-jet pT, dR of the two hardest jets",
                          "cut_and_3_histograms_ms": dist_ms, "events_per_s": N / (dist_ms / 1e3)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": profiled_traffic(),
                     "kernel": "k_sample (fused multichannel sample)",
                     "bytes_per_event": BYTES_PER_EVENT, "avg_launch_ms": avg_launch_s * 1e3},
    }
    ctx.close()
    del out
    if not args.no_extras:
        torch.cuda.empty_cache()
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
