"""Parity of the HIP path (through the C ABI) with the FP64 oracle on the same
seeded inputs.  Tolerances: see tests/parity.py."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from parity import U64, compare, weight_condition

pytestmark = pytest.mark.gpu

CONFIGS = {"c1": W.c1_ee_mumu, "c2": W.c2_pp4j, "c3": W.c3_ttbar6}


@pytest.fixture(scope="module")
def torch():
    import torch as t

    if not t.cuda.is_available():
        pytest.skip("needs a GPU")
    return t


@pytest.fixture(scope="module")
def ctxs(torch):
    from paper_2602_06895_amd import Context

    out = {k: (Context(f()), oracle.Process(f())) for k, f in CONFIGS.items()}
    yield out
    for c, _ in out.values():
        c.close()


def _np(t):
    return None if t is None else t.cpu().numpy()


def random_grid(dims, nb, seed):
    rng = np.random.default_rng(seed)
    g = np.empty((dims, nb + 1))
    for k in range(dims):
        inner = np.sort(rng.random(nb - 1))
        g[k] = np.concatenate([[0.0], inner, [1.0]])
    return g


# --------------------------------------------------------------------------
# RNG
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed,sid,e0,n,d", [(1, 0, 0, 1000, 10), (2**63 + 5, 3, 123456789, 777, 16),
                                             (9, 2**40, 2**62, 64, 5), (0, 0, 0, 1, 1)])
def test_philox_matches_numpy_bit_for_bit(ctxs, torch, seed, sid, e0, n, d):
    ctx = ctxs["c2"][0]
    y = ctx.uniform(seed, sid, e0, n, d)
    torch.cuda.synchronize()
    assert np.array_equal(_np(y), W.philox_uniforms(seed, sid, e0, n, d))


# --------------------------------------------------------------------------
# map (+ weight) of single channels
# --------------------------------------------------------------------------

def _map_case(ctxs, torch, cfg, chan, n, grid_seed, seed):
    ctx, orc = ctxs[cfg]
    d = ctx.dims[chan]
    grid = orc.uniform_grid(chan) if grid_seed is None else random_grid(d, ctx.nbins[chan], grid_seed)
    ctx.set_grid(chan, grid)
    y_h = W.philox_uniforms(seed, 5, 0, n, d)
    y = torch.from_numpy(y_h).to(ctx.device)
    out = ctx.map(chan, y, weight=True)
    torch.cuda.synchronize()
    ref = orc.map(chan, y_h, grid)
    fe = orc.forward_error(chan, y_h, grid, ref=ref)
    ctx.set_grid(chan, orc.uniform_grid(chan))
    got = {k: _np(v) for k, v in out.items()}
    return got, ref, fe


# Floors of the fraction of events whose weight meets the bare 1e-12 (measured
# on 5e5 events per channel with uniform grids: C1 1.0; pp -> 4 jets channels
# 0.736 0.793 0.849 0.933 0.974 0.976 0.989 0.985; pp -> t tbar -> 6 0.362),
# lowered by 0.05 for the sample size and the random grids of the cases below;
# momenta and Jacobians: 0.995 (uniform grids), 0.985 (random grids, measured
# 0.988-0.995).
STRICT_FLOOR = {"c1": [0.999], "c2": [0.68, 0.74, 0.80, 0.88, 0.92, 0.92, 0.94, 0.93], "c3": [0.31]}


@pytest.mark.parametrize("cfg,chan", [("c1", 0)] + [("c2", c) for c in range(8)] + [("c3", 0)])
@pytest.mark.parametrize("grid_seed", [None, 17])
def test_map_parity(ctxs, torch, cfg, chan, grid_seed):
    n = 60013  # several hundred tiles and a ragged tail
    got, ref, fe = _map_case(ctxs, torch, cfg, chan, n, grid_seed, seed=100 + chan)
    rep = compare(got, ref, fe, hadronic=cfg != "c1", label=f"{cfg}/{chan}", detail=True)
    beyond, rel = rep.pop("w_beyond_strict"), rep.pop("w_rel")
    assert rep["w_strict_frac"] >= STRICT_FLOOR[cfg][chan], rep
    jp_floor = 0.995 if grid_seed is None else 0.985  # random grids: narrow bins amplify edge roundings
    assert rep["p_strict_frac"] >= jp_floor and rep["jac_strict_frac"] >= jp_floor, rep
    if cfg == "c1":
        assert rep["w_strict_frac"] == 1.0 and rep["p_strict_frac"] == 1.0
    # every event beyond 1e-12, with its condition estimate: they are the
    # ill-conditioned ones (propagator invariants recomputed from momenta)
    if beyond.size:
        ctx, orc = ctxs[cfg]
        props = [ch.propagators() for ch in orc.channels] if ctx.n_channels > 1 else None
        kap = weight_condition(orc.desc, ref["p"], props)
        keep = (ref["w"] != 0) & (got["w"] != 0)
        within = np.setdiff1d(np.flatnonzero(keep), beyond)
        med_b, med_w = np.median(kap[beyond]), np.median(kap[within]) if within.size else 0.0
        print(f"{cfg}/{chan} grid {grid_seed}: {beyond.size} of {keep.sum()} weights beyond 1e-12; condition "
              f"u kappa median {U64 * med_b:.2e} (p10 {U64 * np.quantile(kap[beyond], 0.1):.2e}) against "
              f"{U64 * med_w:.2e} within; |dw|/w median {np.median(rel[beyond]):.2e} max {rel[beyond].max():.2e}")
        if grid_seed is None:
            # (under random grids narrow VEGAS bins add a conditioning that
            # kappa does not model)
            assert med_b >= 2.0 * med_w
    print(cfg, chan, grid_seed, rep)


def test_weight_entry_matches_oracle(ctxs, torch):
    """msx_weight on the oracle's lab-frame map outputs against the oracle's
    weight of the same inputs."""
    ctx, orc = ctxs["c2"]
    n = 20011
    for chan in (0, 4, 7):
        y_h = W.philox_uniforms(55, 1, 0, n, ctx.dims[chan])
        m = orc.map(chan, y_h, orc.uniform_grid(chan))
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(ctx.device)
        w, a = ctx.weight(chan, dev(m["p"]), dev(m["x1x2"]), dev(m["jac"]), alpha=True)
        torch.cuda.synchronize()
        ref = orc.weight(chan, m["p"], m["x1x2"], m["jac"])
        fe = orc.weight_forward_error(chan, m["p"], m["x1x2"], m["jac"], ref=ref)
        compare({"w": _np(w)}, ref, fe, hadronic=True, label=f"weight/{chan}")
        a = _np(a)
        ok = ref["w"] != 0
        # alpha lies in [0, 1] and sums to 1 over channels: absolute norm
        assert np.abs(a[ok] - ref["alpha"][ok]).max() <= 1e-9


def test_c1_two_body_volume_every_event(ctxs, torch):
    from paper_2602_06895_amd import Context

    ctx = Context(W.c1_ee_mumu(integrand="unit"))
    y = ctx.uniform(1, 0, 0, 100000, 2)
    out = ctx.map(0, y, weight=True)
    torch.cuda.synchronize()
    assert np.allclose(_np(out["w"]), 1 / (8 * math.pi), rtol=1e-14, atol=0)
    ctx.close()


@pytest.mark.parametrize("cfg", ["c2", "c3"])
def test_conservation_and_on_shell_on_gpu(ctxs, torch, cfg):
    ctx, orc = ctxs[cfg]
    for chan in range(ctx.n_channels):
        y = ctx.uniform(77, 0, 0, 50000, ctx.dims[chan])
        out = ctx.map(chan, y)
        torch.cuda.synchronize()
        p = _np(out["p"])
        keep = _np(out["jac"]) > 0
        emax = np.abs(p[0]).max(axis=0)
        bal = np.abs(p[:, 0] + p[:, 1] - p[:, 2:].sum(axis=1)).max(axis=0)
        assert np.all(bal[keep] <= 1e-12 * emax[keep])
        m2 = p[0, 2:] ** 2 - p[1, 2:] ** 2 - p[2, 2:] ** 2 - p[3, 2:] ** 2
        assert np.all(np.abs(m2[:, keep]) <= 1e-12 * emax[keep] ** 2)


# --------------------------------------------------------------------------
# fused multichannel sample
# --------------------------------------------------------------------------

def _sample_case(ctxs, torch, cfg, counts, seed, offset=0):
    ctx, orc = ctxs[cfg]
    ctx.reset_stats()
    out = ctx.sample(counts, seed=seed, stream_id=2, counter_offset=offset)
    torch.cuda.synchronize()
    got = {k: _np(v) for k, v in out.items()}
    off = 0
    reps, stats_ref = {}, []
    for c, k in enumerate(counts):
        k = int(k)
        sl = slice(off, off + k)
        if k:
            y = W.philox_uniforms(seed, 2, offset + off, k, ctx.dims[c])
            ref = orc.map(c, y, orc.uniform_grid(c))
            fe = orc.forward_error(c, y, orc.uniform_grid(c), ref=ref)
            seg = {"w": got["w"][sl], "p": got["p"][:, :, sl],
                   "x1x2": None if got["x1x2"] is None else got["x1x2"][:, sl]}
            reps[c] = compare(seg, ref, fe, hadronic=ctx.hadronic[c], label=f"{cfg} sample ch{c}")
            assert np.all(got["chan"][sl] == c)
            stats_ref.append(oracle.channel_stats(ref["w"]))
        else:
            stats_ref.append(np.zeros(5))
        off += k
    return ctx, got, reps, np.array(stats_ref)


@pytest.mark.parametrize("cfg,counts", [
    ("c1", [70001]),
    ("c2", [30000, 0, 257, 1, 12345, 255, 256, 40001]),
    ("c3", [50021]),
])
def test_sample_parity_and_stats(ctxs, torch, cfg, counts):
    counts = np.array(counts, dtype=np.int64)
    ctx, got, reps, st_ref = _sample_case(ctxs, torch, cfg, counts, seed=11, offset=2**33 + 7)
    print(cfg, reps)
    st = ctx.stats()
    assert np.array_equal(st[:, 2], counts.astype(float))
    for c in range(len(counts)):
        if counts[c] == 0:
            assert np.all(st[c] == 0)
            continue
        assert st[c, 0] == pytest.approx(st_ref[c, 0], rel=1e-9)
        assert st[c, 1] == pytest.approx(st_ref[c, 1], rel=1e-9)
        assert st[c, 4] == pytest.approx(st_ref[c, 4], rel=1e-9)
        assert abs(st[c, 3] - st_ref[c, 3]) <= reps[c]["cut_flips"]


def test_sample_is_independent_of_batching(ctxs, torch):
    """Per-event outputs depend only on (seed, event id): one launch of all
    events equals two launches of the halves with the counter offset moved."""
    ctx, _ = ctxs["c2"]
    counts = np.array([1000, 2000, 0, 3000, 17, 0, 900, 5], dtype=np.int64)
    full = ctx.sample(counts, seed=5, stream_id=1, counter_offset=0)
    w_full = _np(full["w"]).copy()
    # the same events, channel by channel, each as its own launch
    off = 0
    for c, k in enumerate(counts):
        one = np.zeros_like(counts)
        one[c] = k
        part = ctx.sample(one, seed=5, stream_id=1, counter_offset=off)
        torch.cuda.synchronize()
        assert np.array_equal(_np(part["w"]), w_full[off:off + k])
        off += int(k)


@pytest.mark.parametrize("n", [1, 63, 64, 65, 256, 257])
def test_small_and_ragged_sizes(ctxs, torch, n):
    ctx, orc = ctxs["c3"]
    got, ref, fe = _map_case(ctxs, torch, "c3", 0, n, None, seed=900 + n)
    compare(got, ref, fe, hadronic=True, label=f"n={n}")


def test_empty_calls_are_no_ops(ctxs, torch):
    ctx, _ = ctxs["c2"]
    out = ctx.map(0, torch.empty((ctx.dims[0], 0), dtype=torch.float64, device=ctx.device))
    assert out["p"].numel() == 0
    s = ctx.sample(np.zeros(8, dtype=np.int64), seed=1)
    assert s["w"].numel() == 0


def test_extreme_uniforms(ctxs, torch):
    """Uniforms at the ends of (0, 1) and exactly 0 or 1 give finite results or
    a clean cut, never NaN weights."""
    ctx, orc = ctxs["c2"]
    vals = np.array([2.0 ** -53, 1e-300, 0.5, 1 - 2.0 ** -53, 0.0, 1.0])
    rng = np.random.default_rng(3)
    y_h = vals[rng.integers(0, len(vals), size=(ctx.dims[0], 4096))]
    y = torch.from_numpy(y_h).to(ctx.device)
    out = ctx.map(0, y, weight=True)
    torch.cuda.synchronize()
    w = _np(out["w"])
    assert np.all(np.isfinite(w)) and np.all(w >= 0)
    ref = orc.map(0, y_h, orc.uniform_grid(0))
    fe = orc.forward_error(0, y_h, orc.uniform_grid(0), ref=ref)
    compare({"w": w}, ref, fe, hadronic=True, label="extreme uniforms")


def test_bad_arguments_raise(ctxs, torch):
    from paper_2602_06895_amd import MsxError

    ctx, _ = ctxs["c2"]
    y = ctx.uniform(1, 0, 0, 10, 10)
    with pytest.raises(MsxError):
        ctx.map(8, y)
    # the C entry point validates the channel itself
    assert ctx.L.msx_map(ctx.h, 8, 10, y.data_ptr(), y.data_ptr(), None, y.data_ptr(), None, None) == 1
    assert b"out of range" in ctx.L.msx_last_error(ctx.h)
    with pytest.raises(MsxError):
        ctx.sample(np.array([-1, 0, 0, 0, 0, 0, 0, 0]), seed=1)
    bad = np.array([5, -1, 0, 0, 0, 0, 0, 0], dtype=np.int64)
    assert ctx.L.msx_sample(ctx.h, bad.ctypes.data, 1, 0, 0, 0, y.data_ptr(), y.data_ptr(), y.data_ptr(),
                            None, None) == 1
    good = np.array([5, 0, 0, 0, 0, 0, 0, 0], dtype=np.int64)
    assert ctx.L.msx_sample(ctx.h, good.ctypes.data, 1, 0, 0, 64, y.data_ptr(), y.data_ptr(), y.data_ptr(),
                            None, None) == 1
    assert b"flags" in ctx.L.msx_last_error(ctx.h)
    with pytest.raises(MsxError):
        ctx.vegas_update(alpha=-1.0)
    with pytest.raises(ValueError):
        ctx.set_grid(0, np.zeros((3, 3)))


# --------------------------------------------------------------------------
# VEGAS adaptation
# --------------------------------------------------------------------------

def test_vegas_histogram_and_refinement_match_oracle(ctxs, torch):
    ctx, orc = ctxs["c2"]
    chan = 3
    n = 200003
    d, nb = ctx.dims[chan], ctx.nbins[chan]
    grid = orc.uniform_grid(chan)
    for it in range(3):
        y = ctx.uniform(40 + it, 1, 0, n, d)
        m = ctx.map(chan, y, weight=True)
        ctx.vegas_accumulate(chan, y, m["w"])
        ctx.vegas_update(alpha=0.5)
        torch.cuda.synchronize()
        y_h = _np(y)
        ref = orc.map(chan, y_h, grid)
        hist = oracle.vegas_histogram(y_h, ref["w"], nb)
        grid = oracle.vegas_refine(grid, hist, alpha=0.5)
        g = ctx.get_grid(chan)
        assert np.all(np.diff(g, axis=1) > 0) and np.all(g[:, 0] == 0) and np.all(g[:, -1] == 1)
        assert np.abs(g - grid).max() <= 1e-10, f"iteration {it}: {np.abs(g - grid).max():.3e}"
        grid = g  # continue from the device grid (differences stay at rounding level)
    # other channels untouched: empty histograms keep the grid
    assert np.array_equal(ctx.get_grid(0), orc.uniform_grid(0))
    ctx.set_grid(chan, orc.uniform_grid(chan))


# --------------------------------------------------------------------------
# Unweighting efficiency
# --------------------------------------------------------------------------

@pytest.mark.parametrize("kind", ["exp", "ties", "zeros", "tiny", "subnormal", "spread", "one"])
def test_unweighting_efficiency_matches_oracle(ctxs, torch, kind):
    ctx, _ = ctxs["c2"]
    rng = np.random.default_rng(8)
    if kind == "exp":
        w = rng.exponential(size=1_000_003)
    elif kind == "ties":
        w = rng.integers(1, 20, size=100000).astype(np.float64)
    elif kind == "zeros":
        w = np.where(rng.random(300000) < 0.7, 0.0, rng.random(300000) ** 4)
    elif kind == "tiny":
        w = rng.random(5000) * 1e-290
    elif kind == "subnormal":
        w = rng.random(5000) * 1e-310
    elif kind == "spread":
        w = rng.exponential(size=2_000_001) * 10.0 ** rng.uniform(-30, 30, size=2_000_001)
    else:
        w = np.array([2.5])
    eff_o, W_o = oracle.unweighting_efficiency(w, 1e-3)
    wd = torch.from_numpy(w).to(ctx.device)
    eff_g, W_g = ctx.unweight_eff(wd, 1e-3)
    assert W_g == pytest.approx(W_o, rel=1e-12)
    assert eff_g == pytest.approx(eff_o, rel=1e-12)
    # integer bucket sums: the same bits on every call
    eff_2, W_2 = ctx.unweight_eff(wd, 1e-3)
    assert (eff_2, W_2) == (eff_g, W_g)


# --------------------------------------------------------------------------
# Physics pins on the GPU path
# --------------------------------------------------------------------------

def test_gpu_multichannel_volume(torch):
    """All eight 2->4 topologies at fixed sqrt(s) = 1 TeV with f = 1 and local
    channel weights: the sum of channel means is the massless volume."""
    from paper_2602_06895_amd import Context

    ctx = Context(W.volume_process(4, alpha_mu=10.0))
    counts = np.full(8, 400000, dtype=np.int64)
    out = ctx.sample(counts, seed=21)
    torch.cuda.synchronize()
    st = ctx.stats()
    I, err = oracle.integral(st)
    E = 1000.0
    exact = E ** 4 / (math.gamma(4) * math.gamma(3) * math.pi ** 5 * 2 ** 11)
    assert abs(I - exact) < 4 * err
    ctx.close()


def test_full_size_c2_sample_spot_check(ctxs, torch):
    """The benchmark workload (pp -> 4 jets, 8 channels, 1e7 events) in the
    launch configuration bench.py times; windows of events at random positions
    are recomputed by the oracle."""
    ctx, orc = ctxs["c2"]
    counts = np.full(8, 1_250_000, dtype=np.int64)
    # the shape bench.py runs: autotuned for these counts
    ctx.autotune(counts, seed=1, reps=1)
    out = ctx.sample(counts, seed=1, stream_id=0)
    torch.cuda.synchronize()
    ctx.set_launch(1, 0)
    ctx.reset_stats()
    rng = np.random.default_rng(4)
    w = out["w"]
    for _ in range(6):
        c = int(rng.integers(0, 8))
        start = int(rng.integers(0, counts[c] - 3000))
        pos = int(counts[:c].sum()) + start
        y = W.philox_uniforms(1, 0, pos, 3000, ctx.dims[c])
        ref = orc.map(c, y, orc.uniform_grid(c))
        fe = orc.forward_error(c, y, orc.uniform_grid(c), ref=ref)
        seg = {"w": _np(w[pos:pos + 3000]), "p": _np(out["p"][:, :, pos:pos + 3000]),
               "x1x2": _np(out["x1x2"][:, pos:pos + 3000])}
        compare(seg, ref, fe, hadronic=True, label=f"full-size ch{c}@{start}")


def test_full_size_c3_sample_spot_check(ctxs, torch):
    """pp -> t tbar -> 6 at its full size (1e8 events in one fused launch, 16
    dims, Breit-Wigner maps): windows of events at random positions, the
    first and the last events, recomputed by the oracle."""
    ctx, orc = ctxs["c3"]
    N = 100_000_000
    out = ctx.sample(np.array([N]), seed=3, stream_id=0, want_chan=False)
    torch.cuda.synchronize()
    rng = np.random.default_rng(6)
    starts = [0, N - 2000] + [int(rng.integers(0, N - 2000)) for _ in range(4)]
    for start in starts:
        y = W.philox_uniforms(3, 0, start, 2000, ctx.dims[0])
        ref = orc.map(0, y, orc.uniform_grid(0))
        fe = orc.forward_error(0, y, orc.uniform_grid(0), ref=ref)
        seg = {"w": _np(out["w"][start:start + 2000]), "p": _np(out["p"][:, :, start:start + 2000]),
               "x1x2": _np(out["x1x2"][:, start:start + 2000])}
        compare(seg, ref, fe, hadronic=True, label=f"c3 full-size @{start}")
    del out
    torch.cuda.empty_cache()
    ctx.reset_stats()
