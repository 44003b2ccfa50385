"""VEGAS adaptation inside the fused sample (MSX_SAMPLE_ACCUMULATE_VEGAS):
the histograms of sum w^2 per bin that the sample kernel accumulates, and the
grids refined from them, against the oracle's histogram and refinement of the
same events (uniforms regenerated on the host from the same Philox ids, the
oracle's own weights).  Tolerance: grids within 1e-10 (the per-event weights
agree to ~1e-12 relative and the histogram sums differ only in summation
order), per iteration, continuing from the device grid."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t

    if not t.cuda.is_available():
        pytest.skip("needs a GPU")
    return t


def _oracle_refine(orc, ctx, grids, counts, seed, sid, offset, alpha):
    """Oracle histograms and refined grids of one fused sample's events."""
    new = []
    off = offset
    for c, k in enumerate(counts):
        d, nb = ctx.dims[c], ctx.nbins[c]
        if k == 0:
            new.append(grids[c])
            continue
        y = W.philox_uniforms(seed, sid, off, int(k), d)
        ref = orc.map(c, y, grids[c])
        hist = oracle.vegas_histogram(y, ref["w"], nb)
        new.append(oracle.vegas_refine(grids[c], hist, alpha))
        off += int(k)
    return new


@pytest.mark.parametrize("cfg,counts,ept", [
    ("c2", [3000, 0, 257, 1, 1000, 64, 65, 50003], 1),
    ("c2", [20000, 20000, 20000, 20000, 20000, 20000, 20000, 20000], 4),
    ("c3", [60001], 2),
    ("c1", [4099], 1),
])
def test_fused_accumulation_matches_oracle(torch, cfg, counts, ept):
    from paper_2602_06895_amd import SAMPLE_ACCUMULATE_VEGAS, Context

    desc = {"c1": W.c1_ee_mumu, "c2": W.c2_pp4j, "c3": W.c3_ttbar6}[cfg]()
    ctx = Context(desc)
    orc = oracle.Process(desc)
    ctx.set_launch(ept, 0)
    counts = np.array(counts, dtype=np.int64)
    grids = [orc.uniform_grid(c) for c in range(ctx.n_channels)]
    iters = 10 if cfg != "c2" or ept == 4 else 4
    for it in range(iters):
        seed, sid, off = 100 + it, 3, 1000 * it
        ctx.sample(counts, seed=seed, stream_id=sid, counter_offset=off, flags=SAMPLE_ACCUMULATE_VEGAS)
        ctx.vegas_update(alpha=0.5)
        torch.cuda.synchronize()
        want = _oracle_refine(orc, ctx, grids, counts, seed, sid, off, 0.5)
        for c in range(ctx.n_channels):
            g = ctx.get_grid(c)
            assert np.all(np.diff(g, axis=1) > 0) and np.all(g[:, 0] == 0) and np.all(g[:, -1] == 1)
            err = np.abs(g - want[c]).max()
            assert err <= 1e-10, f"{cfg} iteration {it} channel {c}: grid differs by {err:.3e}"
            if counts[c] == 0:
                assert np.array_equal(g, grids[c]), "a channel without events must keep its grid"
        grids = [ctx.get_grid(c) for c in range(ctx.n_channels)]
    ctx.close()


def test_accumulation_is_deterministic_and_graph_equals_eager(torch):
    """Same events, same launch shape: bit-identical grids from two eager
    accumulating samples and from a captured graph replay (device counts);
    the events themselves equal a plain sample's."""
    from paper_2602_06895_amd import SAMPLE_ACCUMULATE_VEGAS, Context

    counts = np.array([5000, 7, 0, 3000, 1025, 1, 2000, 999], dtype=np.int64)
    desc = W.c2_pp4j()
    res = []
    for mode in ("eager", "eager", "graph"):
        ctx = Context(desc)
        ctx.set_launch(2, 0)
        if mode == "eager":
            out = ctx.sample(counts, seed=9, stream_id=2, counter_offset=17, flags=SAMPLE_ACCUMULATE_VEGAS)
        else:
            cap = int(counts.sum()) + 4096
            buf = ctx.sample_buffers(cap)
            dc = torch.from_numpy(counts).to(ctx.device)
            off = torch.tensor([17], dtype=torch.int64, device=ctx.device)
            g = ctx.sample_graph(dc, 9, 2, off, buf, flags=SAMPLE_ACCUMULATE_VEGAS)
            g.launch()
            out = buf
        ctx.vegas_update(alpha=0.7)
        torch.cuda.synchronize()
        N = int(counts.sum())
        res.append(([ctx.get_grid(c) for c in range(8)], out["w"][:N].cpu().numpy(), ctx.stats()))
        plain = Context(desc)
        ref = plain.sample(counts, seed=9, stream_id=2, counter_offset=17)
        torch.cuda.synchronize()
        assert np.array_equal(res[-1][1], ref["w"].cpu().numpy()), "accumulation changed the events"
        plain.close()
        if mode == "graph":
            g.close()
        ctx.close()
    for k in (1, 2):
        for c in range(8):
            assert np.array_equal(res[0][0][c], res[k][0][c]), f"run {k} channel {c}: grids differ"
        assert np.array_equal(res[0][1], res[k][1])


def test_library_adaptation_matches_oracle_loop(torch):
    """msx_vegas_adapt (the library's adaptation phase) equals the oracle's
    loop over the same events: sample, histogram, refine, for 3 iterations;
    the returned statistics are those of the last iteration."""
    from paper_2602_06895_amd import Context, adapt_vegas

    desc = W.c2_pp4j()
    ctx = Context(desc)
    orc = oracle.Process(desc)
    n, iters, seed, sid = 20011, 3, 5, 1
    st = adapt_vegas(ctx, n_per_channel=n, iterations=iters, alpha=0.5, seed=seed, stream_id=sid)
    torch.cuda.synchronize()
    C = ctx.n_channels
    grids = [orc.uniform_grid(c) for c in range(C)]
    counts = np.full(C, n, dtype=np.int64)
    for it in range(iters):
        prev = grids
        grids = _oracle_refine(orc, ctx, grids, counts, seed, sid, it * C * n, 0.5)
    for c in range(C):
        assert np.abs(ctx.get_grid(c) - grids[c]).max() <= 1e-9, f"channel {c}"
    # statistics of the last iteration's events (drawn from the grids before its refinement)
    for c in range(C):
        y = W.philox_uniforms(seed, sid, (iters - 1) * C * n + c * n, n, ctx.dims[c])
        w = orc.map(c, y, prev[c])["w"]
        want = oracle.channel_stats(w)
        assert st[c, 2] == n and st[c, 3] == want[3]
        assert abs(st[c, 0] - want[0]) <= 1e-9 * abs(want[0])
        assert abs(st[c, 1] - want[1]) <= 1e-9 * abs(want[1])
    assert np.all(ctx.stats() == 0.0), "adaptation leaves the statistics reset"
    ctx.close()


def test_accumulate_rejections(torch):
    from paper_2602_06895_amd import SAMPLE_USE_FLOW, Context, MsxError

    ctx = Context(W.c2_pp4j())
    with pytest.raises(MsxError, match="flow"):
        ctx.sample(np.full(8, 10, dtype=np.int64), seed=1, flags=SAMPLE_USE_FLOW)
    with pytest.raises(MsxError, match="flags"):
        ctx.sample(np.full(8, 10, dtype=np.int64), seed=1, flags=1 << 7)
    ctx.close()
