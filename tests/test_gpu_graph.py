"""The persistent multichannel launch: launch-shape invariance, device-resident
counts, HIP-graph capture and replay, the autotuner, and the 24-channel
batch with power-law event counts."""
import numpy as np
import pytest

import oracle
import workloads as W
from parity import compare

pytestmark = pytest.mark.gpu

C2_COUNTS = [300, 0, 257, 1, 1000, 64, 65, 500]


@pytest.fixture(scope="module")
def torch():
    import torch as t

    if not t.cuda.is_available():
        pytest.skip("needs a GPU")
    return t


@pytest.fixture(scope="module")
def c2(torch):
    from paper_2602_06895_amd import Context

    ctx = Context(W.c2_pp4j())
    yield ctx
    ctx.close()


def _host_sample(ctx, counts, seed, sid, off):
    out = ctx.sample(np.asarray(counts), seed=seed, stream_id=sid, counter_offset=off)
    return {k: (v.clone() if v is not None else None) for k, v in out.items()}


def test_results_do_not_depend_on_the_launch_shape(torch, c2):
    ref = None
    stats = []
    for ept, grid in [(1, 0), (2, 512), (4, 256), (1, 3), (3, 1)]:
        c2.set_launch(ept, grid)
        c2.reset_stats()
        out = _host_sample(c2, C2_COUNTS, 5, 2, 1000)
        stats.append(c2.stats())
        torch.cuda.synchronize()
        if ref is None:
            ref = out
            continue
        for k in ("p", "w", "x1x2", "chan"):
            assert torch.equal(out[k], ref[k]), (ept, grid, k)
    c2.set_launch(1, 0)
    for s in stats[1:]:
        assert np.array_equal(s[:, 2:4], stats[0][:, 2:4])
        assert np.allclose(s, stats[0], rtol=1e-12, atol=0)


def test_device_counts_match_host_counts(torch, c2):
    cap = 4000
    buf = c2.sample_buffers(cap)
    counts = torch.tensor(C2_COUNTS, dtype=torch.int64, device="cuda")
    off = torch.tensor([777], dtype=torch.int64, device="cuda")
    status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    c2.sample_device(counts, 9, 4, off, buf, status)
    ref = _host_sample(c2, C2_COUNTS, 9, 4, 777)
    torch.cuda.synchronize()
    n = sum(C2_COUNTS)
    assert int(status.cpu()[0]) == 0
    assert torch.equal(buf["w"][:n], ref["w"]) and torch.equal(buf["chan"][:n], ref["chan"])
    assert torch.equal(buf["p"][:, :, :n], ref["p"]) and torch.equal(buf["x1x2"][:, :n], ref["x1x2"])
    # more events than the buffers hold: nothing sampled, status set
    buf["w"].fill_(-7.0)
    big = torch.tensor([cap, 1, 0, 0, 0, 0, 0, 0], dtype=torch.int64, device="cuda")
    c2.sample_device(big, 9, 4, off, buf, status)
    torch.cuda.synchronize()
    assert int(status.cpu()[0]) == 1 and bool((buf["w"] == -7.0).all())
    neg = torch.tensor([5, -1, 0, 0, 0, 0, 0, 0], dtype=torch.int64, device="cuda")
    c2.sample_device(neg, 9, 4, off, buf, status)
    torch.cuda.synchronize()
    assert int(status.cpu()[0]) == 1 and bool((buf["w"] == -7.0).all())


def test_graph_replays_match_eager_launches(torch, c2):
    cap = 5000
    buf = c2.sample_buffers(cap)
    counts = torch.zeros(8, dtype=torch.int64, device="cuda")
    off = torch.zeros(1, dtype=torch.int64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    g = c2.sample_graph(counts, 11, 6, off, buf, status)
    cases = [(C2_COUNTS, 0), ([1000, 1000, 0, 0, 7, 0, 0, 1], 12345), ([0, 0, 0, 0, 0, 0, 0, 4999], 2 ** 40)]
    for cc, o in cases:
        counts.copy_(torch.tensor(cc, dtype=torch.int64))
        off.fill_(o)
        g.launch()
        torch.cuda.synchronize()
        got = {k: buf[k].clone() for k in ("p", "w", "x1x2", "chan")}
        # eager work between replays, then the reference
        ref = _host_sample(c2, cc, 11, 6, o)
        torch.cuda.synchronize()
        n = sum(cc)
        assert int(status.cpu()[0]) == 0
        assert torch.equal(got["w"][:n], ref["w"]), cc
        assert torch.equal(got["chan"][:n], ref["chan"])
        assert torch.equal(got["p"][:, :, :n], ref["p"])
        assert torch.equal(got["x1x2"][:, :n], ref["x1x2"])
    g.close()


def test_graph_statistics_accumulate_like_eager_calls(torch, c2):
    cap = 3000
    buf = c2.sample_buffers(cap, want_chan=False)
    counts = torch.tensor(C2_COUNTS, dtype=torch.int64, device="cuda")
    off = torch.zeros(1, dtype=torch.int64, device="cuda")
    g = c2.sample_graph(counts, 13, 1, off, buf)
    c2.reset_stats()
    for r in range(3):
        off.fill_(r * 5000)
        g.launch()
    torch.cuda.synchronize()
    sg = c2.stats()
    c2.reset_stats()
    for r in range(3):
        c2.sample(np.asarray(C2_COUNTS), seed=13, stream_id=1, counter_offset=r * 5000)
    se = c2.stats()
    assert np.array_equal(sg[:, 2:4], se[:, 2:4])
    assert np.allclose(sg, se, rtol=1e-12, atol=0)
    g.close()
    c2.reset_stats()


def test_autotune_picks_a_candidate_and_keeps_results(torch, c2):
    counts = np.array([20000] * 8)
    before = _host_sample(c2, counts, 3, 3, 0)
    c2.reset_stats()
    ms = c2.autotune(counts, seed=3, reps=2)
    ept, grid = c2.launch_shape()
    assert ms > 0 and ept in (1, 2, 4)
    cu = torch.cuda.get_device_properties(0).multi_processor_count
    assert grid in (2 * cu, 4 * cu, 8 * cu, 16 * cu)
    assert np.all(c2.stats() == 0)
    after = _host_sample(c2, counts, 3, 3, 0)
    torch.cuda.synchronize()
    for k in ("p", "w", "x1x2", "chan"):
        assert torch.equal(after[k], before[k])
    c2.set_launch(1, 0)
    c2.reset_stats()


def test_c4_batch_in_one_graph(torch):
    """24 channels (C1 and C2 topologies, 6 processes), power-law counts, one
    persistent launch replayed from a graph; every channel's events equal the
    single-channel map of the same uniforms, and the oracle's within the
    per-event parity bound."""
    from paper_2602_06895_amd import Context

    desc, counts = W.c4_context()
    ctx = Context(desc)
    assert ctx.n_channels == 24
    N = int(counts.sum())
    buf = ctx.sample_buffers(N)
    dc = torch.from_numpy(counts.astype(np.int64)).cuda()
    off = torch.zeros(1, dtype=torch.int64, device="cuda")
    g = ctx.sample_graph(dc, 4, 8, off, buf)
    ctx.reset_stats()
    g.launch()
    torch.cuda.synchronize()
    st = ctx.stats()
    assert np.array_equal(st[:, 2], counts.astype(float))
    start = np.concatenate([[0], np.cumsum(counts)])
    chan = buf["chan"].cpu().numpy()
    for c in range(24):
        assert np.all(chan[start[c]:start[c + 1]] == c)
    # spot check: a slice of every channel against msx_map of its uniforms
    for c in range(24):
        lo, hi = int(start[c]), int(min(start[c + 1], start[c] + 300))
        y = ctx.uniform(4, 8, lo, hi - lo, ctx.dims[c])
        ref = ctx.map(c, y, weight=True)
        torch.cuda.synchronize()
        np_ = ctx.n_momenta[c]
        assert torch.equal(buf["w"][lo:hi], ref["w"]), c
        assert torch.equal(buf["p"][:, :np_, lo:hi], ref["p"]), c
        if ctx.hadronic[c]:
            assert torch.equal(buf["x1x2"][:, lo:hi], ref["x1x2"]), c
    assert np.allclose(st[:, 0], [float(buf["w"][start[c]:start[c + 1]].sum()) for c in range(24)], rtol=1e-11)
    # and against the oracle: each context channel is channel j of one of the
    # six processes, whose oracle has that process's channels (the local
    # channel weights); the per-event bound of the parity tests
    procs = desc["processes"]
    owner = [(p, j) for p, d in enumerate(procs) for j in range(len(d["channels"]))]
    orcs = [oracle.Process(d) for d in procs]
    for c in range(24):
        p, j = owner[c]
        lo, hi = int(start[c]), int(min(start[c + 1], start[c] + 2000))
        y = W.philox_uniforms(4, 8, lo, hi - lo, ctx.dims[c])
        ref = orcs[p].map(j, y, orcs[p].uniform_grid(j))
        fe = orcs[p].forward_error(j, y, orcs[p].uniform_grid(j), ref=ref)
        np_ = ctx.n_momenta[c]
        got = {"w": buf["w"][lo:hi].cpu().numpy(), "p": buf["p"][:, :np_, lo:hi].cpu().numpy(),
               "x1x2": buf["x1x2"][:, lo:hi].cpu().numpy() if ctx.hadronic[c] else None}
        compare(got, ref, fe, hadronic=ctx.hadronic[c], label=f"c4 graph channel {c}")
    g.close()
    ctx.close()


def test_graph_with_chili_and_three_body_channels(torch):
    """A process whose channels need the extended kind class (Chili and a
    1 -> 3 decay beside tree channels): graph replays equal eager launches."""
    from paper_2602_06895_amd import Context

    desc = W.c2_pp4j()
    # (the cluster of particles 2, 3, 4 is massless in the tree channels too)
    desc["channels"] = desc["channels"] + [{"chili": True}, {"t_chain": [1, {"d": [2, 3, 4]}], "t_order": ""}]
    ctx = Context(desc)
    cap = 6000
    buf = ctx.sample_buffers(cap)
    counts = torch.zeros(10, dtype=torch.int64, device="cuda")
    off = torch.zeros(1, dtype=torch.int64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    g = ctx.sample_graph(counts, 17, 3, off, buf, status)
    for cc, o in [([300, 0, 257, 1, 1000, 64, 65, 500, 2000, 999], 0), ([0] * 8 + [4097, 1], 99)]:
        counts.copy_(torch.tensor(cc, dtype=torch.int64))
        off.fill_(o)
        g.launch()
        torch.cuda.synchronize()
        got = {k: buf[k].clone() for k in ("p", "w", "x1x2", "chan")}
        ref = _host_sample(ctx, cc, 17, 3, o)
        torch.cuda.synchronize()
        n = sum(cc)
        assert int(status.cpu()[0]) == 0
        for k in ("w", "chan"):
            assert torch.equal(got[k][:n], ref[k]), (cc, k)
        assert torch.equal(got["p"][:, :, :n], ref["p"]) and torch.equal(got["x1x2"][:, :n], ref["x1x2"])
    g.close()
    ctx.close()
