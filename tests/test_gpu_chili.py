"""Chili channels (section 2.4) on the GPU against the oracle: per-event
momenta, momentum fractions, Jacobians and weights through the map and the
fused multichannel sample (also mixed with tree channels under local channel
weights), the closed-form hadronic volume, and the refused inverse."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from parity import compare

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t

    if not t.cuda.is_available():
        pytest.skip("needs a GPU")
    return t


def _pp4j_chili():
    d = W.c2_pp4j()
    d["channels"] = [{"chili": True}]
    return d


CASES = [
    ("pp4j", _pp4j_chili, False),
    ("n3 no cut, massive", lambda: W.chili_process(3, 1000.0, masses=[0.0, 10.0, 80.0], pdf=[-1.2, 3.0]), True),
    ("n6 cut", lambda: W.chili_process(6, 13000.0, masses=[4.7, 0.0, 0.0, 4.7, 0.0, 0.0], pt_min=20.0,
                                       pdf=[-1.2, 3.0]), False),
    ("n8 cut", lambda: W.chili_process(8, 13000.0, pt_min=20.0), True),
]


def _random_grid(d, nb, seed):
    rng = np.random.default_rng(seed)
    g = np.empty((d, nb + 1))
    for k in range(d):
        g[k] = np.concatenate([[0.0], np.sort(rng.random(nb - 1)), [1.0]])
    return g


@pytest.mark.parametrize("name,mk,vegas", CASES)
def test_chili_map_matches_oracle(torch, name, mk, vegas):
    from paper_2602_06895_amd import Context

    desc = mk()
    ctx = Context(desc)
    orc = oracle.Process(desc)
    d = ctx.dims[0]
    assert d == orc.dims[0] == 3 * orc.n - 2
    grid = _random_grid(d, orc.nbins, 5) if vegas else orc.uniform_grid(0)
    ctx.set_grid(0, grid)
    y = W.philox_uniforms(19, 2, 0, 20001, d)  # several tiles and a ragged tail
    out = ctx.map(0, torch.from_numpy(y).cuda(), weight=True)
    torch.cuda.synchronize()
    ref = orc.map(0, y, grid)
    fe = orc.forward_error(0, y, grid, ref=ref)
    got = {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
    compare(got, ref, fe, hadronic=True, label=f"Chili {name}")
    assert (ref["jac"] > 0).mean() > 0.5
    ctx.close()


def test_chili_with_tree_channels_in_sample(torch):
    """The eight pp -> 4 jets tree channels plus a Chili channel under local
    channel weights (the Chili channel has no propagators: its weight
    factor is 1), through the fused multichannel sample."""
    from paper_2602_06895_amd import Context

    desc = W.c2_pp4j()
    desc["channels"] = desc["channels"] + [{"chili": True}]
    ctx = Context(desc)
    orc = oracle.Process(desc)
    counts = np.array([3000, 0, 257, 1, 1000, 255, 256, 999, 20001], dtype=np.int64)
    seed, offset = 13, 2 ** 32 + 3
    out = ctx.sample(counts, seed=seed, stream_id=4, counter_offset=offset)
    torch.cuda.synchronize()
    got = {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
    off = 0
    for c, k in enumerate(counts):
        k = int(k)
        if k:
            sl = slice(off, off + k)
            y = W.philox_uniforms(seed, 4, offset + off, k, ctx.dims[c])
            ref = orc.map(c, y, orc.uniform_grid(c))
            fe = orc.forward_error(c, y, orc.uniform_grid(c), ref=ref)
            seg = {"w": got["w"][sl], "p": got["p"][:, :, sl], "x1x2": got["x1x2"][:, sl]}
            compare(seg, ref, fe, hadronic=True, label=f"tree + Chili sample ch{c}")
            assert np.all(got["chan"][sl] == c)
        off += k
    ctx.close()


def test_chili_volume(torch):
    """f = 1, no cut: the mean weight of 4e6 massless 2 -> 2 and 2 -> 3 events
    against int dtau (-log tau) Phi_n(tau s)."""
    from paper_2602_06895_amd import Context

    for n in (2, 3):
        ctx = Context(W.chili_process(n, 1000.0))
        y = ctx.uniform(3, n, 0, 4_000_000, ctx.dims[0])
        w = ctx.map(0, y, weight=True)["w"]
        torch.cuda.synchronize()
        m, e = float(w.mean()), float(w.std()) / math.sqrt(w.numel())
        phi = (2 * math.pi) ** (4 - 3 * n) * (math.pi / 2) ** (n - 1) / (math.factorial(n - 1) * math.factorial(n - 2))
        exact = phi * 1e6 ** (n - 2) / (n - 1) ** 2
        assert abs(m - exact) < 4.0 * e and e < 0.05 * exact, (n, m, e, exact)
        ctx.close()


def test_chili_refusals(torch):
    from paper_2602_06895_amd import Context, MsxError

    ctx = Context(_pp4j_chili())
    p = torch.zeros(4, 6, 8, dtype=torch.float64, device="cuda")
    x = torch.full((2, 8), 0.5, dtype=torch.float64, device="cuda")
    with pytest.raises(MsxError):
        ctx.inverse_map(0, p, x)
    with pytest.raises(MsxError):
        ctx.multichannel_density(0, p, x, np.ones(1))
    ctx.close()
    d = W.chili_process(3)
    d["beams"] = "fixed"
    with pytest.raises(MsxError):
        Context(d)
