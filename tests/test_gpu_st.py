"""The (s~, t) double-invariant block (section 2.2.5) on the GPU: t-chain
channels with "st" against the oracle, per event (the forward-error bound of
tests/parity.py), in the fused sample beside (phi, t) channels, through the
inverse map, and by the massless phase-space volume."""
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


def _lepton(n, chain, order):
    d = W.rambo_process(n, rambo=False)
    d["channels"] = [{"t_chain": chain, "t_order": order, "st": True}]
    return d


def _hadronic():
    d = W.c2_pp4j()
    d["channels"] = [{"t_chain": [1, 2, 3, 4], "t_order": "AA", "st": True},
                     {"t_chain": [1, 2, 4, 3], "t_order": "AB", "st": True},
                     {"t_chain": [4, 3, 2, 1], "t_order": "BB"}]
    return d


@pytest.mark.parametrize("case", ["lepton4AA", "lepton5AB", "hadronic"])
def test_map_parity(torch, case):
    from paper_2602_06895_amd import Context

    desc = {"lepton4AA": lambda: _lepton(4, [1, 2, 3, 4], "AA"),
            "lepton5AB": lambda: _lepton(5, [1, 2, 5, 3, 4], "ABA"),
            "hadronic": _hadronic}[case]()
    ctx = Context(desc)
    orc = oracle.Process(desc)
    for chan in range(ctx.n_channels):
        n = 30011
        y_h = W.philox_uniforms(21, chan, 0, n, ctx.dims[chan])
        y = torch.from_numpy(y_h).cuda()
        got = ctx.map(chan, y, weight=True)
        torch.cuda.synchronize()
        ref = orc.map(chan, y_h, orc.uniform_grid(chan))
        fe = orc.forward_error(chan, y_h, orc.uniform_grid(chan), ref=ref)
        rep = compare({k: (v.cpu().numpy() if v is not None else None) for k, v in got.items()}, ref, fe,
                      hadronic=ctx.hadronic[chan], label=f"st {case} ch{chan}")
        print(case, chan, rep)
    ctx.close()


def test_sample_parity_beside_phi_t_channels(torch):
    from paper_2602_06895_amd import Context

    desc = _hadronic()
    ctx = Context(desc)
    orc = oracle.Process(desc)
    counts = np.array([20001, 257, 3000], dtype=np.int64)
    out = ctx.sample(counts, seed=5, stream_id=3, counter_offset=77)
    torch.cuda.synchronize()
    got = {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
    off = 0
    for c, k in enumerate(counts):
        k = int(k)
        sl = slice(off, off + k)
        y = W.philox_uniforms(5, 3, 77 + off, k, ctx.dims[c])
        ref = orc.map(c, y, orc.uniform_grid(c))
        fe = orc.forward_error(c, y, orc.uniform_grid(c), ref=ref)
        compare({"w": got["w"][sl], "p": got["p"][:, :, sl], "x1x2": got["x1x2"][:, sl]}, ref, fe, hadronic=True,
                label=f"st sample ch{c}")
        assert np.all(got["chan"][sl] == c)
        off += k
    ctx.close()


def test_inverse_matches_oracle(torch):
    from paper_2602_06895_amd import Context

    desc = _lepton(4, [1, 2, 3, 4], "AA")
    ctx = Context(desc)
    orc = oracle.Process(desc)
    y = W.philox_uniforms(31, 0, 0, 20011, ctx.dims[0])
    ev = orc.map(0, y)
    ok = ev["jac"] > 0
    p = np.ascontiguousarray(ev["p"][:, :, ok])
    ref = orc.inverse(0, p, None)
    fe = orc.inverse_forward_error(0, p, None, ref=ref)
    got = ctx.inverse_map(0, torch.from_numpy(p).cuda())
    torch.cuda.synchronize()
    yg = got["y"].cpu().numpy()
    fin = np.isfinite(ref["y"]).all(axis=0)
    assert np.array_equal(fin, np.isfinite(yg).all(axis=0))
    dy = np.abs(yg[:, fin] - ref["y"][:, fin]).max(axis=0)
    assert np.all(dy <= np.maximum(1e-12, 100.0 * fe["y"][fin])), float(np.max(dy / np.maximum(fe["y"][fin], 1e-300)))
    assert np.median(dy) < 1e-13
    ctx.close()


def test_massless_volume(torch):
    """Massless 2 -> 4 at 1 TeV, unit integrand: the mean weight of 4e6 events
    equals (2 pi)^(4 - 3n) (pi/2)^(n-1) s^(n-2) / ((n-1)! (n-2)!) within 4
    standard errors."""
    from paper_2602_06895_amd import Context

    n = 4
    ctx = Context(_lepton(n, [1, 2, 3, 4], "AA"))
    y = ctx.uniform(3, 1, 0, 4_000_000, ctx.dims[0])
    w = ctx.map(0, y, weight=True)["w"]
    torch.cuda.synchronize()
    m, e = float(w.mean()), float(w.std()) / math.sqrt(w.numel())
    s = 1e6
    V = (2 * math.pi) ** (4 - 3 * n) * (math.pi / 2) ** (n - 1) * s ** (n - 2) / (math.factorial(n - 1) *
                                                                                  math.factorial(n - 2))
    assert abs(m - V) < 4 * e, (m / V, e / V)
    ctx.close()
