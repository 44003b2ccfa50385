"""1 -> 3 decays (section 2.2.6) on the GPU against the oracle: per-event
momenta, Jacobians and weights through the map and the fused multichannel
sample, with the decay at the root, below a two-body decay, above one and
on a hadronic t-channel spine; the massless three-body volume; the inverse
map and its round trip."""
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


def _fixed(chan, masses):
    d = W.volume_process(len(masses), sqrt_s=1000.0, channels=[chan])
    d["masses"] = [float(m) for m in masses]
    return d


def _hadronic(chans, masses, alpha_mu=None):
    d = W.chili_process(len(masses), sqrt_s=13000.0, masses=masses, pt_min=20.0, pdf=[-1.2, 3.0])
    d["shat_min"] = 6400.0
    d["channels"] = chans
    if alpha_mu is not None:
        d["alpha_mu"] = alpha_mu
    return d


CASES = [
    ("root massive", lambda: _fixed({"s": {"d": [1, 2, 3]}}, [10.0, 80.0, 173.0]), False),
    ("below a two-body decay", lambda: _fixed({"s": {"d": [{"d": [1, 2, 3], "m": 173.0, "w": 1.5}, 4]}},
                                              [4.7, 0.0, 0.0, 4.7]), True),
    ("above a two-body decay", lambda: _fixed({"s": {"d": [1, {"d": [2, 3], "m": 80.4, "w": 2.1}, 4]}},
                                              [0.0] * 4), False),
    ("t-channel spine", lambda: _hadronic([{"t_chain": [1, {"d": [2, 3, 4], "m": 300.0, "w": 20.0}],
                                            "t_order": ""}], [0.0] * 4), True),
]


def _random_grid(d, nb, seed):
    rng = np.random.default_rng(seed)
    g = np.empty((d, nb + 1))
    for k in range(d):
        g[k] = np.concatenate([[0.0], np.sort(rng.random(nb - 1)), [1.0]])
    return g


@pytest.mark.parametrize("name,mk,vegas", CASES)
def test_dec3_map_and_inverse_match_oracle(torch, name, mk, vegas):
    from paper_2602_06895_amd import Context

    desc = mk()
    ctx = Context(desc)
    orc = oracle.Process(desc)
    d = ctx.dims[0]
    assert d == orc.dims[0]
    grid = _random_grid(d, orc.nbins, 3) if vegas else orc.uniform_grid(0)
    ctx.set_grid(0, grid)
    had = orc.hadronic
    y = W.philox_uniforms(29, 3, 0, 20001, d)
    out = ctx.map(0, torch.from_numpy(y).cuda(), weight=True)
    torch.cuda.synchronize()
    ref = orc.map(0, y, grid)
    fe = orc.forward_error(0, y, grid, ref=ref)
    got = {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
    compare(got, ref, fe, hadronic=had, label=f"1->3 {name}")
    ok = ref["jac"] > 0
    assert ok.mean() > 0.5
    # inverse on the oracle's momenta, bound by the oracle's own spread
    x = ref["x1x2"] if had else None
    inv_ref = orc.inverse(0, ref["p"], x, grid)
    fei = orc.inverse_forward_error(0, ref["p"], x, grid, inv_ref)
    inv = ctx.inverse_map(0, torch.from_numpy(ref["p"]).cuda(), torch.from_numpy(x).cuda() if had else None)
    torch.cuda.synchronize()
    yg = inv["y"].cpu().numpy()
    dy = np.abs(yg - inv_ref["y"]).max(axis=0)[ok]
    fy = fei["y"][ok]
    assert np.all(dy <= np.maximum(1e-12, 1000.0 * fy)), (name, float(np.max(dy / np.maximum(fy, 1e-15))))
    # round trip: a random grid multiplies differences in r by up to 1 /
    # (bins x bin width), and the hadronic spine recovers small invariants
    assert np.median(np.abs(yg - y).max(axis=0)[ok]) < (1e-11 if vegas else 1e-13)
    ctx.close()


def test_dec3_in_multichannel_sample(torch):
    """A binary-tree channel and a 1 -> 3 channel of the same process under
    local channel weights, through the fused sample."""
    from paper_2602_06895_amd import Context

    chans = [{"t_chain": [1, {"d": [2, {"d": [3, 4]}], "m": 300.0, "w": 20.0}], "t_order": ""},
             {"t_chain": [1, {"d": [2, 3, 4], "m": 300.0, "w": 20.0}], "t_order": ""}]
    desc = _hadronic(chans, [0.0] * 4, alpha_mu=10.0)
    ctx = Context(desc)
    orc = oracle.Process(desc)
    counts = np.array([4097, 20001], dtype=np.int64)
    out = ctx.sample(counts, seed=3, stream_id=2, counter_offset=5)
    torch.cuda.synchronize()
    got = {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
    off = 0
    for c, k in enumerate(counts):
        k = int(k)
        sl = slice(off, off + k)
        y = W.philox_uniforms(3, 2, 5 + off, k, ctx.dims[c])
        ref = orc.map(c, y, orc.uniform_grid(c))
        fe = orc.forward_error(c, y, orc.uniform_grid(c), ref=ref)
        seg = {"w": got["w"][sl], "p": got["p"][:, :, sl], "x1x2": got["x1x2"][:, sl]}
        compare(seg, ref, fe, hadronic=True, label=f"1->3 sample ch{c}")
        off += k
    ctx.close()


def test_dec3_volume_and_round_trip(torch):
    from paper_2602_06895_amd import Context

    ctx = Context(_fixed({"s": {"d": [1, 2, 3]}}, [0.0] * 3))
    y = ctx.uniform(4, 3, 0, 4_000_000, ctx.dims[0])
    out = ctx.map(0, y)
    inv = ctx.inverse_map(0, out["p"], None)
    torch.cuda.synchronize()
    j = out["jac"]
    m, e = float(j.mean()), float(j.std()) / math.sqrt(j.numel())
    exact = 1e6 / (256 * math.pi ** 3)
    assert abs(m - exact) < 4.0 * e and e < 1e-3 * exact
    err = (inv["y"] - y).abs().amax(dim=0)
    assert float(err.median()) < 1e-14 and float(err.max()) < 1e-7
    ctx.close()


def test_dec3_mixed_precision(torch):
    """Mixed mode with a three-body cluster on a t-channel spine: the 1 -> 3
    decay is FP64, the tree's power-law, Breit-Wigner and angle steps FP32;
    weights within the mixed mode's statement (median ~1e-6)."""
    from paper_2602_06895_amd import MIXED, Context

    desc = CASES[3][1]()
    ctx = Context(desc, precision=MIXED)
    orc = oracle.Process(desc)
    y = W.philox_uniforms(37, 2, 0, 50001, ctx.dims[0])
    out = ctx.map(0, torch.from_numpy(y).cuda(), weight=True)
    torch.cuda.synchronize()
    ref = orc.map(0, y, orc.uniform_grid(0))
    wg = out["w"].cpu().numpy()
    assert np.mean((ref["w"] != 0) != (wg != 0)) < 1e-3
    ok = (ref["w"] != 0) & (wg != 0)
    wr = np.abs(wg[ok] / ref["w"][ok] - 1.0)
    assert np.median(wr) < 1e-4 and np.quantile(wr, 0.99) < 1e-2
    ctx.close()


def test_dec3_full_size_spot_check(torch):
    """The 1 -> 3 report's workload (t tbar with three-body top decays, 1e7
    events in one fused launch): windows at random positions against the
    oracle."""
    from paper_2602_06895_amd import Context

    desc = W.c3_ttbar6()
    desc["channels"] = [{"s": {"d": [{"d": [1, 2, 3], "m": 173.0, "w": 1.5, "order": 1},
                                     {"d": [4, 5, 6], "m": 173.0, "w": 1.5, "order": 2}]}}]
    ctx = Context(desc)
    orc = oracle.Process(desc)
    n = 10_000_000
    out = ctx.sample(np.array([n]), seed=9, stream_id=1)
    torch.cuda.synchronize()
    rng = np.random.default_rng(8)
    for _ in range(4):
        start = int(rng.integers(0, n - 3000))
        y = W.philox_uniforms(9, 1, start, 3000, ctx.dims[0])
        ref = orc.map(0, y, orc.uniform_grid(0))
        fe = orc.forward_error(0, y, orc.uniform_grid(0), ref=ref)
        seg = {"w": out["w"][start:start + 3000].cpu().numpy(),
               "p": out["p"][:, :, start:start + 3000].cpu().numpy(),
               "x1x2": out["x1x2"][:, start:start + 3000].cpu().numpy()}
        compare(seg, ref, fe, hadronic=True, label=f"1->3 full-size @{start}")
    ctx.close()
