"""Chili channels (section 2.4) on the GPU against the oracle: per-event
momenta, momentum fractions, Jacobians and weights through the map and the
fused multichannel sample (also mixed with tree channels under local channel
weights), the closed-form hadronic volume, the inverse map and the
multichannel density."""
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
    channel weights (the Chili channel has no propagators: it takes the
    constant weight 1/9, the tree channels share 8/9 by their propagator
    products), through the fused multichannel sample; every channel's events
    carry a visible share of the weight."""
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
            if k > 200:
                kept = ref["jac"] > 0
                assert ref["alpha"][kept].mean() > 1e-3, f"channel {c}: negligible channel weight"
                if c == 8:
                    assert np.all(ref["alpha"][kept] == 1.0 / 9.0)
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


@pytest.mark.parametrize("name,mk,vegas", CASES)
def test_chili_inverse_matches_oracle(torch, name, mk, vegas):
    """Inverse map against the oracle's inverse on the same momenta (bound:
    the oracle's own forward-error spread, as for the tree channels), and
    the density (forward Jacobian at the GPU's y) against the oracle's."""
    from paper_2602_06895_amd import Context

    desc = mk()
    ctx = Context(desc)
    orc = oracle.Process(desc)
    d = ctx.dims[0]
    grid = _random_grid(d, orc.nbins, 7) if vegas else orc.uniform_grid(0)
    ctx.set_grid(0, grid)
    y = W.philox_uniforms(23, 1, 0, 20001, d)
    fwd = orc.map(0, y, grid)
    ok = fwd["jac"] > 0
    ref = orc.inverse(0, fwd["p"], fwd["x1x2"], grid)
    fe = orc.inverse_forward_error(0, fwd["p"], fwd["x1x2"], grid, ref)
    out = ctx.inverse_map(0, torch.from_numpy(fwd["p"]).cuda(), torch.from_numpy(fwd["x1x2"]).cuda())
    torch.cuda.synchronize()
    yg, jg = out["y"].cpu().numpy(), out["jac"].cpu().numpy()
    dy = np.abs(yg - ref["y"]).max(axis=0)[ok]
    fy = fe["y"][ok]
    assert np.all(dy <= np.maximum(1e-12, 1000.0 * fy)), (name, float(np.max(dy / np.maximum(fy, 1e-15))))
    assert np.mean(dy > np.maximum(1e-12, 100.0 * fy)) <= 1e-3
    assert np.median(np.abs(yg - y).max(axis=0)[ok]) < 1e-13
    at = orc.map(0, yg, grid)
    fef = orc.forward_error(0, yg, grid, ref=at)
    keep = ok & (at["jac"] > 0)
    dj = np.abs(jg[keep] / at["jac"][keep] - 1.0)
    assert np.all(dj <= np.maximum(1e-12, 1000.0 * fef["jac"][keep]))
    ctx.close()


def test_chili_density_with_tree_channels(torch):
    """g(p) = sum_c alpha_c / J_c(y_c(p)) over the eight pp -> 4 jets tree
    channels and a Chili channel, for events of the Chili channel and of a
    tree channel, against the oracle's density."""
    from paper_2602_06895_amd import Context

    desc = W.c2_pp4j()
    desc["channels"] = desc["channels"] + [{"chili": True}]
    ctx = Context(desc)
    orc = oracle.Process(desc)
    alpha = np.array([0.1] * 8 + [0.2])
    for chan in (8, 3):
        y = W.philox_uniforms(43, chan, 0, 20001, orc.dims[chan])
        fwd = orc.map(chan, y)
        ok = fwd["jac"] > 0
        g_ref = orc.multichannel_density(fwd["p"], fwd["x1x2"], alpha)
        g = ctx.multichannel_density(0, torch.from_numpy(fwd["p"]).cuda(), torch.from_numpy(fwd["x1x2"]).cuda(),
                                     alpha)
        torch.cuda.synchronize()
        with np.errstate(invalid="ignore", divide="ignore"):  # g = 0 on events every channel cuts
            fe = np.max([np.abs(orc.multichannel_density(fwd["p"], fwd["x1x2"], alpha, variant=v) / g_ref - 1.0)
                         for v in ("x87", "up", "down")], axis=0)[ok]
        r = np.abs(g.cpu().numpy()[ok] / g_ref[ok] - 1.0)
        assert np.all(r <= np.maximum(1e-12, 1000.0 * fe)), (chan, float(np.max(r / np.maximum(fe, 1e-15))))
        assert np.median(r) < 1e-12
    ctx.close()


def test_chili_round_trip_at_scale(torch):
    """1e6 pp -> 4 jets Chili events through the GPU forward map and back."""
    from paper_2602_06895_amd import Context

    ctx = Context(_pp4j_chili())
    y = ctx.uniform(5, 9, 0, 1_000_000, ctx.dims[0])
    fwd = ctx.map(0, y)
    inv = ctx.inverse_map(0, fwd["p"], fwd["x1x2"])
    torch.cuda.synchronize()
    ok = fwd["jac"] > 0
    err = (inv["y"] - y).abs().amax(dim=0)[ok]
    jr = (inv["jac"][ok] / fwd["jac"][ok] - 1.0).abs()
    assert float(err.median()) < 1e-14 and float(err.max()) < 1e-7
    assert float(jr.median()) < 1e-14 and float(jr.max()) < 1e-7
    ctx.close()


def test_chili_lepton_beams_refused(torch):
    from paper_2602_06895_amd import Context, MsxError

    d = W.chili_process(3)
    d["beams"] = "fixed"
    with pytest.raises(MsxError):
        Context(d)


def test_chili_mixed_precision(torch):
    """In the mixed mode the Chili generator stays FP64 (momenta and
    Jacobians as the oracle's); only the integrand's FP32 steps (toy PDFs)
    move the weights, by a few FP32 ulp."""
    from paper_2602_06895_amd import MIXED, Context

    desc = _pp4j_chili()
    ctx = Context(desc, precision=MIXED)
    orc = oracle.Process(desc)
    y = W.philox_uniforms(31, 1, 0, 50001, ctx.dims[0])
    out = ctx.map(0, torch.from_numpy(y).cuda(), weight=True)
    torch.cuda.synchronize()
    ref = orc.map(0, y, orc.uniform_grid(0))
    ok = (ref["w"] != 0) & (out["w"].cpu().numpy() != 0)
    assert np.mean((ref["w"] != 0) != (out["w"].cpu().numpy() != 0)) < 1e-4
    jr = np.abs(out["jac"].cpu().numpy()[ok] / ref["jac"][ok] - 1.0)
    assert np.median(jr) < 1e-14 and np.quantile(jr, 0.999) < 1e-10
    wr = np.abs(out["w"].cpu().numpy()[ok] / ref["w"][ok] - 1.0)
    assert np.median(wr) < 1e-5 and np.quantile(wr, 0.99) < 1e-4
    ctx.close()


def test_chili_full_size_spot_check(torch):
    """The Chili report's workload (pp -> 4 jets through one Chili channel,
    1e7 events in one fused launch, the default launch shape bench.py uses
    for it): windows of events at random positions recomputed by the
    oracle."""
    from paper_2602_06895_amd import Context

    desc = _pp4j_chili()
    ctx = Context(desc)
    orc = oracle.Process(desc)
    n = 10_000_000
    out = ctx.sample(np.array([n]), seed=8, stream_id=1)
    torch.cuda.synchronize()
    rng = np.random.default_rng(6)
    for _ in range(4):
        start = int(rng.integers(0, n - 3000))
        y = W.philox_uniforms(8, 1, start, 3000, ctx.dims[0])
        ref = orc.map(0, y, orc.uniform_grid(0))
        fe = orc.forward_error(0, y, orc.uniform_grid(0), ref=ref)
        seg = {"w": out["w"][start:start + 3000].cpu().numpy(),
               "p": out["p"][:, :, start:start + 3000].cpu().numpy(),
               "x1x2": out["x1x2"][:, start:start + 3000].cpu().numpy()}
        compare(seg, ref, fe, hadronic=True, label=f"Chili full-size @{start}")
    ctx.close()


def test_inverse_marks_events_outside_the_chili_image(torch):
    """Tree-channel events with a jet below the Chili channel's p_T cut are
    outside its image: the GPU inverse gives y = NaN and J = 0 for exactly the
    events the oracle marks, and the global density over the tree channels
    plus Chili matches the oracle's."""
    from paper_2602_06895_amd import Context

    d = W.c2_pp4j()
    d["channels"] = d["channels"] + [{"chili": True}]
    ctx = Context(d)
    orc = oracle.Process(d)
    d0 = W.c2_pp4j()
    d0["integrand"] = dict(d0["integrand"], pt_min=0.0)
    o0 = oracle.Process(d0)
    y = W.philox_uniforms(8, 2, 0, 20_000, o0.dims[0])
    ev = o0.map(0, y)
    keep = ev["jac"] > 0
    p, x = ev["p"][:, :, keep], ev["x1x2"][:, keep]
    ref = orc.inverse(8, p, x)
    pt_ = torch.from_numpy(np.ascontiguousarray(p)).cuda()
    xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    got = ctx.inverse_map(8, pt_, xt)
    torch.cuda.synchronize()
    yg, jg = got["y"].cpu().numpy(), got["jac"].cpu().numpy()
    marked_o = np.isnan(ref["y"]).all(axis=0)
    marked_g = np.isnan(yg).all(axis=0)
    assert marked_o.sum() > 100
    assert np.array_equal(marked_o, marked_g)
    assert np.all(jg[marked_g] == 0.0) and np.all(jg[~marked_g] > 0.0)
    # the global density adds the channels in order, Chili last: where its
    # density is 0 the nine-channel sum equals the eight tree channels' sum
    alpha = np.full(9, 1.0 / 9.0)
    g9 = ctx.multichannel_density(0, pt_, xt, alpha).cpu().numpy()
    c8 = Context(W.c2_pp4j())
    g8 = c8.multichannel_density(0, pt_, xt, alpha[:8]).cpu().numpy()
    assert np.array_equal(g9[marked_g], g8[marked_g])
    assert np.all(g9[~marked_g] >= g8[~marked_g]) and (g9[~marked_g] > g8[~marked_g]).mean() > 0.5
    c8.close()
    ctx.close()
