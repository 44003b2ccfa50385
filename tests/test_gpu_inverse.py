"""Inverse map (msx_inverse_map) against the oracle's inverse on the same
lab-frame momenta, and the GPU forward/inverse round trip.

Both inverses recover invariants from momenta, which is ill-conditioned for
small invariants (see the oracle's pins).  Per event the allowed difference
therefore scales with the oracle's forward error fe on that event: the
spread of its x87 build and of the builds with every libm / sqrt result and
every input momentum moved by one ulp.  Every event within max(1e-12,
1000 fe), all but 1e-3 of them within max(1e-12, 100 fe).  The density (the
forward Jacobian at the recovered y) is compared with the oracle's forward
Jacobian at the GPU's own y, within the forward chain's parity bound."""
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


def _random_grid(d, nb, seed):
    rng = np.random.default_rng(seed)
    g = np.empty((d, nb + 1))
    for k in range(d):
        g[k] = np.concatenate([[0.0], np.sort(rng.random(nb - 1)), [1.0]])
    return g


CASES = [("c1", W.c1_ee_mumu, 0, False)] + [("c2", W.c2_pp4j, c, c in (0, 6)) for c in range(8)] + \
        [("c3", W.c3_ttbar6, 0, True), ("v8", lambda: W.volume_process(8), 0, False)]


@pytest.mark.parametrize("name,mk,chan,vegas", CASES)
def test_inverse_matches_oracle(torch, name, mk, chan, vegas):
    from paper_2602_06895_amd import Context

    desc = mk()
    if name == "v8":
        desc["vegas_bins"] = 128
    ctx = Context(desc)
    orc = oracle.Process(desc)
    d = ctx.dims[chan]
    grid = _random_grid(d, orc.nbins, 17 + chan) if vegas else orc.uniform_grid(chan)
    ctx.set_grid(chan, grid)
    n = 30001  # several tiles and a ragged tail
    y = W.philox_uniforms(21, 3, 0, n, d)
    fwd = orc.map(chan, y, grid)
    ok = fwd["jac"] > 0
    x = fwd["x1x2"] if orc.hadronic else None
    ref = orc.inverse(chan, fwd["p"], x, grid)
    fe = orc.inverse_forward_error(chan, fwd["p"], x, grid, ref)
    out = ctx.inverse_map(chan, torch.from_numpy(fwd["p"]).cuda(),
                          torch.from_numpy(x).cuda() if x is not None else None)
    torch.cuda.synchronize()
    yg = out["y"].cpu().numpy()
    jg = out["jac"].cpu().numpy()
    dy = np.abs(yg - ref["y"]).max(axis=0)[ok]
    fy = fe["y"][ok]
    assert np.all(dy <= np.maximum(1e-12, 1000.0 * fy)), (name, chan, float(np.max(dy / np.maximum(fy, 1e-15))))
    assert np.mean(dy > np.maximum(1e-12, 100.0 * fy)) <= 1e-3
    # the density: the GPU's Jacobian against the oracle's forward Jacobian at
    # the GPU's own y (the y differences above are checked there), within the
    # forward chain's parity bound
    at = orc.map(chan, yg, grid)
    fef = orc.forward_error(chan, yg, grid, ref=at)
    keep = ok & (at["jac"] > 0)
    dj = np.abs(jg[keep] / at["jac"][keep] - 1.0)
    fj = fef["jac"][keep]
    assert np.all(dj <= np.maximum(1e-12, 1000.0 * fj)), (name, chan, float(np.max(dj / np.maximum(fj, 1e-15))))
    # most events agree to the unit roundoff scale (a random grid multiplies
    # differences in r by 1 / (bins x bin width), ~ 1 typically, 16 dims)
    assert np.median(dy) < (1e-11 if vegas else 1e-12)
    ctx.close()


def test_round_trip_at_scale(torch):
    """1e6 events per pp -> 4 jets channel through the GPU forward map and back."""
    from paper_2602_06895_amd import Context

    ctx = Context(W.c2_pp4j())
    for chan in range(8):
        d = ctx.dims[chan]
        y = ctx.uniform(5, 4, 0, 1_000_000, d)
        fwd = ctx.map(chan, y)
        inv = ctx.inverse_map(chan, fwd["p"], fwd["x1x2"])
        torch.cuda.synchronize()
        ok = fwd["jac"] > 0
        err = (inv["y"] - y).abs().amax(dim=0)[ok]
        jr = (inv["jac"][ok] / fwd["jac"][ok] - 1.0).abs()
        q = torch.tensor([0.5, 0.99], dtype=torch.float64, device="cuda")
        e50, e99 = torch.quantile(err[:200_000], q).tolist()
        j50, j99 = torch.quantile(jr[:200_000], q).tolist()
        # the tail (small invariants recovered from momenta) grows with the
        # sample: bound its share rather than its maximum
        tail = float((err > 1e-3).double().mean())
        assert e50 < 1e-11 and e99 < 1e-6 and tail < 1e-4, (chan, e50, e99, tail)
        assert j50 < 1e-10 and j99 < 1e-5, (chan, j50, j99)
    ctx.close()


@pytest.mark.parametrize("n", [1, 255, 257])
def test_ragged_and_tiny_batches(torch, n):
    from paper_2602_06895_amd import Context

    ctx = Context(W.c3_ttbar6())
    y = ctx.uniform(9, 1, 3, n, ctx.dims[0])
    fwd = ctx.map(0, y)
    inv = ctx.inverse_map(0, fwd["p"], fwd["x1x2"])
    torch.cuda.synchronize()
    assert float((inv["y"] - y).abs().max()) < 1e-6
    ctx.close()


def test_empty_and_argument_errors(torch):
    from paper_2602_06895_amd import Context, MsxError

    ctx = Context(W.c1_ee_mumu())
    p = torch.zeros(4, 4, 0, dtype=torch.float64, device="cuda")
    out = ctx.inverse_map(0, p, None)
    assert out["y"].shape == (2, 0)
    with pytest.raises(MsxError):
        ctx.inverse_map(0, torch.zeros(4, 4, 8, dtype=torch.float64, device="cuda"),
                        torch.zeros(2, 8, dtype=torch.float64, device="cuda"))
    ctx.close()


def test_multichannel_density_matches_oracle(torch):
    """g(p) = sum_c alpha_c / J_c(y_c(p)) over the 8 pp -> 4 jets channels
    for events of two of them, against the oracle's density."""
    from paper_2602_06895_amd import Context

    desc = W.c2_pp4j()
    ctx = Context(desc)
    orc = oracle.Process(desc)
    alpha = np.array([0.3, 0.1, 0.1, 0.1, 0.1, 0.1, 0.1, 0.1])
    for chan in (2, 7):
        y = W.philox_uniforms(41, chan, 0, 20001, orc.dims[chan])
        fwd = orc.map(chan, y)
        ok = fwd["jac"] > 0
        g_ref = orc.multichannel_density(fwd["p"], fwd["x1x2"], alpha)
        g = ctx.multichannel_density(0, torch.from_numpy(fwd["p"]).cuda(), torch.from_numpy(fwd["x1x2"]).cuda(),
                                     alpha)
        torch.cuda.synchronize()
        # every channel inverts every event, also far from its own region
        # (worse conditioned): the bound is the oracle's perturbation spread
        fe = np.max([np.abs(orc.multichannel_density(fwd["p"], fwd["x1x2"], alpha, variant=v) / g_ref - 1.0)
                     for v in ("x87", "up", "down")], axis=0)[ok]
        r = np.abs(g.cpu().numpy()[ok] / g_ref[ok] - 1.0)
        assert np.all(r <= np.maximum(1e-12, 1000.0 * fe)), (chan, float(np.max(r / np.maximum(fe, 1e-15))))
        assert np.median(r) < 1e-12
    ctx.close()


@pytest.mark.parametrize("n", [0, 1, 1023, 1025, 100003])
def test_unweighting_matches_oracle(torch, n):
    """Kept indices, count and unit weights bit-identical to the oracle's on
    the same weights and the same Philox stream."""
    from paper_2602_06895_amd import Context

    rng = np.random.default_rng(n)
    w = rng.exponential(1.0, n) ** 3
    w[rng.random(n) < 0.3] = 0.0
    w_max = float(np.quantile(w, 0.99)) if n else 1.0
    ctx = Context(W.c1_ee_mumu())
    out = ctx.unweight(torch.from_numpy(w).cuda(), w_max, seed=5, stream_id=7, counter_offset=11)
    torch.cuda.synchronize()
    u = W.philox_uniforms(5, 7, 11, n, 1)[0] if n else np.zeros(0)
    ref = oracle.unweight(w, w_max, u)
    k = int(out["count"].cpu()[0])
    assert k == ref["keep"].size
    assert np.array_equal(out["keep"][:k].cpu().numpy(), ref["keep"])
    assert np.array_equal(out["uw"][:k].cpu().numpy(), ref["uw"])
    ctx.close()


def test_observables_cuts_histograms_match_oracle(torch):
    """The distributions of the paper's validation (sqrt(s-hat) from the
    summed final state, hardest-jet p_T, separation of the two hardest jets)
    on pp -> 4 jets events: observables per event against the oracle's,
    cuts and weighted histograms of the GPU's own values against the
    oracle's on the same values."""
    from paper_2602_06895_amd import OBS_DR_HARDEST, OBS_ETA, OBS_M, OBS_PHI, OBS_PT, OBS_PT_RANK, Context

    desc = W.c2_pp4j()
    ctx = Context(desc)
    orc = oracle.Process(desc)
    y = W.philox_uniforms(3, 9, 0, 100003, orc.dims[0])
    fwd = orc.map(0, y)
    jets = [0, 1, 2, 3]
    spec = [(OBS_M, jets, 0), (OBS_PT_RANK, jets, 0), (OBS_DR_HARDEST, jets, 0), (OBS_PT, [1], 0),
            (OBS_ETA, [2], 0), (OBS_PHI, [3], 0), (OBS_PT_RANK, jets, 3)]
    p = torch.from_numpy(fwd["p"]).cuda()
    x = ctx.observables(0, p, spec)
    w = torch.from_numpy(fwd["w"]).cuda()
    torch.cuda.synchronize()
    xg = x.cpu().numpy()
    xr = oracle.observables(fwd["p"], spec)
    tol = 1e-13 * np.maximum(1.0, np.abs(xr))
    # the invariant mass of a boosted system cancels: E^2 - p^2 carries
    # ~ u E^2 (FMA contraction on one side only), so dM ~ u E^2 / M
    esum = fwd["p"][0, 2:].sum(axis=0)
    tol[0] += 1e-14 * esum ** 2 / np.maximum(xr[0], 1e-300)
    bad = np.abs(xg - xr) > tol
    assert not bad.any(), [(j, float(np.max(np.abs(xg[j] - xr[j]) / tol[j]))) for j in range(len(spec))]
    lo, hi = [500.0, 50.0, 0.4], [13000.0, np.inf, np.inf]
    wc = ctx.cut(x[:3].contiguous(), lo, hi, w.clone())
    torch.cuda.synchronize()
    assert np.array_equal(wc.cpu().numpy(), oracle.cut(xg[:3], lo, hi, fwd["w"]))
    for j, (bins, a, b) in enumerate([(50, 0.0, 6500.0), (40, 0.0, 2000.0), (30, 0.0, 6.0)]):
        h = ctx.histogram(x[j].contiguous(), wc, bins, a, b)
        torch.cuda.synchronize()
        hr = oracle.histogram(xg[j], wc.cpu().numpy(), bins, a, b)
        assert np.allclose(h.cpu().numpy(), hr, rtol=1e-12, atol=0.0)
    ctx.close()
