"""Pins of the oracle's Chili generator (section 2.4).

Chili samples each final-state particle but the last in (p_T, y, phi) in the
lab frame, fixes the last one's transverse momentum by recoil and its
rapidity within what the beam energy leaves, and reads x1, x2 off the summed
light-cone momenta.  Its weight must integrate the same phase space as the
tree channels: checked against closed forms of the hadronic massless n-body
volume (no cut), against one-dimensional quadratures of the 2-body volume
with a p_T cut or masses, and against the tree-channel integral of the same
integrand, each within the Monte Carlo error."""
import math

import numpy as np
import pytest

import oracle
import workloads as W


def _mc(desc, chan=0, n=2_000_000, seed=1):
    o = oracle.Process(desc)
    y = W.philox_uniforms(seed, chan, 0, n, o.dims[chan])
    f = o.map(chan, y)
    w = f["w"]
    return float(w.mean()), float(w.std() / math.sqrt(n)), f


def _hadronic_volume(n, s):
    """int dx1 dx2 Phi_n(x1 x2 s) for massless particles without cuts:
    Phi_n(s-hat) = (2 pi)^(4-3n) (pi/2)^(n-1) s-hat^(n-2) / ((n-1)! (n-2)!)
    and int_0^1 dtau (-log tau) tau^k = 1/(k+1)^2."""
    phi = (2 * math.pi) ** (4 - 3 * n) * (math.pi / 2) ** (n - 1) / (math.factorial(n - 1) * math.factorial(n - 2))
    return phi * s ** (n - 2) / (n - 1) ** 2


@pytest.mark.parametrize("n", [2, 3])
def test_massless_volume_closed_form(n):
    d = W.chili_process(n, sqrt_s=1000.0)
    m, e, _ = _mc(d)
    exact = _hadronic_volume(n, 1000.0 ** 2)
    assert abs(m - exact) < 4.0 * e, (m, e, exact)
    assert e < 0.1 * exact


def _two_body_quad(t0):
    """int dtau (-log tau) Phi_2 with the 2-body factor sqrt(1 - t0/tau) / (8 pi):
    massless with p_T > p_min (t0 = 4 p_min^2 / s: |cos theta| < sqrt(1 - t0/tau))
    or equal masses m (t0 = 4 m^2 / s: the velocity)."""
    from scipy import integrate

    return integrate.quad(lambda t: -math.log(t) / (8 * math.pi) * math.sqrt(1 - t0 / t), t0, 1.0,
                          epsabs=0.0, epsrel=1e-12, limit=200)[0]


@pytest.mark.parametrize("ptmin", [20.0, 200.0])
def test_two_body_with_pt_cut(ptmin):
    m, e, f = _mc(W.chili_process(2, sqrt_s=1000.0, pt_min=ptmin))
    exact = _two_body_quad(4 * ptmin ** 2 / 1e6)
    assert abs(m - exact) < 4.0 * e, (m, e, exact)
    assert e < 0.01 * exact
    # the first particle's p_T is sampled above the cut
    ok = f["jac"] > 0
    pt = np.hypot(f["p"][1, 2], f["p"][2, 2])[ok]
    assert pt.min() >= ptmin * (1 - 1e-12)


@pytest.mark.parametrize("mass", [50.0, 300.0])
def test_two_body_massive(mass):
    m, e, _ = _mc(W.chili_process(2, sqrt_s=1000.0, masses=[mass, mass]))
    exact = _two_body_quad(4 * mass ** 2 / 1e6)
    assert abs(m - exact) < 4.0 * e, (m, e, exact)
    assert e < 0.01 * exact


@pytest.mark.parametrize("n,masses", [(3, None), (3, 10.0), (4, None), (4, 10.0)])
def test_against_tree_channel(n, masses):
    """Toy PDFs and p_T > 20 GeV: the Chili integral against the t-channel
    tree's, both unbiased estimates of the same integral."""
    ms = None if masses is None else [masses] * n
    d = W.chili_process(n, sqrt_s=1000.0, pt_min=20.0, masses=ms, pdf=[-1.2, 3.0])
    a = _mc(d)
    d2 = W.chili_process(n, sqrt_s=1000.0, pt_min=20.0, masses=ms, pdf=[-1.2, 3.0])
    d2["channels"] = [{"t_chain": list(range(1, n + 1)), "t_order": "A" * (n - 2)}]
    d2["shat_min"] = (n * math.hypot(20.0, masses or 0.0)) ** 2  # implied by the cut
    b = _mc(d2)
    pull = (a[0] - b[0]) / math.hypot(a[1], b[1])
    assert abs(pull) < 4.0, (a[:2], b[:2], pull)


def test_pp4j_against_multichannel():
    """The pp -> 4 jets integrand (toy PDFs, t-propagators, p_T cut) through
    one Chili channel against the eight-channel tree integral."""
    d = W.c2_pp4j()
    d["channels"] = [{"chili": True}]
    a = _mc(d)
    d2 = W.c2_pp4j()
    o2 = oracle.Process(d2)
    tot, var = 0.0, 0.0
    for c in range(8):
        y = W.philox_uniforms(1, 3 + c, 0, 250_000, o2.dims[c])
        w = o2.map(c, y)["w"]
        tot += w.mean()
        var += w.var() / w.size
    pull = (a[0] - tot) / math.hypot(a[1], math.sqrt(var))
    assert abs(pull) < 4.0, (a[:2], tot, math.sqrt(var))


def test_event_kinematics():
    """Momentum conservation, mass shells, x1, x2 in (0, 1] and the beam
    momenta of every kept event."""
    ms = [5.0, 0.0, 80.0, 0.0]
    d = W.chili_process(4, sqrt_s=13000.0, pt_min=20.0, masses=ms)
    o = oracle.Process(d)
    assert o.dims == [10]
    y = W.philox_uniforms(3, 0, 0, 100_000, 10)
    f = o.map(0, y)
    ok = f["jac"] > 0
    assert ok.mean() > 0.5
    p = f["p"][:, :, ok]
    x = f["x1x2"][:, ok]
    scale = p[0].sum(axis=0)
    dp = np.abs(p[:, :2].sum(axis=1) - p[:, 2:].sum(axis=1)).max(axis=0)
    assert np.all(dp < 1e-12 * scale)
    for i, m in enumerate(ms):
        m2 = p[0, i + 2] ** 2 - p[1, i + 2] ** 2 - p[2, i + 2] ** 2 - p[3, i + 2] ** 2
        assert np.all(np.abs(m2 - m * m) < 1e-11 * p[0, i + 2] ** 2)
    assert np.all((x > 0) & (x <= 1))
    h = 6500.0
    assert np.allclose(p[0, 0], x[0] * h, rtol=1e-13) and np.allclose(p[0, 1], x[1] * h, rtol=1e-13)


def test_lepton_beams_refused():
    d = W.chili_process(3)
    d["beams"] = "fixed"
    with pytest.raises(ValueError):
        oracle.Process(d)


@pytest.mark.parametrize("case", ["cut", "nocut"])
def test_inverse_round_trip(case):
    """The inverse recovers the uniforms (through a VEGAS grid) and the
    forward Jacobian at them: median at the unit roundoff, every event
    within what the ill-conditioned recoveries (small p_T, large |y|) allow."""
    if case == "cut":
        d = W.chili_process(4, 13000.0, pt_min=20.0, masses=[5.0, 0.0, 80.0, 0.0], pdf=[-1.2, 3.0])
    else:
        d = W.chili_process(3, 1000.0, masses=[0.0, 10.0, 80.0])
    o = oracle.Process(d)
    dim = o.dims[0]
    rng = np.random.default_rng(3)
    g = np.empty((dim, o.nbins + 1))
    for k in range(dim):
        g[k] = np.concatenate([[0.0], np.sort(rng.random(o.nbins - 1)), [1.0]])
    y = W.philox_uniforms(2, 0, 0, 100_000, dim)
    f = o.map(0, y, g)
    ok = f["jac"] > 0
    inv = o.inverse(0, f["p"], f["x1x2"], g)
    err = np.abs(inv["y"] - y).max(axis=0)[ok]
    assert np.median(err) < 1e-14 and np.quantile(err, 0.99) < 1e-12 and err.max() < 1e-8
    jr = np.abs(inv["jac"][ok] / f["jac"][ok] - 1.0)
    assert np.median(jr) < 1e-14 and jr.max() < 1e-8


def test_chili_beside_tree_channels_keeps_every_channel_weighted():
    """A Chili channel beside the eight pp -> 4 jets diagram channels under
    local channel weights: the Chili channel has no propagator denominators,
    so it takes the constant share 1/9 and the diagram channels share 8/9 by
    their propagator products (a reading: the paper's local weights are
    defined for diagram channels only).  Pins: the nine weights of one event
    sum to 1 and the Chili one equals 1/9 exactly; no channel's mean weight is
    negligible; the nine-channel multichannel integral equals the eight
    tree channels' integral without the Chili channel."""
    d = W.c2_pp4j()
    d["channels"] = d["channels"] + [{"chili": True}]
    o = oracle.Process(d)
    C_ = len(o.dims)
    assert C_ == 9
    # alpha of every channel at the same events (channel 8's events)
    y = W.philox_uniforms(4, 1, 0, 20_000, o.dims[8])
    ev = o.map(8, y)
    keep = ev["jac"] > 0
    alphas = []
    for c in range(C_):
        alphas.append(o.weight(c, ev["p"][:, :, keep], ev["x1x2"][:, keep], ev["jac"][keep])["alpha"])
    alphas = np.array(alphas)
    ok = np.isfinite(alphas).all(axis=0)
    assert np.all(alphas[8][ok] == 1.0 / 9.0)
    assert np.abs(alphas[:, ok].sum(axis=0) - 1.0).max() < 1e-13
    # every channel's own events: its mean alpha is a visible share
    tot, var = 0.0, 0.0
    for c in range(C_):
        yc = W.philox_uniforms(5, 10 + c, 0, 200_000, o.dims[c])
        r = o.map(c, yc)
        k = r["jac"] > 0
        assert r["alpha"][k].mean() > 1e-3, f"channel {c}: mean alpha {r['alpha'][k].mean():.3g}"
        tot += r["w"].mean()
        var += r["w"].var() / r["w"].size
    o2 = oracle.Process(W.c2_pp4j())
    t2, v2 = 0.0, 0.0
    for c in range(8):
        yc = W.philox_uniforms(6, 3 + c, 0, 200_000, o2.dims[c])
        w = o2.map(c, yc)["w"]
        t2 += w.mean()
        v2 += w.var() / w.size
    pull = (tot - t2) / math.sqrt(var + v2)
    assert abs(pull) < 4.0, (tot, t2, math.sqrt(var), math.sqrt(v2))
