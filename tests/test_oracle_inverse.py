"""Pins of the oracle's inverse mappings (momenta -> uniforms and the channel
density, section 2.1: every mapping of the chain is invertible).

Each inverse is checked against something other than itself: the forward
maps on exact intermediate values (the inverse of each map composed with the
map is the identity), the closed form of the two-body angles, and the round
trip through the independently pinned forward chain.  Round-trip errors are
about one unit roundoff for most points; the tail comes from recovering small
invariants from momenta (the same size in an x87 build with extended
intermediates, so it is conditioning, not the algorithm)."""
import ctypes as C

import numpy as np
import pytest

import oracle
import workloads as W


def _lib():
    return oracle.lib()


@pytest.mark.parametrize("nu,m2,xmin,xmax", [(0.8, -1e-3, 400.0, 1.69e8), (0.8, 0.0, 1.0, 1e4),
                                             (1.0, -1e-3, 10.0, 1e6), (0.0, 0.0, 3.0, 7.0),
                                             (0.5, 80.0 ** 2, 90.0 ** 2, 1e5)])
def test_unmap_nu_inverts_the_power_law(nu, m2, xmin, xmax):
    L = _lib()
    for r in np.linspace(0.0, 1.0, 41):
        j = C.c_double()
        x = L.orc_map_nu(r, m2, nu, xmin, xmax, C.byref(j))
        r2 = L.orc_unmap_nu(x, m2, nu, xmin, xmax)
        # x carries one rounding; r = ((x - m2)^e - B) / (A - B) moves by ~u
        assert abs(r2 - r) < 1e-12, (r, r2)


@pytest.mark.parametrize("m,w,xmin,xmax", [(173.0, 1.5, 100.0 ** 2, 300.0 ** 2), (80.4, 2.1, 0.0, 1e4)])
def test_unmap_bw_inverts_the_breit_wigner(m, w, xmin, xmax):
    L = _lib()
    for r in np.linspace(0.0, 1.0, 41):
        j = C.c_double()
        x = L.orc_map_bw(r, m, w, xmin, xmax, C.byref(j))
        assert abs(L.orc_unmap_bw(x, m, w, xmin, xmax) - r) < 1e-12


def test_vegas_unmap_inverts_the_grid():
    L = _lib()
    rng = np.random.default_rng(3)
    nb = 64
    e = np.concatenate([[0.0], np.sort(rng.random(nb - 1)), [1.0]])
    ep = e.ctypes.data_as(C.POINTER(C.c_double))
    for y in rng.random(500):
        j = C.c_double()
        r = L.orc_vegas_map(y, ep, nb, C.byref(j))
        y2 = L.orc_vegas_unmap(r, ep, nb)
        # the bin width sets the conditioning: dy = dr / (nb width)
        i = min(int(y * nb), nb - 1)
        assert abs(y2 - y) <= 1e-14 / (nb * (e[i + 1] - e[i])) + 1e-15
    # the edges map to the bin starts exactly
    for i in range(nb):
        assert L.orc_vegas_unmap(e[i], ep, nb) == pytest.approx(i / nb, abs=1e-15)


def test_two_body_angles_closed_form():
    """e+e- -> mu+mu- at fixed sqrt(s): the two recovered numbers are the
    azimuth (as a fraction of a turn) and (1 + cos theta) / 2 of the first
    outgoing particle, read directly off its momentum."""
    pr = oracle.Process(W.c1_ee_mumu())
    y = W.philox_uniforms(5, 1, 0, 2000, 2)
    out = pr.map(0, y)
    inv = pr.inverse(0, out["p"], None)
    p1 = out["p"][:, 2, :]
    phi = np.arctan2(p1[2], p1[1]) / (2 * np.pi)
    phi = np.where(phi < 0, phi + 1.0, phi)
    cth = p1[3] / np.sqrt(p1[1] ** 2 + p1[2] ** 2 + p1[3] ** 2)
    assert np.abs(inv["y"][0] - phi).max() < 1e-14
    assert np.abs(inv["y"][1] - 0.5 * (1 + cth)).max() < 1e-14
    assert np.abs(inv["y"] - y).max() < 1e-13
    # constant density 1 / (volume) of the two-body phase space
    assert np.allclose(inv["jac"], out["jac"], rtol=1e-15, atol=0)


CASES = [("c1", W.c1_ee_mumu, 0)] + [("c2", W.c2_pp4j, c) for c in range(8)] + \
        [("c3", W.c3_ttbar6, 0), ("v8", lambda: W.volume_process(8), 0)]


@pytest.mark.parametrize("name,mk,chan", CASES)
def test_round_trip_through_the_forward_chain(name, mk, chan):
    pr = oracle.Process(mk())
    d = pr.dims[chan]
    y = W.philox_uniforms(11, 2, 0, 20000, d)
    out = pr.map(chan, y)
    ok = out["jac"] > 0
    inv = pr.inverse(chan, out["p"], out["x1x2"] if pr.hadronic else None)
    err = np.abs(inv["y"] - y)[:, ok].max(axis=0)
    jr = np.abs(inv["jac"][ok] / out["jac"][ok] - 1.0)
    # measured over these channels: median <= 5e-13, p99 <= 1.2e-7, max <= 1.5e-4;
    # the Jacobian (products of power-law factors near their poles) median
    # <= 6e-12, p99 <= 1.1e-6
    assert np.median(err) < 1e-11
    assert np.quantile(err, 0.99) < 1e-6
    assert err.max() < 5e-3
    assert np.median(jr) < 1e-10
    assert np.quantile(jr, 0.99) < 1e-5


def test_round_trip_through_a_vegas_grid():
    """With an adapted (random) grid the forward VEGAS step is undone too;
    medians stay at the unit roundoff."""
    pr = oracle.Process(W.c2_pp4j())
    rng = np.random.default_rng(8)
    for chan in (0, 6):
        d = pr.dims[chan]
        grid = np.empty((d, pr.nbins + 1))
        for k in range(d):
            grid[k] = np.concatenate([[0.0], np.sort(rng.random(pr.nbins - 1)), [1.0]])
        y = W.philox_uniforms(12, 2, 0, 20000, d)
        out = pr.map(chan, y, grid)
        inv = pr.inverse(chan, out["p"], out["x1x2"], grid)
        err = np.abs(inv["y"] - y).max(axis=0)
        assert np.median(err) < 1e-11
        assert np.quantile(err, 0.99) < 1e-6


def test_planted_sign_error_in_the_inverse_rotation_is_caught():
    """Rebuilding the round trip with the azimuth mirrored (what a wrong sign
    in the inverse rotation produces) fails the closed-form test: the pins
    above see such mistakes."""
    pr = oracle.Process(W.c1_ee_mumu())
    y = W.philox_uniforms(5, 1, 0, 200, 2)
    out = pr.map(0, y)
    inv = pr.inverse(0, out["p"], None)
    mirrored = (1.0 - inv["y"][0]) % 1.0
    assert np.abs(mirrored - y[0]).max() > 0.1


def test_multichannel_density_estimates_the_integral():
    """Events drawn from the channel mixture (channel c with probability
    alpha_c) weighted by f / g, g the global density, estimate the same
    integral as the per-channel SDE weights alpha_c(x) f J (two estimators
    of one quantity, independent arithmetic): agreement within 4 combined
    standard errors."""
    pr = oracle.Process(W.c2_pp4j())
    C = len(pr.channels)
    alpha = np.full(C, 1.0 / C)
    n = 40000
    kp, sde = [], []
    for c in range(C):
        y = W.philox_uniforms(31, 6 + c, 0, n, pr.dims[c])
        out = pr.map(c, y)
        g = pr.multichannel_density(out["p"], out["x1x2"], alpha)
        f = out["f"]
        kp.append(np.where(g > 0, f / np.where(g > 0, g, 1.0), 0.0))
        sde.append(out["w"])
    kp = np.concatenate(kp)  # equal counts = the mixture with alpha_c = 1/C
    I_kp, e_kp = kp.mean(), kp.std() / np.sqrt(kp.size)
    I_sde = sum(w.mean() for w in sde)
    e_sde = np.sqrt(sum(w.var() / w.size for w in sde))
    assert abs(I_kp - I_sde) < 4.0 * np.hypot(e_kp, e_sde), (I_kp, e_kp, I_sde, e_sde)


def test_single_channel_density_is_the_inverse_jacobian():
    """One channel with alpha = 1: g = 1 / J of the event's own channel."""
    pr = oracle.Process(W.c3_ttbar6())
    y = W.philox_uniforms(4, 1, 0, 5000, pr.dims[0])
    out = pr.map(0, y)
    g = pr.multichannel_density(out["p"], out["x1x2"], [1.0])
    r = g * out["jac"]
    # measured: median 5e-12, p99 1.7e-10 (Breit-Wigner factors near the poles)
    assert np.median(np.abs(r - 1.0)) < 1e-10 and np.quantile(np.abs(r - 1.0), 0.99) < 1e-8


def _weights(n, seed):
    rng = np.random.default_rng(seed)
    w = rng.exponential(1.0, n) ** 3
    w[rng.random(n) < 0.3] = 0.0  # cut events
    return w


def test_unweighting_extremes():
    w = np.array([0.0, 2.0, 5.0, 0.0, 3.0])
    u = W.philox_uniforms(1, 2, 0, 5, 1)[0]
    out = oracle.unweight(w, 2.0, u)
    assert list(out["keep"]) == [1, 2, 4]  # w >= w_max: always kept (u < 1)
    assert np.array_equal(out["uw"], [1.0, 2.5, 1.5])
    assert oracle.unweight(np.zeros(5), 1.0, u)["keep"].size == 0


def test_unweighting_is_unbiased():
    """Kept count ~ sum min(1, w / w_max), and w_max sum(unit weights) / N
    estimates mean(w) (also with overweight events), within 5 sigma."""
    n = 400000
    w = _weights(n, 3)
    w_max = np.quantile(w, 0.995)
    u = W.philox_uniforms(9, 1, 0, n, 1)[0]
    out = oracle.unweight(w, w_max, u)
    p = np.minimum(1.0, w / w_max)
    assert abs(out["keep"].size - p.sum()) < 5 * np.sqrt((p * (1 - p)).sum())
    est = w_max * out["uw"].sum() / n
    sig = w_max * np.sqrt((p * (1 - p) * np.maximum(1.0, w / w_max) ** 2).sum()) / n
    assert abs(est - w.mean()) < 5 * sig
    assert np.all(np.diff(out["keep"]) > 0)


def _event(parts):
    """p [4][n+2][1] from massless final-state particles given as (pT, eta, phi)."""
    p = np.zeros((4, len(parts) + 2, 1))
    for i, (pt, eta, phi) in enumerate(parts):
        p[:, i + 2, 0] = [pt * np.cosh(eta), pt * np.cos(phi), pt * np.sin(phi), pt * np.sinh(eta)]
    return p


def test_observables_closed_forms():
    O = oracle
    p = _event([(40.0, 0.7, 1.0), (25.0, -1.2, -2.5), (60.0, 0.1, 3.0), (25.0, 2.0, 0.3)])
    x = O.observables(p, [(O.OBS_PT, [0], 0), (O.OBS_ETA, [0], 0), (O.OBS_PHI, [0], 0),
                          (O.OBS_PT_RANK, [0, 1, 2, 3], 0), (O.OBS_PT_RANK, [0, 1, 2, 3], 2),
                          (O.OBS_PT_RANK, [0, 1, 2, 3], 3), (O.OBS_DR_HARDEST, [0, 1, 2, 3], 0),
                          (O.OBS_E, [1], 0)])[:, 0]
    assert x[0] == pytest.approx(40.0, rel=1e-15) and x[1] == pytest.approx(0.7, rel=1e-14)
    assert x[2] == pytest.approx(1.0, rel=1e-15)
    assert x[3] == pytest.approx(60.0, rel=1e-15) and x[4] == pytest.approx(25.0, rel=1e-15)
    assert x[5] == pytest.approx(25.0, rel=1e-15)  # tie between labels 1 and 3
    # two hardest: label 2 (eta 0.1, phi 3.0) and label 0 (eta 0.7, phi 1.0)
    assert x[6] == pytest.approx(np.hypot(0.6, 2.0), rel=1e-14)
    assert x[7] == pytest.approx(25.0 * np.cosh(-1.2), rel=1e-15)
    # wrapped azimuth difference: phi 3.0 and -3.0 are 2 pi - 6 apart
    q = _event([(30.0, 0.0, 3.0), (20.0, 0.0, -3.0)])
    assert O.observables(q, [(O.OBS_DR_HARDEST, [0, 1], 0)])[0, 0] == pytest.approx(2 * np.pi - 6.0, rel=1e-13)
    # back-to-back massless pair: invariant mass 2 E
    b = _event([(50.0, 0.0, 0.4), (50.0, 0.0, 0.4 + np.pi)])
    assert O.observables(b, [(O.OBS_M, [0, 1], 0)])[0, 0] == pytest.approx(100.0, rel=1e-13)


def test_cut_and_histogram_closed_forms():
    x = np.array([[0.0, 1.0, 2.0, 3.0, 4.0]])
    w = np.ones(5)
    assert list(oracle.cut(x, [1.0], [3.0], w)) == [0.0, 1.0, 1.0, 0.0, 0.0]  # [lo, hi)
    xs = np.array([0.05, 0.15, 0.15, 0.95, 1.0, -0.01])
    ws = np.array([1.0, 2.0, 3.0, 4.0, 5.0, 6.0])
    h = oracle.histogram(xs, ws, 10, 0.0, 1.0)
    assert h[0].tolist() == [1.0, 5.0, 0, 0, 0, 0, 0, 0, 0, 4.0]
    assert h[1].tolist() == [1.0, 13.0, 0, 0, 0, 0, 0, 0, 0, 16.0]


def test_events_outside_a_channels_image_get_zero_density():
    """pp -> 4 jets tree-channel events with a jet below 20 GeV are outside
    the image of a Chili channel with that p_T cut: its inverse marks them
    (y = NaN, J = 0) and the global density takes nothing from it there,
    while events inside (the Chili channel's own) are never marked."""
    d = W.c2_pp4j()
    d["channels"] = d["channels"] + [{"chili": True}]
    o = oracle.Process(d)
    # a process without the cut generates jets of any p_T
    d_nocut = W.c2_pp4j()
    d_nocut["integrand"] = dict(d_nocut["integrand"], pt_min=0.0)
    o0 = oracle.Process(d_nocut)
    y = W.philox_uniforms(8, 2, 0, 20_000, o0.dims[0])
    ev = o0.map(0, y)
    keep = ev["jac"] > 0
    p, x = ev["p"][:, :, keep], ev["x1x2"][:, keep]
    pt = np.hypot(p[1, 2:], p[2, 2:])
    below = (pt[:3] < 20.0).any(axis=0)  # the first three Chili particles carry the cut map
    assert below.sum() > 100 and (~below).sum() > 100
    inv = o.inverse(8, p, x)
    assert np.all(np.isnan(inv["y"][:, below])) and np.all(inv["jac"][below] == 0.0)
    assert np.all(np.isfinite(inv["y"][:, ~below])) and np.all(inv["jac"][~below] > 0.0)
    # the global density over the nine channels: no Chili term where it is 0
    alpha = np.full(9, 1.0 / 9.0)
    g9 = o.multichannel_density(p, x, alpha)
    g8 = oracle.Process(W.c2_pp4j()).multichannel_density(p, x, alpha[:8])
    assert np.allclose(g9[below], g8[below], rtol=1e-14, atol=0.0)
    assert np.all(g9[~below] >= g8[~below]) and (g9[~below] > g8[~below]).mean() > 0.5
    # the Chili channel's own events are in its image
    yc = W.philox_uniforms(9, 2, 0, 20_000, o.dims[8])
    evc = o.map(8, yc)
    kc = evc["jac"] > 0
    invc = o.inverse(8, evc["p"][:, :, kc], evc["x1x2"][:, kc])
    assert np.all(np.isfinite(invc["y"])) and np.all(invc["jac"] > 0.0)
