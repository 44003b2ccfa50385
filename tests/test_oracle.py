"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed
forms (phase-space volumes, two-body momenta, Jacobian normalisation by
quadrature), invariants (momentum conservation, on-shell masses, recomputed
invariants), brute force on tiny inputs, and values printed in the paper.
"""
import ctypes as C
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
dp = C.POINTER(C.c_double)


def _arr(v):
    a = (C.c_double * len(v))(*v)
    return a


def _gl(n, a=0.0, b=1.0):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (b - a) * x + 0.5 * (b + a), 0.5 * (b - a) * w


def massless_volume(n, E):
    """Closed-form massless n-body phase-space volume (section 4.1)."""
    return E ** (2 * n - 4) / (math.gamma(n) * math.gamma(n - 1) * math.pi ** (2 * n - 3) * 2 ** (4 * n - 5))


def _minkowski(p):
    return p[0] ** 2 - p[1] ** 2 - p[2] ** 2 - p[3] ** 2


# --------------------------------------------------------------------------
# Elementary operations
# --------------------------------------------------------------------------

@pytest.mark.parametrize("m0,m1,m2,expect", [
    (1000.0, 0.0, 0.0, 500.0),
    (1000.0, 173.0, 173.0, 0.5 * math.sqrt(1000.0 ** 2 - 4 * 173.0 ** 2)),
    (500.0, 80.4, 4.7, None),
])
def test_two_body_decay_momentum_closed_form(m0, m1, m2, expect):
    """|p| = lambda^(1/2)(m0^2, m1^2, m2^2)/(2 m0) and E_{1,2} in the rest frame
    (section 2.2.3); p1 + p2 = P and p_i^2 = m_i^2 after the boost."""
    L = oracle.lib()
    rng = np.random.default_rng(3)
    s = m0 * m0
    lam = (s - m1 ** 2 - m2 ** 2) ** 2 - 4 * m1 ** 2 * m2 ** 2
    q = math.sqrt(lam) / (2 * m0)
    if expect is not None:
        assert q == pytest.approx(expect, rel=1e-14)
    for _ in range(20):
        rest = _arr([m0, 0.0, 0.0, 0.0])
        p1, p2 = _arr([0] * 4), _arr([0] * 4)
        L.orc_two_body_decay(rest, s, m1, m2, rng.random(), rng.random(), p1, p2)
        assert math.sqrt(p1[1] ** 2 + p1[2] ** 2 + p1[3] ** 2) == pytest.approx(q, rel=1e-13)
        assert p1[0] == pytest.approx((s + m1 ** 2 - m2 ** 2) / (2 * m0), rel=1e-14)
        assert p2[0] == pytest.approx((s - m1 ** 2 + m2 ** 2) / (2 * m0), rel=1e-14)
        # moving parent
        pz = rng.normal() * 300
        px = rng.normal() * 200
        P = [math.sqrt(s + pz * pz + px * px), px, 0.0, pz]
        L.orc_two_body_decay(_arr(P), s, m1, m2, rng.random(), rng.random(), p1, p2)
        for c in range(4):
            assert p1[c] + p2[c] == pytest.approx(P[c], abs=1e-12 * P[0])
        assert _minkowski(p1) == pytest.approx(m1 ** 2, abs=1e-10 * P[0] ** 2)
        assert _minkowski(p2) == pytest.approx(m2 ** 2, abs=1e-10 * P[0] ** 2)


def test_two_body_decay_jacobian_is_measure():
    """The decay Jacobian is sqrt(lambda)/(8 m0^2) * 4 pi (eq. ps2_phi_theta)."""
    L = oracle.lib()
    for (m0, m1, m2) in [(1000.0, 0.0, 0.0), (1000.0, 173.0, 173.0), (200.0, 80.4, 91.2)]:
        s = m0 * m0
        lam = (s - m1 ** 2 - m2 ** 2) ** 2 - 4 * m1 ** 2 * m2 ** 2
        j = L.orc_two_body_decay(_arr([m0, 0, 0, 0]), s, m1, m2, 0.3, 0.6, _arr([0] * 4), _arr([0] * 4))
        assert j == pytest.approx(math.sqrt(lam) / (8 * s) * 4 * math.pi, rel=1e-14)


@pytest.mark.parametrize("nu", [0.0, 0.3, 0.8, 1.0, 1.5])
@pytest.mark.parametrize("m2,xmin,xmax", [(-1e-3, 0.0, 1.69e8), (0.0, 6400.0, 1.69e8), (100.0, 400.0, 9000.0)])
def test_power_law_map_pins(nu, m2, xmin, xmax):
    """G_nu (eqs. prop_stable_nu, prop_stable_nu1, prop_flat): the weight of the
    integrand (x - m^2)^-nu is constant, the map is monotone onto [xmin, xmax],
    and int_0^1 J dr = xmax - xmin (Gauss-Legendre)."""
    L = oracle.lib()
    j = C.c_double()
    r, wq = _gl(400)
    xs, js = [], []
    for ri in r:
        xs.append(L.orc_map_nu(ri, m2, nu, xmin, xmax, C.byref(j)))
        js.append(j.value)
    xs, js = np.array(xs), np.array(js)
    assert np.all(np.diff(xs) > 0) and xs[0] >= xmin and xs[-1] <= xmax
    assert L.orc_map_nu(0.0, m2, nu, xmin, xmax, C.byref(j)) == pytest.approx(xmin, rel=1e-12, abs=1e-9)
    assert L.orc_map_nu(1.0, m2, nu, xmin, xmax, C.byref(j)) == pytest.approx(xmax, rel=1e-12)
    if nu == 1.0:
        const = js / (xs - m2)
        expect = math.log((xmax - m2) / (xmin - m2))
    else:
        const = js * (xs - m2) ** (-nu)
        e = 1 - nu
        expect = ((xmax - m2) ** e - (xmin - m2) ** e) / e
    assert np.allclose(const, expect, rtol=1e-13)
    if nu in (0.0, 0.3):  # smooth enough for the quadrature to converge
        # an endpoint singularity r^0.43 when xmin - m^2 is tiny slows the rule
        tol = 1e-11 if xmin - m2 >= 1.0 else 1e-7
        assert float(np.dot(js, wq)) == pytest.approx(xmax - xmin, rel=tol)


@pytest.mark.parametrize("m,w,xmin,xmax", [(173.0, 1.5, 0.0, 1e6), (80.4, 2.1, 100.0, 30000.0),
                                           (91.19, 2.5, 8000.0, 8400.0)])
def test_breit_wigner_map_pins(m, w, xmin, xmax):
    """G_BW (eq. prop_massive): f_BW J = (u2 - u1)/(m Gamma) for every r."""
    L = oracle.lib()
    j = C.c_double()
    u1, u2 = math.atan((xmin - m * m) / (m * w)), math.atan((xmax - m * m) / (m * w))
    rng = np.random.default_rng(0)
    for r in rng.random(200):
        x = L.orc_map_bw(r, m, w, xmin, xmax, C.byref(j))
        assert xmin <= x <= xmax
        f = 1.0 / ((x - m * m) ** 2 + (m * w) ** 2)
        assert f * j.value == pytest.approx((u2 - u1) / (m * w), rel=1e-12)


def _block_inputs(kind, rng):
    rs = 800.0
    if kind == "com":
        return [rs / 2, 0, 0, rs / 2], [rs / 2, 0, 0, -rs / 2], 0.0, 0.0
    if kind == "massive":
        return [rs / 2, 0, 0, rs / 2], [rs / 2, 0, 0, -rs / 2], 173.0, 240.0
    # spacelike p_A after a previous emission, boosted system
    pa = np.array([rs / 2, 0, 0, rs / 2])
    k = np.array([150.0, 60.0, -40.0, 120.0])
    k[0] = math.sqrt(k[1] ** 2 + k[2] ** 2 + k[3] ** 2)
    return list(pa - k), [rs / 2, 0, 0, -rs / 2], 30.0, 0.0


@pytest.mark.parametrize("kind", ["com", "massive", "spacelike"])
def test_two_to_two_block_invariants(kind):
    """(phi, t) block (section 2.2.4): (p_A - p1)^2 = -|t|, p1^2 = m1^2,
    p2^2 = m2^2, p1 + p2 = p_A + p_B; |t| range from cos(theta) = +-1."""
    L = oracle.lib()
    rng = np.random.default_rng(1)
    pA, pB, m1, m2 = _block_inputs(kind, rng)
    P = [pA[c] + pB[c] for c in range(4)]
    inv = (_minkowski(P), _minkowski(pA), _minkowski(pB))
    tlo, thi = C.c_double(), C.c_double()
    L.orc_t_range(*inv, m1, m2, C.byref(tlo), C.byref(thi))
    for _ in range(50):
        p1, p2, at = _arr([0] * 4), _arr([0] * 4), C.c_double()
        L.orc_two_to_two(_arr(pA), _arr(pB), *inv, m1, m2, rng.random(), rng.random(), 0.8, 1e-3,
                         p1, p2, C.byref(at))
        E = max(abs(x) for x in P)
        q = [pA[c] - p1[c] for c in range(4)]
        assert _minkowski(q) == pytest.approx(-at.value, abs=1e-10 * E * E)
        assert tlo.value - 1e-9 * E * E <= at.value <= thi.value + 1e-9 * E * E
        assert _minkowski(p1) == pytest.approx(m1 * m1, abs=1e-10 * E * E)
        assert _minkowski(p2) == pytest.approx(m2 * m2, abs=1e-10 * E * E)
        for c in range(4):
            assert p1[c] + p2[c] == pytest.approx(P[c], abs=1e-12 * E)
    if kind == "com":
        s = _minkowski(P)
        assert tlo.value == pytest.approx(0.0, abs=1e-9) and thi.value == pytest.approx(s, rel=1e-14)
    if kind == "massive":
        # explicit construction: p1 along +-z in the centre-of-mass frame
        s = _minkowski(P)
        rs = math.sqrt(s)
        lam = (s - m1 ** 2 - m2 ** 2) ** 2 - 4 * m1 ** 2 * m2 ** 2
        e1, q = (s + m1 ** 2 - m2 ** 2) / (2 * rs), math.sqrt(lam) / (2 * rs)
        for sign, ref in [(1, tlo.value), (-1, thi.value)]:
            p1 = [e1, 0, 0, sign * q]
            t = _minkowski([pA[c] - p1[c] for c in range(4)])
            assert -t == pytest.approx(ref, rel=1e-12)


@pytest.mark.parametrize("kind", ["com", "massive", "spacelike"])
def test_two_to_two_jacobian_integrates_to_two_body_volume(kind):
    """int dr_phi dr_t J_block = pi sqrt(lambda(m0^2, m1^2, m2^2))/(2 m0^2), the
    (phi, theta) measure, for any nu (eqs. ps2_phi_t vs ps2_phi_theta); with
    nu = 0 the Jacobian is that constant for massless legs."""
    L = oracle.lib()
    pA, pB, m1, m2 = _block_inputs(kind, np.random.default_rng(2))
    P = [pA[c] + pB[c] for c in range(4)]
    s = _minkowski(P)
    inv = (s, _minkowski(pA), _minkowski(pB))
    lam = (s - m1 ** 2 - m2 ** 2) ** 2 - 4 * m1 ** 2 * m2 ** 2
    expect = math.pi * math.sqrt(lam) / (2 * s)
    r, wq = _gl(200)
    for nu in (0.0, 0.3):
        tot = 0.0
        for ri, wi in zip(r, wq):
            j = L.orc_two_to_two(_arr(pA), _arr(pB), *inv, m1, m2, 0.37, ri, nu, 1e-3,
                                 _arr([0] * 4), _arr([0] * 4), None)
            tot += wi * j
            if nu == 0.0 and kind == "com":
                assert j == pytest.approx(math.pi / 2, rel=1e-14)
        # nu = 0.3 with the regulator has an r^0.43 endpoint singularity
        assert tot == pytest.approx(expect, rel=1e-6 if nu else 1e-13)


def test_r_to_x1x2_toy_pdf_closed_form():
    """int_0^1 dr s_lab J_x f(x1) f(x2) with f(x) = x^-1.2 (1-x)^3 equals
    tau^-1.2 int_tau^1 dx/x (1-x)^3 (1-tau/x)^3, expanded term by term
    (eqs. pdf_conv, pdf_sampling)."""
    L = oracle.lib()
    s_lab = 1.69e8
    for shat in (6400.0, 1e6, 5e7):
        tau = shat / s_lab
        closed = 0.0
        for i in range(4):
            for j in range(4):
                c = math.comb(3, i) * math.comb(3, j) * (-1) ** (i + j) * tau ** j
                pw = i - j
                closed += c * (-math.log(tau) if pw == 0 else (1 - tau ** pw) / pw)
        closed *= tau ** -1.2
        r, wq = _gl(300)
        x1, x2 = C.c_double(), C.c_double()
        tot = 0.0
        for ri, wi in zip(r, wq):
            jx = L.orc_r_to_x1x2(ri, shat, s_lab, C.byref(x1), C.byref(x2))
            assert x1.value * x2.value == pytest.approx(tau, rel=1e-14)
            f = lambda x: x ** -1.2 * (1 - x) ** 3
            tot += wi * s_lab * jx * f(x1.value) * f(x2.value)
        assert tot == pytest.approx(closed, rel=1e-12)


# --------------------------------------------------------------------------
# Channels
# --------------------------------------------------------------------------

def test_c1_every_weight_is_two_body_volume():
    """For f = 1 every e+e- -> mu+mu- event weighs Phi_2 = 1/(8 pi)."""
    P = oracle.Process(W.c1_ee_mumu(integrand="unit"))
    y = W.philox_uniforms(1, 0, 0, 20000, P.dims[0])
    out = P.map(0, y, P.uniform_grid(0))
    assert np.allclose(out["jac"], 1 / (8 * math.pi), rtol=1e-14, atol=0)
    assert np.allclose(out["w"], 1 / (8 * math.pi), rtol=1e-14, atol=0)


def test_c1_angular_integral_exact_by_quadrature():
    """int dPhi_2 (1 + cos^2 theta) = 1/(6 pi) (16 pi/3 in dOmega units):
    Gauss-Legendre over r_theta integrates the polynomial exactly."""
    P = oracle.Process(W.c1_ee_mumu())
    r, wq = _gl(8)
    y = np.stack([np.full_like(r, 0.123), r])  # dims: (r_phi, r_theta) of the decay
    out = P.map(0, y, None)
    assert float(np.dot(out["w"], wq)) == pytest.approx(1 / (6 * math.pi), rel=1e-14)
    y = W.philox_uniforms(1, 0, 0, 100000, 2)
    w = P.map(0, y, P.uniform_grid(0))["w"]
    mc, err = w.mean(), w.std() / math.sqrt(w.size)
    assert abs(mc - 1 / (6 * math.pi)) < 4 * err
    # massless: dPhi_2 = dOmega / (32 pi^2)
    assert abs(mc * 32 * math.pi ** 2 - 16 * math.pi / 3) < 4 * err * 32 * math.pi ** 2


def _mc_volume(P, chan, n, seed):
    y = W.philox_uniforms(seed, 1, 0, n, P.dims[chan])
    w = P.map(chan, y, None)["w"]
    return w.mean(), w.std() / math.sqrt(n)


@pytest.mark.parametrize("chan", range(8))
def test_massless_four_body_volume_per_channel(chan):
    """Each 2->4 topology (pure t, mixed, pure s) at E_CM = 1 TeV, nu = 0.3,
    f = 1, reproduces the analytic volume (section 4.1) within 4 sigma."""
    P = oracle.Process(W.volume_process(4))
    mean, err = _mc_volume(P, chan, 400000, seed=10 + chan)
    assert err / mean < 3e-3
    assert abs(mean - massless_volume(4, 1000.0)) < 4 * err


@pytest.mark.parametrize("n,chan", [(3, {"t_chain": [1, 2, 3], "t_order": "B"}),
                                    (5, {"t_chain": [1, {"d": [2, 3]}, 4, 5], "t_order": "BA"}),
                                    (6, {"t_chain": [1, 2, 3, 4, 5, 6], "t_order": "ABBA"}),
                                    (6, {"s": {"d": [{"d": [1, {"d": [2, 3]}]}, {"d": [4, {"d": [5, 6]}]}]}})])
def test_massless_volume_other_multiplicities(n, chan):
    P = oracle.Process(W.volume_process(n, channels=[chan]))
    mean, err = _mc_volume(P, 0, 400000, seed=40 + n)
    assert abs(mean - massless_volume(n, 1000.0)) < 4 * err


def test_volume_preserved_by_random_vegas_grid():
    """A VEGAS grid only re-parametrises the unit cube: with random edges the
    massless four-body volume is unchanged (catches a dropped J_v)."""
    P = oracle.Process(W.volume_process(4))
    rng = np.random.default_rng(13)
    nb = P.nbins
    grid = np.stack([np.concatenate([[0.0], np.sort(rng.random(nb - 1)), [1.0]]) for _ in range(P.dims[3])])
    y = W.philox_uniforms(31, 1, 0, 600000, P.dims[3])
    w = P.map(3, y, grid)["w"]
    mean, err = w.mean(), w.std() / math.sqrt(w.size)
    assert abs(mean - massless_volume(4, 1000.0)) < 4 * err


def test_multichannel_volume_alpha_weighted():
    """SDE multichannel (eq. multi-channel-mg): sum_c E_c[alpha_c J_c] equals the
    volume, which holds only if sum_c alpha_c(x) = 1 at every point."""
    P = oracle.Process(W.volume_process(4, alpha_mu=10.0))
    tot, var = 0.0, 0.0
    for c in range(8):
        y = W.philox_uniforms(20 + c, 1, 0, 300000, P.dims[c])
        w = P.map(c, y, None)["w"]
        tot += w.mean()
        var += w.var() / w.size
    assert abs(tot - massless_volume(4, 1000.0)) < 4 * math.sqrt(var)


def test_massive_two_body_volume():
    """t tbar at sqrt(s) = 1 TeV: every weight equals pi sqrt(lambda)/(2 s) (2 pi)^-2."""
    desc = W.volume_process(2, channels=[{"s": {"d": [1, 2]}}])
    desc["masses"] = [173.0, 173.0]
    P = oracle.Process(desc)
    y = W.philox_uniforms(2, 0, 0, 1000, 2)
    out = P.map(0, y, None)
    s = 1e6
    lam = s * s - 4 * s * 173.0 ** 2
    assert np.allclose(out["w"], math.pi * math.sqrt(lam) / (2 * s) / (2 * math.pi) ** 2, rtol=1e-13)
    p = out["p"]
    assert np.allclose(np.sqrt(p[1, 2] ** 2 + p[2, 2] ** 2 + p[3, 2] ** 2), 0.5 * math.sqrt(s - 4 * 173.0 ** 2), rtol=1e-13)


@pytest.mark.parametrize("cfg", ["c1", "c2", "c3"])
def test_conservation_and_on_shell_every_event(cfg):
    P = oracle.Process(W.CONFIG_NAMES[cfg]())
    for c in range(len(P.channels)):
        y = W.philox_uniforms(3, 0, 0, 20000, P.dims[c])
        out = P.map(c, y, P.uniform_grid(c))
        p = out["p"]
        emax = np.abs(p[0]).max(axis=0)
        bal = p[:, 0] + p[:, 1] - p[:, 2:].sum(axis=1)
        assert np.all(np.abs(bal) <= 1e-12 * emax)
        for i, m in enumerate(P.masses):
            m2 = p[0, i + 2] ** 2 - p[1, i + 2] ** 2 - p[2, i + 2] ** 2 - p[3, i + 2] ** 2
            assert np.all(np.abs(m2 - m * m) <= 1e-12 * emax ** 2)
        assert np.all(np.isfinite(out["w"])) and np.all(out["w"] >= 0)
        if P.hadronic:
            x1, x2 = out["x1x2"]
            s = p[0, 0] + p[0, 1]
            # incoming momenta are x_i * sqrt(s_lab)/2 along the beams
            assert np.allclose(p[0, 0], x1 * math.sqrt(P.s_lab) / 2, rtol=1e-13)
            assert np.allclose(p[0, 1], x2 * math.sqrt(P.s_lab) / 2, rtol=1e-13)


@pytest.mark.parametrize("chan", [0, 1, 2, 3, 4, 5])
def test_t_chain_samples_the_spine_propagators(chan):
    """Every 2->2 block samples one t-channel propagator of the diagram,
    q_j = p_a - sum_{i<=j} P(leg_i) along the spine (section 2.2.8 with the
    leg update p_A -> p_A - p1 / p_B -> p_B - p2): the sampled |t| values are
    exactly {-q_j^2}, whatever the A/B generation order."""
    P = oracle.Process(W.c2_pp4j())
    ch = P.channels[chan]
    y = W.philox_uniforms(8, 0, 0, 5000, P.dims[chan])
    out = P.map(chan, y, None, want_inv=True)
    p = out["p"]
    pa = p[:, 0]
    legs = ch.children[0]
    acc = np.zeros_like(pa)
    spine = []
    for leg in legs[:-1]:
        for k in ch.particles(leg):
            acc = acc + p[:, k + 2]
        q = pa - acc
        spine.append(-(q[0] ** 2 - q[1] ** 2 - q[2] ** 2 - q[3] ** 2))
    spine = np.sort(np.array(spine), axis=0)
    got = np.sort(out["tabs"], axis=0)
    scale = (p[0, 0] + p[0, 1]) ** 2
    assert np.all(np.abs(spine - got) <= 1e-10 * scale)


def _massive_three_body_volume(S, m1, m2, m3):
    """Phi_3 = int ds/(2 pi) Phi_2(S; m1, sqrt(s)) Phi_2(s; m2, m3) by Gauss-Legendre
    (recursive factorisation of the n-body measure), Phi_2 = sqrt(lambda)/(8 pi S)."""
    def phi2(s, a, b):
        lam = (s - a * a - b * b) ** 2 - 4 * a * a * b * b
        return math.sqrt(max(lam, 0.0)) / (8 * math.pi * s)
    lo, hi = (m2 + m3) ** 2, (math.sqrt(S) - m1) ** 2
    x, wq = _gl(400, lo, hi)
    return sum(wi * phi2(S, m1, math.sqrt(xi)) * phi2(xi, m2, m3) for xi, wi in zip(x, wq)) / (2 * math.pi)


@pytest.mark.parametrize("order", ["A", "B"])
def test_massive_t_chain_volume(order):
    """A t-chain with massive legs (bound s_max,i = (sqrt(s_{i-1}) - m_sigma(i))^2)
    reproduces the massive three-body volume, and no event is unphysical."""
    desc = W.volume_process(3, channels=[{"t_chain": [1, 2, 3], "t_order": order}])
    desc["masses"] = [173.0, 10.0, 173.0]
    P = oracle.Process(desc)
    y = W.philox_uniforms(50, 1, 0, 400000, P.dims[0])
    out = P.map(0, y, None)
    assert np.all(out["jac"] > 0)
    w = out["w"]
    mean, err = w.mean(), w.std() / math.sqrt(w.size)
    ref = _massive_three_body_volume(1e6, 173.0, 10.0, 173.0)
    assert abs(mean - ref) < 4 * err


def test_c3_sampled_invariants_match_final_momenta():
    """Each resonance invariant equals the mass^2 of its decay products, and
    the s-channel bounds hold: sqrt(s_parent) >= sum of children masses."""
    P = oracle.Process(W.c3_ttbar6())
    y = W.philox_uniforms(4, 0, 0, 20000, P.dims[0])
    out = P.map(0, y, P.uniform_grid(0), want_inv=True)
    ch = P.channels[0]
    p = out["p"]
    for j in range(len(ch.kind)):
        if ch.kind[j] != oracle.CLUSTER:
            continue
        parts = ch.particles(j)
        q = p[:, [k + 2 for k in parts]].sum(axis=1)
        m2 = q[0] ** 2 - q[1] ** 2 - q[2] ** 2 - q[3] ** 2
        scale = q[0] ** 2
        assert np.all(np.abs(m2 - out["inv"][j]) <= 1e-11 * scale)
        kids = ch.children[j]
        mk = sum(np.sqrt(out["inv"][k]) if ch.kind[k] == oracle.CLUSTER else 0.0 for k in kids)
        assert np.all(np.sqrt(out["inv"][j]) >= mk * (1 - 1e-14))


def test_paper_compute_graph_example():
    """The 2->3 example of the compute-graph figure: seven random numbers in the
    printed order (s-hat, s, x1, r_phi, r_t, r_phi, r_theta), five momenta out,
    and the Jacobian equals 0.000102118 x the product of the printed factors
    evaluated with the printed arguments (s_lab = 1.69e8, nu = 0.8)."""
    g = {}
    for line in open(os.path.join(GOLDEN, "compute_graph_2to3.txt")):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            g[k] = float(v)
    P = oracle.Process(W.paper_example_2to3())
    assert P.dims[0] == int(g["n_random_dims"])
    assert P.n + 2 == int(g["n_momenta_out"])
    assert P.s_lab == g["s_lab"] and P.nu == g["nu"]
    L = oracle.lib()
    a = P.reg_a
    rng = np.random.default_rng(5)
    y = rng.random((7, 300))
    out = P.map(0, y, None)
    j = C.c_double()
    for e in range(y.shape[1]):
        r = y[:, e]
        shat = L.orc_map_nu(r[0], -a, g["nu"], 0.0, g["s_lab"], C.byref(j)); j12 = j.value
        s = L.orc_map_nu(r[1], -a, g["nu"], 0.0, shat, C.byref(j)); j15 = j.value
        x1, x2 = C.c_double(), C.c_double()
        j19 = L.orc_r_to_x1x2(r[2], shat, g["s_lab"], C.byref(x1), C.byref(x2))
        h = math.sqrt(shat) / 2
        pa, pb = _arr([h, 0, 0, h]), _arr([h, 0, 0, -h])
        p26, p27 = _arr([0] * 4), _arr([0] * 4)
        j29 = L.orc_two_to_two(pa, pb, shat, 0.0, 0.0, math.sqrt(s), 0.0, r[3], r[4], g["nu"], a,
                               p26, p27, None)
        j33 = L.orc_two_body_decay(p26, s, 0.0, 0.0, r[5], r[6], _arr([0] * 4), _arr([0] * 4))
        expect = g["reduce_product_constant"] * j12 * j15 * j19 * j29 * j33 * 1.0
        if out["jac"][e] > 0:
            assert out["jac"][e] == pytest.approx(expect, rel=5e-6)
    assert (out["jac"] > 0).mean() > 0.99


# --------------------------------------------------------------------------
# VEGAS
# --------------------------------------------------------------------------

def test_vegas_uniform_grid_is_identity():
    P = oracle.Process(W.c2_pp4j())
    y = W.philox_uniforms(6, 0, 0, 5000, 10)
    a = P.map(0, y, P.uniform_grid(0))
    b = P.map(0, y, None)
    assert np.array_equal(a["jac"], b["jac"])  # J_v = 64 * (1/64) = 1 exactly


def test_vegas_jacobian_averages_to_one_on_any_grid():
    """E[J_v] = 1: the bin-midpoint rule is exact since J_v is constant per bin."""
    L = oracle.lib()
    rng = np.random.default_rng(7)
    nb = 64
    e = np.concatenate([[0.0], np.sort(rng.random(nb - 1)), [1.0]])
    ea = (C.c_double * (nb + 1))(*e)
    j = C.c_double()
    tot = 0.0
    for i in range(nb):
        x = L.orc_vegas_map((i + 0.5) / nb, ea, nb, C.byref(j))
        assert e[i] <= x <= e[i + 1]
        tot += j.value / nb
    assert tot == pytest.approx(1.0, rel=1e-14)


def test_vegas_refine_fixed_point_and_edges():
    nb = 64
    edges = np.tile(np.arange(nb + 1) / nb, (3, 1))
    out = oracle.vegas_refine(edges, np.full((3, nb), 2.5), alpha=0.5)
    assert np.allclose(out, edges, atol=1e-15, rtol=0)
    rng = np.random.default_rng(8)
    d = rng.random((3, nb)) ** 4
    out = oracle.vegas_refine(edges, d, alpha=1.0)
    assert np.all(out[:, 0] == 0.0) and np.all(out[:, -1] == 1.0)
    assert np.all(np.diff(out, axis=1) > 0)


def _vegas_fixed_point_linear(nb):
    """Grid whose bins carry equal sum of w^2 for f(x) = 2x with a
    piecewise-constant density: Delta_i (e_{i+1}^3 - e_i^3) = K for all i, K
    found by bisection so that the last edge is 1 (brute force)."""
    def last_edge(K):
        e = 0.0
        for _ in range(nb):
            lo, hi = e, 2.0
            for _ in range(100):
                mid = 0.5 * (lo + hi)
                if (mid - e) * (mid ** 3 - e ** 3) < K:
                    lo = mid
                else:
                    hi = mid
            e = 0.5 * (lo + hi)
        return e

    lo, hi = 0.0, 1.0
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        if last_edge(mid) < 1.0:
            lo = mid
        else:
            hi = mid
    K = 0.5 * (lo + hi)
    edges = [0.0]
    for _ in range(nb):
        e = edges[-1]
        a, b = e, 2.0
        for _ in range(100):
            mid = 0.5 * (a + b)
            if (mid - e) * (mid ** 3 - e ** 3) < K:
                a = mid
            else:
                b = mid
        edges.append(0.5 * (a + b))
    return np.array(edges)


def test_vegas_converges_to_optimal_grid_for_linear_integrand():
    """For f(x) = 2x the refinement converges to the grid on which every bin
    collects the same sum of w^2 (close to sqrt(i/N), exact in the fine-bin
    limit)."""
    L = oracle.lib()
    nb = 32
    edges = np.arange(nb + 1, dtype=np.float64) / nb
    rng = np.random.default_rng(9)
    j = C.c_double()
    for it in range(30):
        y = (np.arange(20000) + rng.random(20000)) / 20000
        ea = (C.c_double * (nb + 1))(*edges)
        w = np.empty_like(y)
        for i, yi in enumerate(y):
            x = L.orc_vegas_map(yi, ea, nb, C.byref(j))
            w[i] = 2 * x * j.value
        d = oracle.vegas_histogram(y[None, :], w, nb)
        edges = oracle.vegas_refine(edges[None, :], d, alpha=1.0)[0]
    assert np.allclose(edges, _vegas_fixed_point_linear(nb), atol=2e-3)
    assert np.allclose(edges[4:], np.sqrt(np.arange(4, nb + 1) / nb), atol=1e-2)


def test_vegas_histogram_brute_force():
    rng = np.random.default_rng(10)
    y = rng.random((2, 50))
    w = rng.random(50)
    d = oracle.vegas_histogram(y, w, 4)
    for k in range(2):
        for b in range(4):
            expect = sum(w[e] ** 2 for e in range(50) if b / 4 <= y[k, e] < (b + 1) / 4)
            assert d[k, b] == pytest.approx(expect, rel=1e-14)


# --------------------------------------------------------------------------
# Unweighting efficiency and statistics
# --------------------------------------------------------------------------

def _bisect_wmax(w, frac):
    lo, hi = 0.0, float(np.max(w))
    target = frac * float(np.sum(w))
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if np.maximum(w - mid, 0.0).sum() > target:
            lo = mid
        else:
            hi = mid
    return hi


def test_unweighting_brute_force_and_closed_forms():
    # equal weights w: N (w - W) = 1e-3 N w  ->  W = w (1 - 1e-3), eps = 1/(1 - 1e-3)
    eff, W1 = oracle.unweighting_efficiency(np.full(1000, 3.0))
    assert W1 == pytest.approx(3.0 * (1 - 1e-3), rel=1e-12)
    assert eff == pytest.approx(1 / (1 - 1e-3), rel=1e-12)
    rng = np.random.default_rng(11)
    for n in (1, 2, 7, 100):
        w = rng.random(n) ** 3
        eff, Wm = oracle.unweighting_efficiency(w, 0.1)
        assert Wm == pytest.approx(_bisect_wmax(w, 0.1), rel=1e-12)
        assert eff == pytest.approx(w.mean() / Wm, rel=1e-14)
    # w ~ Exp(1): E[(w - W)+] = exp(-W) = 1e-3 -> W = ln(1000), eps = 1/ln(1000)
    w = rng.exponential(size=2_000_000)
    eff, Wm = oracle.unweighting_efficiency(w, 1e-3)
    assert Wm == pytest.approx(math.log(1000.0), rel=0.02)
    assert eff == pytest.approx(1 / math.log(1000.0), rel=0.02)


def test_integral_and_error_from_stats():
    rng = np.random.default_rng(12)
    ws = [rng.random(1000), 2 * rng.random(3000)]
    st = np.array([oracle.channel_stats(w) for w in ws])
    I, err = oracle.integral(st)
    assert I == pytest.approx(ws[0].mean() + ws[1].mean(), rel=1e-13)
    assert err == pytest.approx(math.sqrt(ws[0].var(ddof=1) / 1000 + ws[1].var(ddof=1) / 3000), rel=1e-10)
    assert st[0, 4] == ws[0].max() and st[0, 3] == 0


# --------------------------------------------------------------------------
# Input generator
# --------------------------------------------------------------------------

def test_philox_uniforms_addressing_and_range():
    a = W.philox_uniforms(9, 3, 0, 1000, 7)
    b = W.philox_uniforms(9, 3, 500, 500, 7)
    assert np.array_equal(a[:, 500:], b)
    assert a.min() > 0 and a.max() < 1
    big = W.philox_uniforms(1, 0, 0, 400000, 1)[0]
    assert abs(big.mean() - 0.5) < 4 * math.sqrt(1 / 12 / big.size)
    assert abs(big.var() - 1 / 12) < 0.002
    hist = np.bincount((big * 64).astype(int), minlength=64)
    chi2 = ((hist - big.size / 64) ** 2 / (big.size / 64)).sum()
    assert chi2 < 120  # 63 dof


@pytest.mark.parametrize("cfg,bound,median", [("c1", 1e-14, 1e-15), ("c2", 1e-7, 1e-11), ("c3", 1e-8, 1e-10)])
def test_fp64_forward_error_stays_bounded(cfg, bound, median):
    """Two roundings of the same formulas (SSE2 and x87 builds, plus one-ulp
    input moves) agree closely: the t-range roots come from the product of
    roots and the blocks use the sampled invariants, so no event loses more
    than a few digits.  (Evaluated naively from momenta, some pure t-channel
    events disagreed at the 1e-1 level.)"""
    P = oracle.Process(W.CONFIG_NAMES[cfg]())
    for c in range(len(P.channels)):
        y = W.philox_uniforms(2, 0, 0, 50000, P.dims[c])
        fe = P.forward_error(c, y, P.uniform_grid(c))
        assert fe["w"].max() < bound
        assert fe["p"].max() < 1e-4
        assert np.median(fe["w"]) < median
