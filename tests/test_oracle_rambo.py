"""Pins of the oracle's FastRambo (section 2.2.9): the single-bin
rational-quadratic map, its table of slopes, and the massless n-body
phase space it generates."""
import math
import os

import numpy as np
import pytest
from scipy import integrate, optimize

import oracle
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "rambo_fit.txt")


def _table():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    return {int(k): float(c) for k, c in rows}


def test_ck_table_matches_the_paper():
    L = oracle.lib()
    for k, c in _table().items():
        assert L.orc_rambo_ck(k) == c


def test_ck_table_is_the_least_squares_fit():
    """c_k* minimises the integral of (G_RQF(y, c) - G_diet(y, k))^2 over
    [0, 1] with G_diet(y, k) = (k + 1) y - k y^(1 + 1/k) (eq. r_to_x_orig);
    the fit through the oracle's G_RQF reproduces the paper's table."""
    L = oracle.lib()
    for k, c_paper in _table().items():
        def loss(c):
            return integrate.quad(lambda y: (L.orc_rqf(y, c) - ((k + 1) * y - k * y ** (1 + 1 / k))) ** 2,
                                  0.0, 1.0, epsabs=1e-14, epsrel=1e-12)[0]
        res = optimize.minimize_scalar(loss, bounds=(1.0, 6.0), method="bounded",
                                       options={"xatol": 1e-9})
        assert res.x == pytest.approx(c_paper, abs=2e-6), (k, res.x)


def test_rqf_closed_forms():
    L = oracle.lib()
    for y in np.linspace(0.0, 1.0, 21):
        # k = 1, c = 2: the RamboOnDiet map 2y - y^2 itself
        assert L.orc_rqf(y, 2.0) == pytest.approx(2 * y - y * y, abs=1e-15)
        for c in (0.5, 2.712001, 3.662872):
            r = L.orc_rqf(y, c)
            assert L.orc_rqf_inverse(r, c) == pytest.approx(y, abs=1e-14)
    # endpoint slopes c and 0
    h = 1e-7
    assert (L.orc_rqf(h, 3.0) - L.orc_rqf(0.0, 3.0)) / h == pytest.approx(3.0, rel=1e-5)
    assert (L.orc_rqf(1.0, 3.0) - L.orc_rqf(1.0 - h, 3.0)) / h == pytest.approx(0.0, abs=1e-5)


def _massless_volume(n, s):
    return (2 * math.pi) ** (4 - 3 * n) * (math.pi / 2) ** (n - 1) * s ** (n - 2) / (math.gamma(n) * math.gamma(n - 1))


def test_three_body_is_exactly_flat():
    pr = oracle.Process(W.rambo_process(3))
    out = pr.map(0, W.philox_uniforms(3, 3, 0, 5000, pr.dims[0]))
    assert np.allclose(out["jac"], _massless_volume(3, 1e6), rtol=1e-12, atol=0)


@pytest.mark.parametrize("n", [4, 5, 6, 8])
def test_massless_volume_and_near_flatness(n):
    """The mean weight is the massless n-body volume (within 4 standard
    errors); the weights are close to flat (the local factor w_n of eq.
    mass_measure_rqs: measured spread 4-14%)."""
    pr = oracle.Process(W.rambo_process(n))
    out = pr.map(0, W.philox_uniforms(2, n, 0, 100000, pr.dims[0]))
    j = out["jac"]
    V = _massless_volume(n, 1e6)
    assert abs(j.mean() - V) < 4.0 * j.std() / np.sqrt(j.size)
    assert j.std() / j.mean() < 0.2 and j.min() > 0.3 * V and j.max() < 2.5 * V
    p = out["p"]
    assert np.abs(p[0, 2:].sum(axis=0) - 1000.0).max() < 1e-11
    assert np.abs(p[1:, 2:].sum(axis=1)).max() < 1e-11
    m2 = p[0, 2:] ** 2 - p[1, 2:] ** 2 - p[2, 2:] ** 2 - p[3, 2:] ** 2
    assert np.abs(m2).max() < 1e-14 * 1e6


def test_round_trip():
    pr = oracle.Process(W.rambo_process(6))
    y = W.philox_uniforms(7, 1, 0, 20000, pr.dims[0])
    out = pr.map(0, y)
    inv = pr.inverse(0, out["p"], None)
    err = np.abs(inv["y"] - y).max(axis=0)
    assert np.median(err) < 1e-14 and err.max() < 1e-9
    assert np.median(np.abs(inv["jac"] / out["jac"] - 1)) < 1e-13


@pytest.mark.parametrize("masses", [[100.0, 50.0, 0.0], [173.0, 173.0, 80.0, 5.0], [10.0, 20.0, 30.0, 40.0, 50.0]])
def test_massive_volume_matches_the_decay_chain(masses):
    """With masses the FastRambo cluster map (M_i = mu_i + u_i (M_{i-1} -
    m_{i-1} - mu_i), the massless chain of K_i = M_i - mu_i) and the power-law
    decay chain of the same topology estimate the same massive n-body volume
    (two independent estimators): agreement within 4 combined standard
    errors, FastRambo with the smaller spread."""
    n = len(masses)
    est = []
    for rb in (True, False):
        pr = oracle.Process(W.rambo_process(n, masses=masses, rambo=rb))
        j = pr.map(0, W.philox_uniforms(2, n, 0, 400000, pr.dims[0]))["jac"]
        est.append((j.mean(), j.std() / np.sqrt(j.size), j.std() / j.mean()))
    (a, ea, sa), (b, eb, sb) = est
    assert abs(a - b) < 4.0 * np.hypot(ea, eb), est
    assert sa < sb
