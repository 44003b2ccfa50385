"""Pins of the oracle's 1 -> 3 decay (section 2.2.6).

The decay samples E1, E2 linearly in their ranges and the directions of p1
and of p2 about p1; p3 takes the rest.  Checked: the massless three-body
volume in closed form; massive volumes, also inside a hadronic t-channel
process, against the two-body decay chains of the same phase space; the
mass shell of p3 (which fixes the angle between p1 and p2) and momentum
conservation per event; the inverse round trip."""
import math

import numpy as np
import pytest

import oracle
import workloads as W


def _mc(desc, n=1_000_000, seed=1, key="jac"):
    o = oracle.Process(desc)
    y = W.philox_uniforms(seed, 0, 0, n, o.dims[0])
    f = o.map(0, y)
    w = f[key]
    return float(w.mean()), float(w.std() / math.sqrt(n)), f, y, o


def _proc(chan, masses):
    d = W.volume_process(len(masses), sqrt_s=1000.0, channels=[chan])
    d["masses"] = [float(m) for m in masses]
    return d


def test_massless_volume():
    m, e, f, _, o = _mc(_proc({"s": {"d": [1, 2, 3]}}, [0.0] * 3))
    assert o.dims == [5]
    exact = 1000.0 ** 2 / (256 * math.pi ** 3)  # Phi_3 = s / (256 pi^3)
    assert abs(m - exact) < 4.0 * e and e < 1e-3 * exact


@pytest.mark.parametrize("masses", [[10.0, 80.0, 173.0], [300.0, 0.0, 50.0], [0.0, 0.0, 400.0]])
def test_massive_against_two_body_chain(masses):
    a = _mc(_proc({"s": {"d": [1, 2, 3]}}, masses))
    b = _mc(_proc({"s": {"d": [1, {"d": [2, 3]}]}}, masses), seed=2)
    pull = (a[0] - b[0]) / math.hypot(a[1], b[1])
    assert abs(pull) < 4.0, (a[:2], b[:2])


def test_inside_hadronic_t_channel():
    """pp -> 4 with a massive three-body cluster on the t-channel spine,
    toy PDFs and a p_T cut, against the same cluster as nested two-body
    decays."""
    def desc(cl):
        d = W.chili_process(4, sqrt_s=13000.0, pt_min=20.0, pdf=[-1.2, 3.0])
        d["shat_min"] = 6400.0
        d["channels"] = [{"t_chain": [1, cl], "t_order": ""}]
        return d

    a = _mc(desc({"d": [2, 3, 4], "m": 300.0, "w": 20.0}), key="w")
    b = _mc(desc({"d": [2, {"d": [3, 4]}], "m": 300.0, "w": 20.0}), seed=2, key="w")
    pull = (a[0] - b[0]) / math.hypot(a[1], b[1])
    assert abs(pull) < 4.0, (a[:2], b[:2])


def test_kinematics_and_round_trip():
    masses = [10.0, 80.0, 173.0]
    _, _, f, y, o = _mc(_proc({"s": {"d": [1, 2, 3]}}, masses), n=100_000)
    p = f["p"]
    ok = f["jac"] > 0
    assert ok.all()
    assert np.abs(p[:, :2].sum(axis=1) - p[:, 2:].sum(axis=1)).max() < 1e-10
    for i, m in enumerate(masses):
        m2 = p[0, i + 2] ** 2 - (p[1:, i + 2] ** 2).sum(axis=0)
        assert np.abs(m2 - m * m).max() < 1e-9 * 1000.0 ** 2 / 4
    inv = o.inverse(0, p, None, o.uniform_grid(0))
    err = np.abs(inv["y"] - y).max(axis=0)
    assert np.median(err) < 1e-14 and err.max() < 1e-9
    jr = np.abs(inv["jac"] / f["jac"] - 1.0)
    assert np.median(jr) < 1e-14 and jr.max() < 1e-9


def test_fastrambo_cluster_must_be_binary():
    with pytest.raises(ValueError):
        oracle.Process(_proc({"s": {"d": [1, 2, 3], "rambo": True}}, [0.0] * 3))
