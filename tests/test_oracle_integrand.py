"""Pins of the oracle's toy integrand and local channel weights.

The toy integrand (the workloads' f: PDFs x propagator factors) and the
channel weights alpha_c (eq. multi-channel-mg, weights from the diagrams'
propagator denominators, section 2.1.1) are checked against closed forms that
do not evaluate the oracle's own formulas:

- a massless 2 -> 2 process with one t-channel factor 1/(|t| + mu^2), sampled
  by the log map whose auxiliary mass is mu^2, has a constant weight
  ln((s + mu^2)/mu^2) / (8 pi s) at every event (the integral of that factor
  over the two-body phase space, d Phi_2 = d|t| / (8 pi s));
- a Breit-Wigner factor on a Breit-Wigner-mapped invariant leaves the
  constant (u2 - u1)/(M Gamma) per event (eq. prop_massive), times Jacobians
  with closed forms (the PDF convolution's -log(tau)/s_lab, the two-body
  decay factors);
- the toy PDFs through the full hadronic chain integrate to a one-dimensional
  quadrature in tau of the elementary closed form of the PDF convolution
  (eqs. pdf_conv, pdf_sampling);
- every pp -> 4 jets channel's propagator set in alpha_c is listed by hand
  from its diagram, and the oracle's alpha_c at arbitrary momenta equals the
  ratio of the hand-listed denominator products.

Each check is a function of the oracle build, so that builds with planted
mistakes (oracle.build_mutant) can be shown to fail them.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

MU = 10.0


def _t_prop_process(nu=1.0, reg=MU * MU, particles=(1,)):
    return {"sqrt_s": 1000.0, "beams": "fixed", "masses": [0.0, 0.0], "nu": nu, "regulator": reg,
            "vegas_bins": 8, "integrand": {"props": [{"t": True, "particles": list(particles), "mu": MU}]},
            "channels": [{"t_chain": [1, 2]}]}


def check_t_propagator_weight(variant="ref"):
    """Every event: w = ln((s + mu^2)/mu^2) / (8 pi s).  The factor takes
    t = (p_a - p_1)^2 recomputed from the momenta, whose rounding (a few ulp
    of s) is relative to |t| + mu^2 >= mu^2: tolerance 64 u s / mu^2."""
    P = oracle.Process(_t_prop_process())
    s = P.s_lab
    y = W.philox_uniforms(61, 0, 0, 20000, P.dims[0])
    w = P.map(0, y, None, variant=variant)["w"]
    expect = math.log((s + MU * MU) / (MU * MU)) / (8 * math.pi * s)
    rel = np.abs(w / expect - 1.0)
    return bool(rel.max() < 64 * 2.0 ** -53 * s / MU ** 2), rel.max()


def check_t_propagator_massive(variant="ref"):
    """Massive t tbar at 1 TeV (massless beams): the log map with auxiliary
    mass mu^2 between the closed-form limits |t| = s/2 (1 -+ beta) - m^2 makes
    every weight ln((|t|max + mu^2)/(|t|min + mu^2)) / (8 pi s).  Unlike the
    massless case, the sign convention of q = p_a - p_1 matters here:
    (p_a + p_1)^2 = 2 m^2 + |t|."""
    m = 173.0
    desc = _t_prop_process()
    desc["masses"] = [m, m]
    P = oracle.Process(desc)
    s = P.s_lab
    beta = math.sqrt(1.0 - 4 * m * m / s)
    tmin, tmax = s / 2 * (1 - beta) - m * m, s / 2 * (1 + beta) - m * m
    y = W.philox_uniforms(66, 0, 0, 20000, P.dims[0])
    w = P.map(0, y, None, variant=variant)["w"]
    expect = math.log((tmax + MU * MU) / (tmin + MU * MU)) / (8 * math.pi * s)
    rel = np.abs(w / expect - 1.0)
    return bool(rel.max() < 64 * 2.0 ** -53 * s / (tmin + MU ** 2)), rel.max()


def check_t_propagator_integral(variant="ref"):
    """Default power-law |t| map (nu = 0.8, tiny regulator): the Monte Carlo
    integral equals ln((s + mu^2)/mu^2) / (8 pi s) within 4 standard errors."""
    P = oracle.Process(_t_prop_process(nu=0.8, reg=1e-3))
    s = P.s_lab
    y = W.philox_uniforms(62, 0, 0, 400000, P.dims[0])
    w = P.map(0, y, None, variant=variant)["w"]
    mean, err = w.mean(), w.std() / math.sqrt(w.size)
    expect = math.log((s + MU * MU) / (MU * MU)) / (8 * math.pi * s)
    return bool(abs(mean - expect) < 4 * err and err / mean < 2e-3), (mean / expect - 1, err / mean)


M_BW, G_BW = 91.19, 2.5


def _bw_hadronic_process():
    return {"sqrt_s": 13000.0, "beams": "hadronic", "shat_min": 1e4, "masses": [0.0, 0.0], "nu": 0.8,
            "regulator": 1e-3, "vegas_bins": 8,
            "integrand": {"props": [{"t": False, "particles": [1, 2], "bw": True, "m": M_BW, "w": G_BW}]},
            "channels": [{"s": {"d": [1, 2], "m": M_BW, "w": G_BW}}]}


def check_bw_hadronic(variant="ref"):
    """s-hat mapped by G_BW, f = Breit-Wigner of (p1 + p2)^2 = s-hat: every
    event weighs (u2 - u1)/(M Gamma) x (-log(x1 x2))/s_lab x 1/(8 pi)."""
    P = oracle.Process(_bw_hadronic_process())
    y = W.philox_uniforms(63, 0, 0, 20000, P.dims[0])
    out = P.map(0, y, None, variant=variant)
    mg = M_BW * G_BW
    u1, u2 = math.atan((1e4 - M_BW ** 2) / mg), math.atan((P.s_lab - M_BW ** 2) / mg)
    tau = out["x1x2"][0] * out["x1x2"][1]
    expect = (u2 - u1) / mg * (-np.log(tau)) / P.s_lab / (8 * math.pi)
    rel = np.abs(out["w"] / expect - 1.0)
    return bool(rel.max() < 1e-11), rel.max()


def _bw_chain_process():
    return {"sqrt_s": 1000.0, "beams": "fixed", "masses": [0.0, 0.0, 0.0], "nu": 0.8, "regulator": 1e-3,
            "vegas_bins": 8,
            "integrand": {"props": [{"t": False, "particles": [1, 2], "bw": True, "m": M_BW, "w": G_BW}]},
            "channels": [{"s": {"d": [{"d": [1, 2], "m": M_BW, "w": G_BW}, 3]}}]}


def check_bw_decay_chain(variant="ref"):
    """e+e- -> (12) 3 -> 1 2 3 at 1 TeV with s_12 mapped by G_BW: every event
    weighs (2 pi)^-5 (u2 - u1)/(M Gamma) x pi (s - s_12)/(2 s) x pi/2 (the
    two massless decay factors pi sqrt(lambda)/(2 m0^2)), s_12 = (p1 + p2)^2."""
    P = oracle.Process(_bw_chain_process())
    y = W.philox_uniforms(64, 0, 0, 20000, P.dims[0])
    out = P.map(0, y, None, variant=variant)
    s = P.s_lab
    q = out["p"][:, 2] + out["p"][:, 3]
    s12 = q[0] ** 2 - q[1] ** 2 - q[2] ** 2 - q[3] ** 2
    mg = M_BW * G_BW
    u1, u2 = math.atan((0.0 - M_BW ** 2) / mg), math.atan((s - M_BW ** 2) / mg)
    expect = (2 * math.pi) ** -5 * (u2 - u1) / mg * math.pi * (s - s12) / (2 * s) * math.pi / 2
    rel = np.abs(out["w"] / expect - 1.0)
    return bool(rel.max() < 1e-10), rel.max()


def _pdf_convolution_closed_form(tau, a=-1.2, b=3):
    """int_0^1 dr (-log tau) f(x1) f(x2), x1 = tau^r, x2 = tau^(1-r),
    f(x) = x^a (1-x)^b with integer b: tau^a int_tau^1 dx/x (1-x)^b (1-tau/x)^b
    expanded term by term."""
    tot = 0.0
    for i in range(b + 1):
        for j in range(b + 1):
            c = math.comb(b, i) * math.comb(b, j) * (-1) ** (i + j) * tau ** j
            pw = i - j
            tot += c * (-math.log(tau) if pw == 0 else (1 - tau ** pw) / pw)
    return tau ** a * tot


def check_pdf_full_chain(variant="ref"):
    """pp -> 2 massless at 13 TeV, f = toy PDFs only: the Monte Carlo integral
    over s-hat and the rapidity equals (1/(8 pi)) int dtau F(tau), F the
    closed form of the PDF convolution, by Gauss-Legendre in log tau."""
    tmin = 1e-4
    desc = {"sqrt_s": 13000.0, "beams": "hadronic", "shat_min": tmin * 1.69e8, "masses": [0.0, 0.0],
            "nu": 0.8, "regulator": 1e-3, "vegas_bins": 8, "integrand": {"pdf": [-1.2, 3.0]},
            "channels": [{"s": {"d": [1, 2]}}]}
    P = oracle.Process(desc)
    x, wq = np.polynomial.legendre.leggauss(400)
    lt = 0.5 * math.log(tmin) * (1 - x)  # log tau in [log tmin, 0]
    ref = sum(wi * 0.5 * -math.log(tmin) * math.exp(l) * _pdf_convolution_closed_form(math.exp(l))
              for l, wi in zip(lt, wq)) / (8 * math.pi)
    y = W.philox_uniforms(65, 0, 0, 1_000_000, P.dims[0])
    w = P.map(0, y, None, variant=variant)["w"]
    mean, err = w.mean(), w.std() / math.sqrt(w.size)
    return bool(abs(mean - ref) < 4 * err and err / mean < 3e-3), (mean / ref - 1, err / mean)


def test_t_propagator_weight_is_constant():
    ok, worst = check_t_propagator_weight()
    assert ok, worst


def test_t_propagator_weight_is_constant_massive():
    ok, worst = check_t_propagator_massive()
    assert ok, worst


def test_t_propagator_integral_default_map():
    ok, info = check_t_propagator_integral()
    assert ok, info


def test_breit_wigner_factor_hadronic_per_event():
    ok, worst = check_bw_hadronic()
    assert ok, worst


def test_breit_wigner_factor_decay_chain_per_event():
    ok, worst = check_bw_decay_chain()
    assert ok, worst


def test_toy_pdf_through_full_chain_matches_quadrature():
    ok, info = check_pdf_full_chain()
    assert ok, info


# -- channel weights ---------------------------------------------------------

# Internal lines of the eight pp -> 4 jets diagrams, written down from the
# topologies (legs of a t-channel spine are accumulated from the incoming
# parton a: line j carries q = p_a - sum of the first j legs; s-channel lines
# carry the summed momenta of their cluster; a pure s-channel diagram's root
# line carries s-hat = (p1 + p2 + p3 + p4)^2).
C2_LINES = {
    0: {("t", (1,)), ("t", (1, 2)), ("t", (1, 2, 3))},            # spine 1 2 3 4
    1: {("t", (4,)), ("t", (3, 4)), ("t", (2, 3, 4))},            # spine 4 3 2 1
    2: {("t", (1,)), ("t", (1, 2)), ("t", (1, 2, 4))},            # spine 1 2 4 3
    3: {("t", (1,)), ("t", (1, 2, 3)), ("s", (2, 3))},            # spine 1 (23) 4
    4: {("t", (1, 2)), ("s", (1, 2)), ("s", (3, 4))},             # spine (12) (34)
    5: {("t", (1,)), ("s", (2, 3, 4)), ("s", (2, 3))},            # spine 1 (234), (234) -> (23) 4
    6: {("s", (1, 2, 3, 4)), ("s", (1, 2)), ("s", (3, 4))},       # s-hat -> (12) (34)
    7: {("s", (1, 2, 3, 4)), ("s", (1, 2, 3)), ("s", (1, 2))},    # s-hat -> (123) 4, (123) -> (12) 3
}


def _lines_of(P, c):
    out = set()
    for t, mask, m, w in P.channels[c].propagators():
        assert m == 0.0 and w == 0.0
        out.add(("t" if t else "s", tuple(k + 1 for k in range(P.n) if mask >> k & 1)))
    return out


def check_c2_line_sets(P):
    return all(_lines_of(P, c) == C2_LINES[c] for c in range(8))


def _hand_alpha(p, mu):
    """alpha_c from the hand-listed lines: P_c = prod 1/(|q^2| + mu^2)^2."""
    pa = p[:, 0]
    Ps = []
    for c in range(8):
        prod = np.ones(p.shape[2])
        for kind, parts in sorted(C2_LINES[c]):
            q = sum(p[:, k + 1] for k in parts)
            if kind == "t":
                q = pa - q
            q2 = q[0] ** 2 - q[1] ** 2 - q[2] ** 2 - q[3] ** 2
            prod = prod / (np.abs(q2) + mu * mu) ** 2
        Ps.append(prod)
    Ps = np.array(Ps)
    return Ps / Ps.sum(axis=0)


def _random_momenta(n, seed):
    """Arbitrary four-vectors (no conservation, no mass shells): alpha_c is a
    function of the momenta alone."""
    rng = np.random.default_rng(seed)
    p = rng.normal(0.0, 300.0, size=(4, 6, n))
    p[0] = np.abs(p[0]) + 400.0
    return p


def check_c2_alpha(variant="ref", P=None):
    P = P or oracle.Process(W.c2_pp4j())
    n = 4000
    p = _random_momenta(n, 71)
    x1x2 = np.full((2, n), 0.3)
    expect = _hand_alpha(p, 10.0)
    worst = 0.0
    for c in range(8):
        a = P.weight(c, p, x1x2, np.ones(n), variant=variant)["alpha"]
        worst = max(worst, float(np.max(np.abs(a - expect[c]) / np.maximum(expect[c], 1e-300))))
    return worst < 1e-12, worst


def test_c2_channel_line_sets_hand_listed():
    assert check_c2_line_sets(oracle.Process(W.c2_pp4j()))


def test_c2_alpha_from_hand_listed_lines():
    ok, worst = check_c2_alpha()
    assert ok, worst


# -- planted mistakes ----------------------------------------------------------

@pytest.mark.parametrize("k,check", [
    (1, check_pdf_full_chain),          # (1 - x) exponent off by one
    (2, check_t_propagator_weight),     # mu instead of mu^2
    (2, check_t_propagator_integral),
    (2, check_t_propagator_massive),
    (3, check_t_propagator_massive),    # q = p_a + sum p
    (3, check_c2_alpha),
    (4, check_bw_hadronic),             # Gamma^2 instead of M^2 Gamma^2
    (4, check_bw_decay_chain),
])
def test_planted_mistake_fails_a_pin(tmp_path, k, check):
    variant = oracle.build_mutant(k, str(tmp_path))
    ok, info = check(variant)
    assert not ok, f"mistake {k} passed {check.__name__}: {info}"


@pytest.mark.parametrize("mistake", ["drop_root", "t_from_b", "drop_s"])
def test_planted_line_set_mistake_fails(monkeypatch, mistake):
    """A wrong line selection in the channel compiler (the root line of a
    pure s-channel diagram dropped, t lines accumulated from the wrong end,
    s-channel lines dropped) fails the hand-listed sets and the alpha pin."""
    orig = oracle.ChannelTree.propagators

    def bad(self):
        out = orig(self)
        n = getattr(self, "n_final", None) or len([k for k in self.kind if k == oracle.LEAF])
        full = (1 << n) - 1
        if mistake == "drop_root":
            return [q for q in out if not (q[0] == 0 and q[1] == full)]
        if mistake == "t_from_b":
            return [(t, (full & ~s) if t else s, m, w) for t, s, m, w in out]
        return [q for q in out if q[0] == 1]

    monkeypatch.setattr(oracle.ChannelTree, "propagators", bad)
    P = oracle.Process(W.c2_pp4j())
    assert not check_c2_line_sets(P)
    ok, _ = check_c2_alpha(P=P)
    assert not ok
