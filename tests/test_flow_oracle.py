"""Pins of the FP64 flow oracle (oracle/flow.py) against what the paper and
the mathematics fix: the single-bin RQF of the FastRambo section (forward,
derivative and the paper's closed-form inverse), the RamboOnDiet k = 1 case,
the identity at zero parameters, inverse round trips, finite-difference
log-determinants and gradients, and the first Adam step."""
import math

import numpy as np
import pytest
import torch

from oracle import flow as F
import workloads as W

DT = torch.float64


def _k1(c):
    """Single bin, slope c at 0 and 0 at 1."""
    xk = torch.tensor([[0.0, 1.0]], dtype=DT)
    yk = torch.tensor([[0.0, 1.0]], dtype=DT)
    d = torch.tensor([[c, 0.0]], dtype=DT)
    return xk, yk, d


@pytest.mark.parametrize("c", [0.3, 1.0, 2.0, 3.7])
def test_single_bin_is_the_papers_rqf(c):
    y = torch.linspace(0.0, 1.0, 101, dtype=DT)
    xk, yk, d = _k1(c)
    n = y.numel()
    r, g = F.rqs_forward(y, xk.expand(n, 2), yk.expand(n, 2), d.expand(n, 2))
    om = y * (1 - y)
    G = (y * y + c * om) / (1 + (c - 2) * om)          # G_RQF, section 2.2.9
    gg = (2 * om + c * (1 - y) ** 2) / (1 + (c - 2) * om) ** 2  # g_RQF
    assert torch.allclose(r, G, rtol=0, atol=1e-15)
    assert torch.allclose(g, gg, rtol=1e-14, atol=1e-15)
    # the paper's inverse: 2r / (b + sqrt(b^2 + 4 r (1 - b))), b = c - (c - 2) r
    rr = torch.linspace(0.0, 1.0, 101, dtype=DT)
    b = c - (c - 2) * rr
    yinv = 2 * rr / (b + torch.sqrt(b * b + 4 * rr * (1 - b)))
    x, dxdy = F.rqs_inverse(rr, xk.expand(n, 2), yk.expand(n, 2), d.expand(n, 2))
    assert torch.allclose(x, yinv, rtol=0, atol=1e-15)
    inner = (rr > 0) & (rr < 1)
    _, gfwd = F.rqs_forward(x, xk.expand(n, 2), yk.expand(n, 2), d.expand(n, 2))
    assert torch.allclose((dxdy * gfwd)[inner], torch.ones_like(rr)[inner], rtol=1e-12)


def test_c2_reproduces_rambo_on_diet_k1():
    y = torch.linspace(0.0, 1.0, 57, dtype=DT)
    xk, yk, d = _k1(2.0)
    n = y.numel()
    r, _ = F.rqs_forward(y, xk.expand(n, 2), yk.expand(n, 2), d.expand(n, 2))
    assert torch.allclose(r, 2 * y - y * y, rtol=0, atol=1e-15)


def test_zero_parameters_give_the_identity():
    K = 16
    theta = torch.zeros(1000, 3 * K + 1, dtype=DT)
    xk, yk, d = F.rqs_bins(theta, K)
    assert torch.allclose(xk[0], torch.arange(K + 1, dtype=DT) / K, atol=1e-15)
    assert torch.allclose(d, torch.ones_like(d), atol=1e-15)
    x = torch.rand(1000, dtype=DT, generator=torch.Generator().manual_seed(1))
    y, g = F.rqs_forward(x, xk, yk, d)
    assert torch.allclose(y, x, atol=1e-15) and torch.allclose(g, torch.ones_like(g), atol=1e-13)


def _random_bins(n, K, seed, scale=2.0):
    g = torch.Generator().manual_seed(seed)
    theta = scale * torch.randn(n, 3 * K + 1, dtype=DT, generator=g)
    return F.rqs_bins(theta, K)


@pytest.mark.parametrize("K", [1, 4, 16])
def test_spline_round_trip_derivative_and_monotonicity(K):
    n = 4000
    xk, yk, d = _random_bins(n, K, 3)
    assert torch.all(xk[:, 1:] > xk[:, :-1]) and torch.all(yk[:, 1:] > yk[:, :-1])
    assert torch.all(xk[:, -1] == 1.0) and torch.all(yk[:, -1] == 1.0)
    x = torch.rand(n, dtype=DT, generator=torch.Generator().manual_seed(4))
    y, g = F.rqs_forward(x, xk, yk, d)
    xb, gi = F.rqs_inverse(y, xk, yk, d)
    # in units of y (the inverse is as ill-conditioned as the slope is small)
    assert float(((xb - x).abs() * g).max()) < 1e-13
    assert torch.allclose(g * gi, torch.ones_like(g), rtol=1e-8)
    h = 1e-6
    xp, xm = torch.clamp(x + h, max=1.0), torch.clamp(x - h, min=0.0)
    fd = (F.rqs_forward(xp, xk, yk, d)[0] - F.rqs_forward(xm, xk, yk, d)[0]) / (xp - xm)
    # away from knots (the derivative is continuous there, the difference is not smooth)
    near = torch.zeros(n, dtype=torch.bool)
    for k in range(K + 1):
        near |= (x - xk[:, k]).abs() < 2 * h
    ok = ~near
    assert torch.allclose(fd[ok], g[ok], rtol=1e-5)
    # endpoints and knots map to knots
    e0, _ = F.rqs_forward(torch.zeros(n, dtype=DT), xk, yk, d)
    e1, _ = F.rqs_forward(torch.ones(n, dtype=DT), xk, yk, d)
    assert torch.all(e0 == 0.0) and torch.allclose(e1, torch.ones_like(e1), atol=1e-15)
    knot = xk[:, min(1, K)]
    yk1, _ = F.rqs_forward(knot, xk, yk, d)
    assert torch.allclose(yk1, yk[:, min(1, K)], atol=1e-14)


def test_knot_derivatives_are_the_spline_slopes():
    K = 5
    xk, yk, d = _random_bins(200, K, 8)
    for k in range(1, K):
        g = F.rqs_forward(xk[:, k], xk, yk, d)[1]
        assert torch.allclose(g, d[:, k], rtol=1e-10)


def test_masks_partition_and_cover():
    d = 16
    for layer in range(8):
        t, c = F.transformed(d, layer), F.conditioning(d, layer)
        assert sorted(t + c) == list(range(d)) and len(t) == d // 2
    assert F.transformed(d, 2) == list(range(0, 16, 2)) and F.transformed(d, 1) == list(range(8, 16))


def test_parameter_count_matches_the_shape():
    f = F.Flow(16, 8, 16, 128)
    assert f.per_layer == 8 * 128 + 128 + 2 * (128 * 128 + 128) + 392 * 128 + 392
    assert f.n_params == 677952


def test_flow_identity_init_round_trip_and_logdet():
    gen = np.random.default_rng(5)
    p0 = torch.as_tensor(W.flow_params(5, 8, 4, 6, 16), dtype=DT)
    f = F.Flow(8, 4, 6, 16, params=p0)
    u = torch.rand(300, 8, dtype=DT, generator=torch.Generator().manual_seed(6))
    y, ld = f.forward(u)
    assert torch.allclose(y, u, rtol=0, atol=1e-15) and float(ld.abs().max()) < 1e-14
    # random last layers: a genuine flow
    p = p0 + 0.2 * torch.as_tensor(gen.standard_normal(p0.numel()))
    f = F.Flow(8, 4, 6, 16, params=p)
    y, ld = f.forward(u)
    assert not torch.allclose(y, u)
    ub, ldi = f.inverse(y)
    assert torch.allclose(ub, u, atol=1e-10)
    assert torch.allclose(ldi, -ld, atol=1e-9)
    # log|det dy/du| against a central-difference Jacobian matrix
    h = 1e-6
    for i in range(3):
        J = torch.zeros(8, 8, dtype=DT)
        for j in range(8):
            up, um = u[i:i + 1].clone(), u[i:i + 1].clone()
            up[0, j] += h
            um[0, j] -= h
            J[:, j] = (f.forward(up)[0][0] - f.forward(um)[0][0]) / (2 * h)
        sign, logabs = torch.linalg.slogdet(J)
        assert sign > 0
        assert abs(float(logabs) - float(ld[i])) < 1e-6


def test_loss_gradient_against_central_differences():
    gen = np.random.default_rng(9)
    f = F.Flow(4, 4, 3, 5, params=None)
    p = torch.as_tensor(gen.standard_normal(f.n_params) * 0.7)
    f.params = p
    y = torch.as_tensor(gen.uniform(0.02, 0.98, (64, 4)))
    Fv = torch.as_tensor(gen.uniform(0.5, 2.0, 64))
    lqo = torch.as_tensor(gen.uniform(-0.3, 0.3, 64))
    L, g = f.loss_and_grad(y, Fv, lqo)
    assert L == pytest.approx(float(f.loss(y, Fv, lqo)), rel=1e-15)
    idx = gen.choice(f.n_params, 40, replace=False)
    h = 1e-6
    for i in idx:
        pp, pm = p.clone(), p.clone()
        pp[i] += h
        pm[i] -= h
        fd = (float(f.loss(y, Fv, lqo, pp)) - float(f.loss(y, Fv, lqo, pm))) / (2 * h)
        assert abs(fd - float(g[i])) <= 1e-6 * max(1.0, abs(fd)), (i, fd, float(g[i]))


def test_loss_at_the_sampling_point_is_the_mean_square_weight():
    gen = np.random.default_rng(10)
    f = F.Flow(4, 4, 3, 5, params=torch.as_tensor(gen.standard_normal(F.Flow(4, 4, 3, 5).n_params) * 0.5))
    u = torch.as_tensor(gen.uniform(0.01, 0.99, (50, 4)))
    y, ld = f.forward(u)
    fj = torch.as_tensor(gen.uniform(0.1, 3.0, 50))  # f J of each event
    w = fj * torch.exp(ld)                            # weight of the sampled event
    L = f.loss(y, fj * fj, -ld)
    assert float(L) == pytest.approx(float(torch.mean(w * w)), rel=1e-10)


def test_adam_first_step():
    g = torch.tensor([1e-3, -2.0, 0.0, 5e-9], dtype=DT)
    p = torch.tensor([1.0, 2.0, 3.0, 4.0], dtype=DT)
    a = F.Adam(4, lr=1e-3)
    q = a.step(p, g)
    exp = p - 1e-3 * g / (g.abs() + 1e-8)
    assert torch.allclose(q, exp, rtol=0, atol=1e-15)
    # second step with the same gradient: m and v bias corrections still cancel
    q2 = a.step(q, g)
    assert torch.allclose(q2, exp - 1e-3 * g / (g.abs() + 1e-8), atol=1e-15)


def test_bf16_rounding():
    t = torch.tensor([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -9, 1 + 2 ** -7, -3.0, 1e-40], dtype=DT)
    r = F.bf16(t)
    assert r.tolist()[:5] == [1.0, 1.0, 1 + 2 ** -7, 1 + 2 ** -7, -3.0]


def test_bf16_mlp_differs_by_bf16_rounding_only():
    gen = np.random.default_rng(11)
    p = torch.as_tensor(W.flow_params(11, 16, 2, 16, 128, last_scale=0.01), dtype=DT)
    a = F.Flow(16, 2, 16, 128, params=p)
    b = F.Flow(16, 2, 16, 128, params=p, bf16_mlp=True)
    cond = torch.as_tensor(gen.uniform(0, 1, (100, 8)))
    ta, tb = a.mlp(p, 0, cond), b.mlp(p, 0, cond)
    rel = float((ta - tb).abs().max() / ta.abs().max())
    assert 1e-5 < rel < 3 * 2 ** -8
