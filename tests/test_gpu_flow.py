"""The coupling-flow kernels (through the C ABI of include/msx_flow.h) against
the FP64 flow oracle on the same seeded inputs.

FP32 mode: every step in FP32, compared with the FP64 oracle on the same
float32 parameters and inputs.  BF16 mode: compared with the oracle run with
the same BF16 rounding of MLP inputs, weights and hidden activations.
Tolerances are stated per test with the reason."""
import numpy as np
import pytest
import torch as _t

import workloads as W
from oracle import flow as F

pytestmark = pytest.mark.gpu

D, L, K, H = 16, 8, 16, 128  # the learned-sampler shape (16 dims, 8 layers, 16 bins, 3 x 128)


@pytest.fixture(scope="module")
def torch():
    if not _t.cuda.is_available():
        pytest.skip("needs a GPU")
    return _t


def _flow(mlp, params, d=D, layers=L, bins=K, hidden=H):
    from paper_2602_06895_amd import Flow

    f = Flow(d, layers, bins, hidden, mlp=mlp)
    f.set_params(params)
    return f


def _oracle(params, bf16=False, d=D, layers=L, bins=K, hidden=H):
    return F.Flow(d, layers, bins, hidden, params=_t.as_tensor(params.astype(np.float64)), bf16_mlp=bf16)


def _u(n, seed=3, d=D):
    return W.philox_uniforms_f32(seed, 9, 0, n, d)


@pytest.mark.parametrize("mlp", [1, 0])
def test_forward_and_inverse_match_oracle(torch, mlp):
    params = W.flow_params(21, D, L, K, H, last_scale=0.05)
    f = _flow(mlp, params)
    u = _u(5000)
    y, ld = f.forward(torch.from_numpy(u).cuda())
    ub, lq = f.inverse(y)
    torch.cuda.synchronize()
    orc = _oracle(params, bf16=(mlp == 0))
    yr, ldr = orc.forward(_t.from_numpy(u.T.astype(np.float64)))
    yg, ldg = y.cpu().numpy().T.astype(np.float64), ld.cpu().numpy().astype(np.float64)
    dy = np.abs(yg - yr.numpy()).max()
    dld = np.abs(ldg - ldr.numpy()).max()
    print(f"mlp={mlp} max|dy|={dy:.3g} max|dlogdet|={dld:.3g} spread logdet={ldr.numpy().std():.3g}")
    if mlp == 1:
        # FP32 through 8 layers of 8 splines and a 4-layer MLP each: a few
        # hundred roundings of 6e-8, amplified by spline slopes of O(1)
        assert dy < 2e-5 and dld < 2e-4
    else:
        # BF16 rounding decisions taken on FP32 accumulators here and FP64 ones
        # in the oracle differ for a few activations (one BF16 ulp, 2^-8)
        assert dy < 2e-3 and dld < 2e-2
    # inverse of the forward on the GPU itself
    dub = (ub.cpu().numpy().T - u.T).astype(np.float64)
    assert np.abs(dub).max() < 2e-5
    assert np.abs(lq.cpu().numpy() + ld.cpu().numpy()).max() < 2e-4


def test_zero_parameters_are_the_identity(torch):
    params = W.flow_params(22, D, L, K, H, last_scale=0.0)
    f = _flow(0, params)
    u = _u(4096, seed=4)
    y, ld = f.forward(torch.from_numpy(u).cuda())
    torch.cuda.synchronize()
    # FP32 spline with all bins equal: only rounding of the knots (K 6e-8)
    assert np.abs(y.cpu().numpy() - u).max() < 4e-7
    assert np.abs(ld.cpu().numpy()).max() < 2e-5


@pytest.mark.parametrize("mlp", [1, 0])
def test_gradient_matches_oracle(torch, mlp):
    params = W.flow_params(23, D, L, K, H, last_scale=0.05)
    f = _flow(mlp, params)
    n = 2048
    u = _u(n, seed=5)
    y, ld = f.forward(torch.from_numpy(u).cuda())
    rng = np.random.default_rng(6)
    wfj = torch.from_numpy(rng.uniform(0.5, 2.0, n)).cuda()
    lqo = -ld
    g, loss = f.gradient(y, wfj, lqo)
    torch.cuda.synchronize()
    orc = _oracle(params, bf16=(mlp == 0))
    yy = _t.from_numpy(y.cpu().numpy().T.astype(np.float64))
    fj = _t.from_numpy(wfj.cpu().numpy())
    lr, gr = orc.loss_and_grad(yy, fj * fj, _t.from_numpy(lqo.cpu().numpy().astype(np.float64)))
    gg = g.cpu().numpy().astype(np.float64)
    grn = gr.numpy()
    rel = np.linalg.norm(gg - grn) / np.linalg.norm(grn)
    cos = float(gg @ grn / (np.linalg.norm(gg) * np.linalg.norm(grn)))
    print(f"mlp={mlp} loss gpu={float(loss.cpu()[0]):.8g} oracle={lr:.8g} grad rel={rel:.3g} cos={cos:.8f}")
    assert abs(float(loss.cpu()[0]) - lr) <= 1e-4 * abs(lr)
    if mlp == 1:
        assert rel < 1e-3
    else:
        assert rel < 5e-2 and cos > 0.998


def test_adam_first_step(torch):
    params = W.flow_params(24, D, 2, K, 32, last_scale=0.05)
    f = _flow(1, params, layers=2, hidden=32)
    n = 1024
    u = _u(n, seed=7)
    y, ld = f.forward(torch.from_numpy(u).cuda())
    wfj = torch.from_numpy(np.random.default_rng(8).uniform(0.5, 2.0, n)).cuda()
    g, loss = f.gradient(y, wfj, -ld)
    f.train_step(y, wfj, -ld, lr=1e-3)
    torch.cuda.synchronize()
    p1 = f.get_params().astype(np.float64)
    # the step descends log L: gradient g / L
    gg = g.cpu().numpy().astype(np.float64) / float(loss.cpu()[0])
    exp = params.astype(np.float64) - 1e-3 * gg / (np.abs(gg) + 1e-8)
    # the step is lr sign(g) wherever |g| >> eps; FP32 parameters (ulp 6e-8)
    assert np.abs(p1 - exp).max() < 1e-6


def test_training_reduces_the_loss_on_a_peaked_target(torch):
    """A few hundred Adam steps on f(y) = prod exp(-(y - 0.3)^2 / 0.02) in 4
    dims: the loss (mean w^2 at fixed integral) must fall well below its
    identity-flow value."""
    d = 4
    f = _flow(0, W.flow_params(25, d, 4, 8, 32), d=d, layers=4, bins=8, hidden=32)
    n = 4096
    losses = []
    for step in range(200):
        u = torch.from_numpy(W.philox_uniforms_f32(10, 11, step * n, n, d)).cuda()
        y, ld = f.forward(u)
        yy = y.double()
        fj = torch.exp(-((yy - 0.3) ** 2).sum(dim=0) / 0.02)
        loss = f.train_step(y, fj, -ld, lr=3e-3)
        losses.append(float(loss.cpu()[0]))
    first, last = np.mean(losses[:10]), np.mean(losses[-10:])
    print(f"loss {first:.4g} -> {last:.4g}")
    assert last < 0.5 * first


def test_flow_sample_matches_map_of_its_points(torch):
    from paper_2602_06895_amd import Context

    ctx = Context(W.c3_ttbar6())
    params = W.flow_params(26, D, L, K, H, last_scale=0.05)
    f = _flow(0, params)
    n = 3000
    out = f.sample(ctx, 0, n, seed=12, stream_id=3, counter_offset=77)
    torch.cuda.synchronize()
    y = out["y"]
    yd = y.double().clamp(2.0 ** -26, 1.0 - 2.0 ** -24)
    ref = ctx.map(0, yd, weight=True)
    torch.cuda.synchronize()
    assert torch.equal(out["p"], ref["p"]) and torch.equal(out["wfj"], ref["w"])
    # y is the flow of the 24-bit uniforms of (seed, stream, counter)
    u = W.philox_uniforms_f32(12, 3, 77, n, D)
    y2, ld2 = f.forward(torch.from_numpy(u).cuda())
    torch.cuda.synchronize()
    assert torch.equal(y2, y)
    assert torch.allclose(out["logq"], -ld2)
    w = ref["w"] * torch.exp(ld2.double())
    assert torch.allclose(out["w"], w, rtol=1e-12, atol=0)
    ctx.close()


def test_bad_arguments(torch):
    from paper_2602_06895_amd import Flow, MsxError, load_library
    import ctypes as C

    with pytest.raises(MsxError):
        Flow(15)
    with pytest.raises(MsxError):
        Flow(16, bins=33)
    f = Flow(4, 2, 4, 8)
    with pytest.raises(ValueError):
        f.set_params(np.zeros(3, dtype=np.float32))
    Lb = load_library()
    assert Lb.msx_flow_forward(f.h, -1, None, None, None, None) == 1
    assert Lb.msx_flow_train_step(f.h, 10, None, None, None, C.c_float(1e-3), None, None) == 1
    y = torch.rand(4, 10, device="cuda", dtype=torch.float32)
    lq = torch.zeros(10, device="cuda", dtype=torch.float32)
    wfj = torch.ones(10, device="cuda", dtype=torch.float64)
    with pytest.raises(MsxError):
        f.train_step(y, wfj, lq, lr=-1.0)
    from paper_2602_06895_amd import Context
    ctx = Context(W.c3_ttbar6())
    with pytest.raises(MsxError):
        f.sample(ctx, 0, 10, seed=1)
    ctx.close()
    f.close()


@pytest.mark.parametrize("mlp", [1, 0])
def test_gradient_per_parameter_block(torch, mlp):
    """The gradient block by block (W1 b1 W2 b2 W3 b3 W4 b4 of each of the 8
    layers), so that a wrong block cannot hide in the norm of the whole.
    FP32 mode: every block within 1e-3 relative of the FP64 oracle on the
    same float32 parameters.  BF16 mode: the tolerance of a block is derived
    from BF16 rounding itself -- the oracle's gradient with BF16 rounding of
    MLP inputs, weights and hidden activations differs from its FP64 gradient
    by d_bf16 (per block); the GPU must agree with the BF16 oracle within
    2 d_bf16 + 1e-3 (rounding decisions taken on FP32 accumulators here and
    FP64 ones in the oracle differ, each worth at most one such rounding),
    and every block's direction within cos >= 0.99."""
    params = W.flow_params(23, D, L, K, H, last_scale=0.05)
    f = _flow(mlp, params)
    n = 2048
    u = _u(n, seed=5)
    y, ld = f.forward(torch.from_numpy(u).cuda())
    rng = np.random.default_rng(6)
    wfj = torch.from_numpy(rng.uniform(0.5, 2.0, n)).cuda()
    lqo = -ld
    g, _ = f.gradient(y, wfj, lqo)
    torch.cuda.synchronize()
    yy = _t.from_numpy(y.cpu().numpy().T.astype(np.float64))
    fj2 = _t.from_numpy(wfj.cpu().numpy()) ** 2
    lq = _t.from_numpy(lqo.cpu().numpy().astype(np.float64))
    _, g64 = _oracle(params, bf16=False).loss_and_grad(yy, fj2, lq)
    g64 = g64.numpy()
    if mlp == 0:
        _, gbf = _oracle(params, bf16=True).loss_and_grad(yy, fj2, lq)
        gref = gbf.numpy()
    else:
        gref = g64
    gg = g.cpu().numpy().astype(np.float64)
    shapes = [(H, D // 2), (H,), (H, H), (H,), (H, H), (H,), (D // 2 * (3 * K + 1), H), (D // 2 * (3 * K + 1),)]
    sizes = [int(np.prod(s)) for s in shapes]
    off, worst = 0, 0.0
    total = np.linalg.norm(gref)
    for layer in range(L):
        for b, sz in enumerate(sizes):
            a, r, r64 = gg[off:off + sz], gref[off:off + sz], g64[off:off + sz]
            off += sz
            nr = np.linalg.norm(r)
            if nr < 1e-9 * total:
                assert np.linalg.norm(a) < 1e-6 * total, (layer, b)
                continue
            rel = np.linalg.norm(a - r) / nr
            cos = float(a @ r / (np.linalg.norm(a) * nr))
            if mlp == 1:
                tol = 1e-3
            else:
                tol = 2.0 * np.linalg.norm(r - r64) / nr + 1e-3
            worst = max(worst, rel / tol)
            assert rel <= tol and cos >= 0.99, f"layer {layer} block {b}: rel {rel:.3g} (tol {tol:.3g}) cos {cos:.5f}"
    assert off == gg.size
    print(f"mlp={mlp}: worst block error / tolerance {worst:.3f}")
