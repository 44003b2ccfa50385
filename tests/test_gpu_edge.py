"""Edge cases of the HIP path against the oracle or against another entry
point of the same library: ragged and tiny flow batches, empty calls, the
largest register class (8 final-state particles, 14 momentum slots) at the
largest VEGAS grid, the mixed-precision fused sample, and device-count
launches with nothing to do."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle import flow as F
from parity import compare

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t

    if not t.cuda.is_available():
        pytest.skip("needs a GPU")
    return t


@pytest.mark.parametrize("n", [1, 63, 65, 1000])
def test_flow_ragged_batches_match_oracle(torch, n):
    from paper_2602_06895_amd import FLOW_FP32, Flow

    params = W.flow_params(41, 16, 8, 16, 128, last_scale=0.05)
    f = Flow(16, 8, 16, 128, mlp=FLOW_FP32)
    f.set_params(params)
    u = W.philox_uniforms_f32(7, 3, 11, n, 16)
    y, ld = f.forward(torch.from_numpy(u).cuda())
    ub, lq = f.inverse(y)
    torch.cuda.synchronize()
    orc = F.Flow(16, 8, 16, 128, params=torch.as_tensor(params.astype(np.float64)))
    yr, ldr = orc.forward(torch.from_numpy(u.T.astype(np.float64)))
    assert np.abs(y.cpu().numpy().T - yr.numpy()).max() < 2e-5
    assert np.abs(ld.cpu().numpy() - ldr.numpy()).max() < 2e-4
    assert np.abs(ub.cpu().numpy() - u).max() < 2e-5
    # a gradient of a batch of one event is finite and matches the oracle
    if n == 1:
        wfj = torch.ones(1, dtype=torch.float64, device="cuda")
        g, loss = f.gradient(y, wfj, -ld)
        torch.cuda.synchronize()
        _, gr = orc.loss_and_grad(torch.as_tensor(y.cpu().numpy().T.astype(np.float64)), torch.ones(1, dtype=torch.float64),
                                  torch.as_tensor(-ld.cpu().numpy().astype(np.float64)))
        gg = g.cpu().numpy().astype(np.float64)
        assert np.isfinite(gg).all()
        assert np.linalg.norm(gg - gr.numpy()) <= 1e-3 * np.linalg.norm(gr.numpy())
    f.close()


def test_flow_empty_calls_are_no_ops(torch):
    from paper_2602_06895_amd import Context, Flow

    f = Flow(16, 2, 4, 8)
    u = torch.empty(16, 0, dtype=torch.float32, device="cuda")
    y, ld = f.forward(u)
    ub, lq = f.inverse(u)
    ctx = Context(W.c3_ttbar6())
    out = f.sample(ctx, 0, 0, seed=1)
    torch.cuda.synchronize()
    assert y.shape == (16, 0) and out["w"].shape == (0,)
    ctx.close()
    f.close()


def test_eight_particle_channel_at_128_bins(torch):
    """2 -> 8 massless t-chain (14 momentum slots, the largest register class)
    with a 128-bin random grid: per-event parity with the oracle."""
    from paper_2602_06895_amd import Context

    desc = W.volume_process(8)
    desc["vegas_bins"] = 128
    ctx = Context(desc)
    orc = oracle.Process(desc)
    d = ctx.dims[0]
    rng = np.random.default_rng(5)
    grid = np.empty((d, 129))
    for k in range(d):
        grid[k] = np.concatenate([[0.0], np.sort(rng.random(127)), [1.0]])
    ctx.set_grid(0, grid)
    n = 20000
    y_h = W.philox_uniforms(8, 2, 0, n, d)
    out = ctx.map(0, torch.from_numpy(y_h).cuda(), weight=True)
    torch.cuda.synchronize()
    ref = orc.map(0, y_h, grid)
    fe = orc.forward_error(0, y_h, grid, ref=ref)
    got = {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
    compare(got, ref, fe, hadronic=False, label="2->8 at 128 bins")
    ctx.close()


def test_mixed_fused_sample_equals_mixed_map(torch):
    """The mixed-precision instantiation of the fused kernel gives exactly the
    events of the mixed-precision single-channel map of the same uniforms."""
    from paper_2602_06895_amd import MIXED, Context

    ctx = Context(W.c2_pp4j(), precision=MIXED)
    counts = np.array([1000, 0, 313, 5, 64, 700, 1, 256])
    out = ctx.sample(counts, seed=21, stream_id=2, counter_offset=99)
    torch.cuda.synchronize()
    start = np.concatenate([[0], np.cumsum(counts)])
    for c in range(8):
        if counts[c] == 0:
            continue
        lo, hi = int(start[c]), int(start[c + 1])
        y = ctx.uniform(21, 2, 99 + lo, hi - lo, ctx.dims[c])
        ref = ctx.map(c, y, weight=True)
        torch.cuda.synchronize()
        assert torch.equal(out["w"][lo:hi], ref["w"]), c
        assert torch.equal(out["p"][:, :, lo:hi], ref["p"]), c
    ctx.close()


def test_device_counts_all_zero(torch):
    from paper_2602_06895_amd import Context

    ctx = Context(W.c2_pp4j())
    buf = ctx.sample_buffers(512)
    buf["w"].fill_(-3.0)
    counts = torch.zeros(8, dtype=torch.int64, device="cuda")
    off = torch.zeros(1, dtype=torch.int64, device="cuda")
    status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    ctx.reset_stats()
    g = ctx.sample_graph(counts, 1, 1, off, buf, status)
    g.launch()
    torch.cuda.synchronize()
    assert int(status.cpu()[0]) == 0 and bool((buf["w"] == -3.0).all())
    assert np.all(ctx.stats() == 0)
    g.close()
    ctx.close()


def test_fused_forward_with_padded_layer_blocks(torch):
    """d = 10 (five transformed coordinates): layer blocks of 65,397 parameters,
    padded in the BF16 operand copy so that the fused layer kernel can run;
    forward against the BF16-rounded oracle and the unfused inverse round
    trip."""
    from paper_2602_06895_amd import FLOW_BF16, Flow

    d = 10
    params = W.flow_params(43, d, 8, 16, 128, last_scale=0.05)
    f = Flow(d, 8, 16, 128, mlp=FLOW_BF16)
    f.set_params(params)
    u = W.philox_uniforms_f32(9, 4, 0, 3000, d)
    y, ld = f.forward(torch.from_numpy(u).cuda())
    ub, lq = f.inverse(y)
    torch.cuda.synchronize()
    orc = F.Flow(d, 8, 16, 128, params=torch.as_tensor(params.astype(np.float64)), bf16_mlp=True)
    yr, ldr = orc.forward(torch.from_numpy(u.T.astype(np.float64)))
    # BF16 rounding decisions on FP32 accumulators vs FP64 ones (one BF16 ulp)
    assert np.abs(y.cpu().numpy().T - yr.numpy()).max() < 2e-3
    assert np.abs(ld.cpu().numpy() - ldr.numpy()).max() < 2e-2
    assert np.abs(ub.cpu().numpy() - u).max() < 2e-5
    assert np.abs(lq.cpu().numpy() + ld.cpu().numpy()).max() < 2e-4
    f.close()
