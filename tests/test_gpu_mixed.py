"""Mixed precision (MSX_MIXED) against the FP64 oracle on the same seeded
inputs: the per-quantity error statement of the mode.

Bounds, from the arithmetic: the FP32 steps (power laws with exponents
1/(1 - nu) <= 5, exp/log, sin/cos of angles) carry relative errors of a few
FP32 ulp (u = 6e-8), amplified at most ~5x by the power laws; momenta
inherit them through the boosts (normalised by the event's largest energy),
weights through a product of ~10 Jacobian factors.  Near-threshold
differences are FP64, so no amplification beyond that is expected except
in the far tails of the t maps, which the max bounds absorb.  Where FP32
decides a cut (pT, the energy sign), a few events may flip; the integral
shift must stay below 0.1 Monte Carlo standard errors."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

CONFIGS = {"c1": W.c1_ee_mumu, "c2": W.c2_pp4j, "c3": W.c3_ttbar6}
N = 100_000


@pytest.fixture(scope="module")
def torch():
    import torch as t

    if not t.cuda.is_available():
        pytest.skip("needs a GPU")
    return t


def _errors(torch, cfg, chan, seed):
    from paper_2602_06895_amd import MIXED, Context
    from paper_2602_06895_amd.report import precision_error

    desc = CONFIGS[cfg]()
    ctx = Context(desc, precision=MIXED)
    assert ctx.precision == MIXED
    orc = oracle.Process(desc)
    d = ctx.dims[chan]
    y_h = W.philox_uniforms(seed, 5, 0, N, d)
    out = ctx.map(chan, torch.from_numpy(y_h).cuda(), weight=True)
    torch.cuda.synchronize()
    ref = orc.map(chan, y_h, orc.uniform_grid(chan))
    err = precision_error(out["p"], out["w"], torch.from_numpy(ref["p"]).cuda(), torch.from_numpy(ref["w"]).cuda(),
                          ctx.n_momenta[chan])
    ctx.close()
    print(cfg, chan, {k: (float(f"{v:.3g}") if isinstance(v, float) else v) for k, v in err.items()})
    return err


@pytest.mark.parametrize("cfg,chan", [("c1", 0)] + [("c2", c) for c in range(8)] + [("c3", 0)])
def test_mixed_precision_error_statement(torch, cfg, chan):
    e = _errors(torch, cfg, chan, seed=31)
    assert e["momenta_median"] < 2e-6 and e["momenta_p99"] < 2e-5 and e["momenta_max"] < 1e-3
    assert e["weight_median"] < 2e-5 and e["weight_p99"] < 1e-3
    assert e["cut_flips"] <= 1e-4 * N
    assert abs(e["integral_shift_sigma"]) < 0.1


def test_mixed_c1_two_body_volume_is_still_exact_enough(torch):
    """f = 1: every weight is 1/(8 pi) up to the FP32 angle (which does not
    enter the weight) -- the mixed mode must keep the FP64 Jacobian."""
    from paper_2602_06895_amd import MIXED, Context

    ctx = Context(W.c1_ee_mumu("unit"), precision=MIXED)
    y = torch.from_numpy(W.philox_uniforms(2, 1, 0, 4096, 2)).cuda()
    w = ctx.map(0, y, weight=True)["w"]
    torch.cuda.synchronize()
    assert np.allclose(w.cpu().numpy(), 1.0 / (8.0 * np.pi), rtol=1e-14, atol=0)
    ctx.close()
