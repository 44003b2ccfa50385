"""Mixed precision (MSX_MIXED) against the FP64 oracle on the same seeded
inputs: the per-quantity error statement of the mode.

The FP32 steps (power laws with exponents 1/(1 - nu) <= 5, exp/log, sin/cos
of azimuths) carry relative errors of a few FP32 ulp (u = 6e-8), amplified
at most ~5x by the power laws.  Momenta inherit them through the boosts
(normalised by the event's largest energy: measured p99 <= 3e-6).

Each event therefore sits at a point displaced by ~1e-7 relative from its
FP64 position, and every factor evaluated there is exact for that point: the
mixed weight equals the FP64 integrand of the mixed momenta (measured 5e-7,
the FP32 toy-PDF power), and the integral does not move (measured shift
<= 2e-5 Monte Carlo standard errors).  Compared with the FP64 event of the
same uniforms, the displacement is amplified where a factor is steep:
near-threshold t ranges (Jacobian differences up to 0.2 in rare events),
Breit-Wigner factors of invariants recomputed from TeV momenta (C3 weight
median 8e-5), and t-channel invariants of nearly collinear legs in other
channels' local weights (C2 weight p99 7e-3).  The bounds below are about
2-3 times the measured values of 1e5-event samples."""
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
    c64 = Context(desc)
    assert ctx.precision == MIXED
    orc = oracle.Process(desc)
    d = ctx.dims[chan]
    y_h = W.philox_uniforms(seed, 5, 0, N, d)
    out = ctx.map(chan, torch.from_numpy(y_h).cuda(), weight=True)
    # FP64 integrand of the mixed momenta (the weight entry of an FP64 context)
    w64 = c64.weight(chan, out["p"], out["x1x2"], out["jac"])
    torch.cuda.synchronize()
    ref = orc.map(chan, y_h, orc.uniform_grid(chan))
    err = precision_error(out["p"], out["w"], torch.from_numpy(ref["p"]).cuda(), torch.from_numpy(ref["w"]).cuda(),
                          ctx.n_momenta[chan], jac=out["jac"], jac_ref=torch.from_numpy(ref["jac"]).cuda())
    kept = out["w"] != 0
    self_rel = float(((out["w"] - w64).abs() / w64.abs())[kept].max()) if bool(kept.any()) else 0.0
    ctx.close()
    c64.close()
    err["self_consistency_max"] = self_rel
    print(cfg, chan, {k: (float(f"{v:.3g}") if isinstance(v, float) else v) for k, v in err.items()})
    return err


@pytest.mark.parametrize("cfg,chan", [("c1", 0)] + [("c2", c) for c in range(8)] + [("c3", 0)])
def test_mixed_precision_error_statement(torch, cfg, chan):
    e = _errors(torch, cfg, chan, seed=31)
    assert e["momenta_median"] < 1e-6 and e["momenta_p99"] < 1e-5 and e["momenta_max"] < 1e-3
    assert e["jac_median"] < 5e-6 and e["jac_p99"] < 5e-4 and e["jac_max"] < 0.5
    # only the toy-PDF power x^a is FP32 in the integrand: |a log tau| u < 2e-6
    assert e["self_consistency_max"] < 1e-5
    assert abs(e["integral_shift_sigma"]) < 0.1
    assert e["weight_median"] < 2e-4 and e["weight_p99"] < 3e-2
    assert e["cut_flips"] <= 1e-4 * N


def test_mixed_c1_two_body_volume_is_still_exact_enough(torch):
    """f = 1: every weight is 1/(8 pi); the FP32 angles do not enter the
    weight and the Jacobian product stays FP64."""
    from paper_2602_06895_amd import MIXED, Context

    ctx = Context(W.c1_ee_mumu("unit"), precision=MIXED)
    y = torch.from_numpy(W.philox_uniforms(2, 1, 0, 4096, 2)).cuda()
    w = ctx.map(0, y, weight=True)["w"]
    torch.cuda.synchronize()
    assert np.allclose(w.cpu().numpy(), 1.0 / (8.0 * np.pi), rtol=1e-14, atol=0)
    ctx.close()
