"""Error of a result against an FP64 result of the same events (the
per-quantity statement of the mixed-precision mode).  Runs on whatever device
the tensors live on; measurement only, not part of the sampling path."""


def _quantiles(x, qs):
    import torch

    x = x.flatten()
    n = x.numel()
    if n == 0:
        return [0.0 for _ in qs]
    xs = torch.sort(x).values
    return [float(xs[min(n - 1, int(q * (n - 1) + 0.5))]) for q in qs]


def precision_error(p, w, p_ref, w_ref, np_, jac=None, jac_ref=None):
    """Compare (p, w) with the FP64 (p_ref, w_ref) of the same events.

    p, p_ref: [4][np][n] momenta; w, w_ref: [n] weights.  Returns a dict:
      momenta_{median,p99,max}: max_{i,mu} |dp_i^mu| / max_i E_i(ref) per event,
        over events that both sides keep (w != 0);
      weight_{median,p99,max}: |dw| / |w_ref| over events kept by both;
      cut_flips: events kept by exactly one side;
      integral_shift_sigma: (sum w - sum w_ref) / n over the Monte Carlo
        standard error of the reference mean;
      jac_{median,p99,max} (when jac, jac_ref are given): |dJ| / |J_ref|.
    """
    import torch

    n = w_ref.numel()
    p = p.reshape(4, np_, n)
    p_ref = p_ref.reshape(4, np_, n)
    both = (w != 0) & (w_ref != 0)
    flips = int(((w != 0) ^ (w_ref != 0)).sum())
    emax = p_ref[0].abs().amax(dim=0)
    dp = (p - p_ref).abs().amax(dim=(0, 1)) / emax
    dp = dp[both]
    dw = ((w - w_ref).abs() / w_ref.abs())[both]
    mp = _quantiles(dp, [0.5, 0.99, 1.0])
    mw = _quantiles(dw, [0.5, 0.99, 1.0])
    mean_ref = w_ref.double().mean()
    sigma = float(w_ref.double().std() / n ** 0.5) if n > 1 else 0.0
    shift = float((w.double().mean() - mean_ref))
    out = {}
    if jac is not None and jac_ref is not None:
        kept = (jac != 0) & (jac_ref != 0)
        mj = _quantiles(((jac - jac_ref).abs() / jac_ref.abs())[kept], [0.5, 0.99, 1.0])
        out = {"jac_median": mj[0], "jac_p99": mj[1], "jac_max": mj[2]}
    return {
        **out,
        "momenta_median": mp[0], "momenta_p99": mp[1], "momenta_max": mp[2],
        "weight_median": mw[0], "weight_p99": mw[1], "weight_max": mw[2],
        "cut_flips": flips, "events": n,
        "integral_shift_sigma": shift / sigma if sigma > 0 else 0.0,
    }
