"""Seeded synthetic workloads for the phase-space hot path.

This module holds *inputs only*: process/channel descriptions (plain data)
and seeded uniform random numbers.  It contains none of the method's
arithmetic, so both the FP64 oracle and the HIP library can consume it.

Uniforms come from numpy's Philox4x64-10 bit generator (Salmon et al.,
SC'11), addressed so that the uniform for (seed, stream, event id e, dim k)
is a pure function of those four values:

    key     = (seed, stream)
    counter = (e, k // 4, 0, 0)             -> four 64-bit words
    u[k]    = ((word[k % 4] >> 11) + 0.5) * 2**-53   in (0, 1)

numpy's generator increments its counter *before* producing a block, so a
generator started at counter (e0 - 1, g, 0, 0) yields blocks for events
e0, e0+1, ... of dimension group g.
"""
from __future__ import annotations

import copy
import json
import math

import numpy as np

__all__ = [
    "c1_ee_mumu", "c2_pp4j", "c3_ttbar6", "c4_multichannel", "volume_process",
    "paper_example_2to3", "philox_uniforms", "philox_raw", "counts_powerlaw",
    "to_json", "CONFIG_NAMES",
]

_TWO_M53 = 2.0 ** -53


# ---------------------------------------------------------------------------
# Process / channel descriptions
#
# A process fixes the beams, the outgoing masses (particles are labelled
# 1..n), the integrand and the list of channels.  A channel is a diagram
# topology:
#   {"t_chain": [leg, ..., leg], "t_order": "AB.."}   legs attached along the
#        t-channel spine from incoming leg a to incoming leg b; t_order has one
#        letter per generation step i < kappa saying whether the leg peeled off
#        next is the one closest to leg A or leg B.
#   {"s": cluster}   pure s-channel: the whole final state decays from s-hat.
# A leg is either a particle label (int) or a cluster
#   {"d": [child, child], "m": mass, "w": width, "nu": nu, "order": k}
# which is an s-channel propagator decaying into two children.
# ---------------------------------------------------------------------------

def c1_ee_mumu(integrand: str = "1+cos2") -> dict:
    """e+e- -> mu+mu- at fixed sqrt(s) = 1000 GeV, one channel, two dims."""
    ig = {"ang": 1} if integrand == "1+cos2" else {}
    return {
        "name": "ee_mumu",
        "sqrt_s": 1000.0,
        "beams": "fixed",
        "masses": [0.0, 0.0],
        "nu": 0.8,
        "regulator": 1e-3,
        "vegas_bins": 64,
        "integrand": ig,
        "channels": [{"s": {"d": [1, 2]}}],
    }


def _c2_channels() -> list:
    """Eight 2->4 diagram topologies (pure t, mixed, pure s)."""
    return [
        {"t_chain": [1, 2, 3, 4], "t_order": "AA"},
        {"t_chain": [4, 3, 2, 1], "t_order": "BB"},
        {"t_chain": [1, 2, 4, 3], "t_order": "AB"},
        {"t_chain": [1, {"d": [2, 3]}, 4], "t_order": "B"},
        {"t_chain": [{"d": [1, 2]}, {"d": [3, 4]}]},
        {"t_chain": [1, {"d": [{"d": [2, 3]}, 4]}]},
        {"s": {"d": [{"d": [1, 2]}, {"d": [3, 4]}]}},
        {"s": {"d": [{"d": [{"d": [1, 2]}, 3]}, 4]}},
    ]


def c2_pp4j() -> dict:
    """pp -> 4 massless jets at 13 TeV with a toy PDF and t-propagator integrand.

    f = f_pdf(x1) f_pdf(x2) * prod_j 1/(|t_j| + mu^2), t_j = (p_a - sum_{k<=j} p_k)^2,
    mu = 10 GeV, pT > 20 GeV on every jet; s-hat >= (4 * 20 GeV)^2.
    """
    return {
        "name": "pp4j",
        "sqrt_s": 13000.0,
        "beams": "hadronic",
        "shat_min": 6400.0,
        "masses": [0.0, 0.0, 0.0, 0.0],
        "nu": 0.8,
        "regulator": 1e-3,
        "vegas_bins": 64,
        "integrand": {
            "pdf": [-1.2, 3.0],
            "pt_min": 20.0,
            "props": [
                {"t": True, "particles": [1], "mu": 10.0},
                {"t": True, "particles": [1, 2], "mu": 10.0},
                {"t": True, "particles": [1, 2, 3], "mu": 10.0},
            ],
        },
        "alpha_mu": 10.0,
        "channels": _c2_channels(),
    }


def c3_ttbar6() -> dict:
    """pp -> t tbar -> b W+ bbar W- -> 6 massless final states at 13 TeV.

    Particles: 1 b, 2 l+, 3 nu, 4 bbar, 5 l-, 6 nubar.  Breit-Wigner mappings for
    t (173, 1.5) and W (80.4, 2.1); integrand = toy PDFs x product of the four
    Breit-Wigner denominators recomputed from the final momenta.
    """
    mt, gt, mw, gw = 173.0, 1.5, 80.4, 2.1
    top = {"d": [1, {"d": [2, 3], "m": mw, "w": gw, "order": 3}], "m": mt, "w": gt, "order": 1}
    atop = {"d": [4, {"d": [5, 6], "m": mw, "w": gw, "order": 4}], "m": mt, "w": gt, "order": 2}
    return {
        "name": "ttbar6",
        "sqrt_s": 13000.0,
        "beams": "hadronic",
        "shat_min": 40000.0,
        "masses": [0.0] * 6,
        "nu": 0.8,
        "regulator": 1e-3,
        "vegas_bins": 64,
        "integrand": {
            "pdf": [-1.2, 3.0],
            "props": [
                {"t": False, "particles": [1, 2, 3], "bw": True, "m": mt, "w": gt},
                {"t": False, "particles": [4, 5, 6], "bw": True, "m": mt, "w": gt},
                {"t": False, "particles": [2, 3], "bw": True, "m": mw, "w": gw},
                {"t": False, "particles": [5, 6], "bw": True, "m": mw, "w": gw},
            ],
        },
        "channels": [{"s": {"d": [top, atop]}}],
    }


def volume_process(n: int, sqrt_s: float = 1000.0, nu: float = 0.3, channels=None,
                   alpha_mu: float | None = None) -> dict:
    """Massless 2->n at fixed sqrt(s) with f = 1 (phase-space volume test)."""
    if channels is None:
        if n == 4:
            channels = _c2_channels()
        else:
            channels = [{"t_chain": list(range(1, n + 1)), "t_order": "A" * (n - 2)}]
    d = {
        "name": f"volume{n}",
        "sqrt_s": sqrt_s,
        "beams": "fixed",
        "masses": [0.0] * n,
        "nu": nu,
        "regulator": 1e-3,
        "vegas_bins": 64,
        "integrand": {},
        "channels": copy.deepcopy(channels),
    }
    if alpha_mu is not None:
        d["alpha_mu"] = alpha_mu
    return d


def paper_example_2to3() -> dict:
    """The hadronic 2->3 example diagram: one massless t-channel propagator and
    one massless s-channel propagator (section 3.2.1, compute-graph figure)."""
    return {
        "name": "example2to3",
        "sqrt_s": 13000.0,
        "beams": "hadronic",
        "shat_min": 0.0,
        "masses": [0.0, 0.0, 0.0],
        "nu": 0.8,
        "regulator": 1e-3,
        "vegas_bins": 64,
        "integrand": {},
        "channels": [{"t_chain": [{"d": [1, 2]}, 3]}],
    }


def c4_multichannel(seed: int = 4, n_channels: int = 24, lo: float = 1e3, hi: float = 1e6):
    """24 channels drawn from the C1 and C2 topologies (topology = c mod 9:
    0 -> C1, 1..8 -> C2 channels 0..7) with power-law event counts.

    Returns (list of (process, channel index) pairs, counts)."""
    counts = counts_powerlaw(n_channels, seed=seed, lo=lo, hi=hi)
    members = []
    for c in range(n_channels):
        t = c % 9
        members.append(("c1", 0) if t == 0 else ("c2", t - 1))
    return members, counts


def c4_context(seed: int = 4, n_channels: int = 24, lo: float = 1e3, hi: float = 1e6):
    """The multichannel batch as one context: consecutive runs of the
    c4_multichannel members become processes (a C1 process with one channel,
    a C2 process with the C2 channels that follow it), so every channel keeps
    the local weights of its own process.  Returns (description, counts)."""
    members, counts = c4_multichannel(seed, n_channels, lo, hi)
    procs = []
    c2 = _c2_channels()
    for cfg, ch in members:
        if cfg == "c1":
            procs.append(c1_ee_mumu())
        else:
            if not procs or procs[-1]["name"] != "pp4j":
                d = c2_pp4j()
                d["channels"] = []
                procs.append(d)
            procs[-1]["channels"].append(c2[ch])
    return {"processes": procs}, counts


def counts_powerlaw(n: int, seed: int, lo: float, hi: float, exponent: float = -1.5) -> np.ndarray:
    """Event counts with density ~ n^exponent on [lo, hi] by inverse-CDF sampling
    of seeded Philox uniforms (one per channel)."""
    u = philox_uniforms(seed, stream=7, e0=0, n=n, d=1)[0]
    a = exponent + 1.0
    x = (lo ** a + u * (hi ** a - lo ** a)) ** (1.0 / a)
    return np.floor(x).astype(np.int64)


CONFIG_NAMES = {"c1": c1_ee_mumu, "c2": c2_pp4j, "c3": c3_ttbar6}


def to_json(desc: dict) -> str:
    return json.dumps(desc, separators=(",", ":"))


# ---------------------------------------------------------------------------
# Philox uniforms
# ---------------------------------------------------------------------------

def philox_raw(seed: int, stream: int, e0: int, n: int, group: int) -> np.ndarray:
    """Raw Philox4x64-10 output words [n, 4] for counters (e0..e0+n-1, group, 0, 0)."""
    if n == 0:
        return np.zeros((0, 4), dtype=np.uint64)
    if e0 < 0 or e0 + n > 2 ** 64 - 1:
        raise ValueError("event id range out of counter space")
    # numpy increments the 256-bit counter (with full carry) before each
    # block, so start one below the first wanted counter (e0, group, 0, 0).
    top = 2 ** 64 - 1
    if e0 > 0:
        ctr = np.array([e0 - 1, group, 0, 0], dtype=np.uint64)
    elif group > 0:
        ctr = np.array([top, group - 1, 0, 0], dtype=np.uint64)
    else:
        ctr = np.array([top, top, top, top], dtype=np.uint64)
    bg = np.random.Philox(key=np.array([seed % 2 ** 64, stream % 2 ** 64], dtype=np.uint64),
                          counter=ctr)
    return bg.random_raw(4 * n).reshape(n, 4)


def philox_uniforms(seed: int, stream: int, e0: int, n: int, d: int) -> np.ndarray:
    """Uniforms in (0, 1), layout [d][n] (event index fastest)."""
    out = np.empty((d, n), dtype=np.float64)
    for g in range((d + 3) // 4):
        raw = philox_raw(seed, stream, e0, n, g)
        for j in range(4):
            k = 4 * g + j
            if k >= d:
                break
            out[k] = ((raw[:, j] >> np.uint64(11)).astype(np.float64) + 0.5) * _TWO_M53
    return out


def philox_uniforms_f32(seed: int, stream: int, e0: int, n: int, d: int) -> np.ndarray:
    """24-bit uniforms in (0, 1) as float32, layout [d][n]: the top 24 bits of
    the same Philox words, (k + 0.5) 2^-24."""
    out = np.empty((d, n), dtype=np.float32)
    for g in range((d + 3) // 4):
        raw = philox_raw(seed, stream, e0, n, g)
        for j in range(4):
            k = 4 * g + j
            if k >= d:
                break
            out[k] = ((raw[:, j] >> np.uint64(40)).astype(np.float64) + 0.5) * 2.0 ** -24
    return out


def flow_shapes(dims: int, bins: int, hidden: int):
    """Per-layer parameter blocks of the coupling flow, in storage order:
    W1 [hidden][d/2], b1, W2 [hidden][hidden], b2, W3, b3,
    W4 [(d/2)(3 bins + 1)][hidden], b4."""
    nh = dims // 2
    no = nh * (3 * bins + 1)
    return [(hidden, nh), (hidden,), (hidden, hidden), (hidden,), (hidden, hidden), (hidden,), (no, hidden), (no,)]


def flow_params(seed: int, dims: int, layers: int, bins: int, hidden: int, last_scale: float = 0.0) -> np.ndarray:
    """Flat float32 starting parameters: hidden layers uniform in
    +-1/sqrt(fan_in); the last layer N(0, last_scale^2) (zero: the flow starts
    as the identity)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(layers):
        shapes = flow_shapes(dims, bins, hidden)
        for i, s in enumerate(shapes):
            n = int(np.prod(s))
            if i >= 6:
                out.append(rng.standard_normal(n) * last_scale if last_scale else np.zeros(n))
            else:
                fan_in = s[1] if len(s) == 2 else shapes[i - 1][1]
                lim = 1.0 / np.sqrt(fan_in)
                out.append(rng.uniform(-lim, lim, n))
    return np.concatenate(out).astype(np.float32)


def rambo_process(n: int, sqrt_s: float = 1000.0, masses=None, rambo: bool = True) -> dict:
    """e+e- -> n particles (massless unless `masses`) at fixed sqrt(s) through
    one decay chain Q_1 -> 1 + Q_2, Q_2 -> 2 + Q_3, ..., Q_{n-1} -> n-1 + n,
    with FastRambo cluster masses (or, rambo=False, the power-law maps)."""
    leg = {"d": [n - 1, n], "rambo": rambo}
    for q in range(n - 2, 0, -1):
        leg = {"d": [q, leg], "rambo": rambo}
    leg.pop("rambo")  # the root decays at s-hat
    m = [0.0] * n if masses is None else [float(x) for x in masses]
    return {"name": f"rambo{n}", "sqrt_s": sqrt_s, "beams": "fixed", "masses": m, "nu": 0.8,
            "regulator": 1e-3, "vegas_bins": 64, "integrand": {}, "channels": [{"s": leg}]}


def chili_process(n: int, sqrt_s: float = 1000.0, masses=None, pt_min: float = 0.0, pdf=None,
                  props=None) -> dict:
    """Hadronic 2->n through one Chili channel (section 2.4): f = 1 unless a
    p_T cut, toy PDFs [a, b] or propagator factors are given."""
    ig = {}
    if pt_min > 0.0:
        ig["pt_min"] = float(pt_min)
    if pdf is not None:
        ig["pdf"] = [float(pdf[0]), float(pdf[1])]
    if props:
        ig["props"] = copy.deepcopy(props)
    m = [0.0] * n if masses is None else [float(x) for x in masses]
    return {"name": f"chili{n}", "sqrt_s": sqrt_s, "beams": "hadronic", "masses": m, "nu": 0.8,
            "regulator": 1e-3, "vegas_bins": 64, "integrand": ig, "channels": [{"chili": True}]}
