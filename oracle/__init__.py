"""Plain FP64 CPU oracle for the phase-space hot path of MadSpace (arXiv:2602.06895).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code
with the HIP library (``paper_2602_06895_amd``) and never imports it.

The per-event chain (VEGAS lookup, s-hat and invariant sampling, PDF
convolution, 2->2 t-channel blocks, (phi, theta) decays, beam boost, Jacobian
product, unphysical cut, integrand and local channel weight) lives in
``oracle.c``.  This module compiles a process description into the oracle's
own node-tree form, and implements in numpy the host-level pieces: VEGAS grid
refinement, per-channel statistics and the unweighting efficiency.

Parity status of each function is listed in the docstrings; everything here is
pinned by the ``-m "not gpu"`` tests against closed forms, invariants and
brute force, except where a docstring says "parity unpinned".
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
# Builds of the same source: the reference (SSE2 doubles, no FMA
# contraction); an x87 build whose intermediates carry extra precision; and
# two builds in which every transcendental and square-root result is moved by
# one ulp up / down.  The others only serve as re-roundings of the same
# formulas: their spread estimates each event's FP64 forward error.
_VARIANTS = {
    "ref": ("liboracle.so", ["-ffp-contract=off"]),
    "x87": ("liboracle_x87.so", ["-ffp-contract=off", "-mfpmath=387"]),
    "up": ("liboracle_up.so", ["-ffp-contract=off", "-DORC_LIBM_NUDGE=1"]),
    "down": ("liboracle_down.so", ["-ffp-contract=off", "-DORC_LIBM_NUDGE=-1"]),
}

LEAF, CLUSTER, TNODE = 0, 1, 2


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (plain -O2, no fast-math, OpenMP)."""
    for name, (so, flags) in _VARIANTS.items():
        out = os.path.join(_HERE, so)
        if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
            tmp = out + ".tmp%d" % os.getpid()
            cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-Wall",
                   "-Wno-unused-function"] + flags + [_SRC, "-o", tmp, "-lm"]
            subprocess.run(cmd, check=True)
            os.replace(tmp, out)
    return os.path.join(_HERE, _VARIANTS["ref"][0])


_libs = {}


def build_mutant(k: int, directory: str) -> str:
    """Build oracle.c with planted mistake k (ORC_MUTATE, see the source) into
    `directory` and register it as variant "mutant<k>" of lib(): pin-strength
    tests check that their pins reject it."""
    name = f"mutant{k}"
    out = os.path.join(directory, f"liboracle_{name}.so")
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-Wall", "-Wno-unused-function",
           "-ffp-contract=off", f"-DORC_MUTATE={int(k)}", _SRC, "-o", out, "-lm"]
    subprocess.run(cmd, check=True)
    _libs.pop(name, None)
    _libs[name] = _load(out)
    return name


def build_timing(directory: str) -> str:
    """Build the same oracle source for timing on this host (-O3
    -march=native, still no FMA contraction, OpenMP) into `directory` and
    register it as variant "timing" of lib(): the CPU baseline's build.
    Compiled where it runs, since -march=native targets the build machine."""
    out = os.path.join(directory, "liboracle_timing.so")
    cmd = ["gcc", "-O3", "-march=native", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-Wall",
           "-Wno-unused-function", "-ffp-contract=off", _SRC, "-o", out, "-lm"]
    subprocess.run(cmd, check=True)
    _libs.pop("timing", None)
    _libs["timing"] = _load(out)
    return "timing"


def lib(variant: str = "ref"):
    if variant not in _libs:
        build()
        _libs[variant] = _load(os.path.join(_HERE, _VARIANTS[variant][0]))
    return _libs[variant]


def _load(path: str):
    """Open one build of oracle.c and declare its C signatures."""
    L = C.CDLL(path)
    dp = C.POINTER(C.c_double)
    L.orc_map.restype = C.c_int
    L.orc_weight.restype = C.c_int
    L.orc_kallen.restype = C.c_double
    L.orc_kallen.argtypes = [C.c_double] * 3
    L.orc_map_nu.restype = C.c_double
    L.orc_map_nu.argtypes = [C.c_double] * 5 + [dp]
    L.orc_map_bw.restype = C.c_double
    L.orc_map_bw.argtypes = [C.c_double] * 5 + [dp]
    L.orc_two_body_decay.restype = C.c_double
    L.orc_two_body_decay.argtypes = [dp, C.c_double, C.c_double, C.c_double, C.c_double,
                                     C.c_double, dp, dp]
    L.orc_two_to_two.restype = C.c_double
    L.orc_two_to_two.argtypes = [dp, dp] + [C.c_double] * 9 + [dp, dp, dp]
    L.orc_two_to_two_st.restype = C.c_double
    L.orc_two_to_two_st.argtypes = [dp, dp, dp] + [C.c_double] * 9 + [dp, dp, dp, dp]
    L.orc_two_to_two_st_inverse.restype = None
    L.orc_two_to_two_st_inverse.argtypes = [dp, dp, dp] + [C.c_double] * 5 + [dp, C.c_double, C.c_double, dp, dp]
    L.orc_t_range.restype = None
    L.orc_t_range.argtypes = [C.c_double] * 5 + [dp, dp]
    L.orc_r_to_x1x2.restype = C.c_double
    L.orc_r_to_x1x2.argtypes = [C.c_double, C.c_double, C.c_double, dp, dp]
    L.orc_vegas_map.restype = C.c_double
    L.orc_vegas_map.argtypes = [C.c_double, dp, C.c_int32, dp]
    L.orc_boost.restype = None
    L.orc_boost.argtypes = [dp, C.c_double, dp, dp]
    L.orc_inverse.restype = C.c_int
    L.orc_unmap_nu.restype = C.c_double
    L.orc_unmap_nu.argtypes = [C.c_double] * 5
    L.orc_unmap_bw.restype = C.c_double
    L.orc_unmap_bw.argtypes = [C.c_double] * 5
    L.orc_rqf.restype = C.c_double
    L.orc_rqf.argtypes = [C.c_double, C.c_double]
    L.orc_rqf_inverse.restype = C.c_double
    L.orc_rqf_inverse.argtypes = [C.c_double, C.c_double]
    L.orc_rambo_ck.restype = C.c_double
    L.orc_rambo_ck.argtypes = [C.c_int32]
    L.orc_vegas_unmap.restype = C.c_double
    L.orc_vegas_unmap.argtypes = [C.c_double, dp, C.c_int32]
    return L


OBS_E, OBS_PT, OBS_ETA, OBS_PHI, OBS_M, OBS_PT_RANK, OBS_DR_HARDEST = range(7)


def observables(p: np.ndarray, spec) -> np.ndarray:
    """Observables of lab-frame events p [4][np][n] (final-state particle i
    at index i + 2) for spec = [(kind, labels, rank), ...] (the distributions
    of section 4.2): energy, transverse momentum, pseudorapidity asinh(p_z /
    p_T), azimuth and invariant mass of the summed momentum of the labels;
    p_T of the rank-th hardest label (p_T descending, lower label first on
    ties) and the separation sqrt(d_eta^2 + d_phi^2) of the two hardest."""
    p = np.asarray(p, np.float64)
    n = p.shape[2]
    out = np.empty((len(spec), n))
    for j, (kind, labels, rank) in enumerate(spec):
        labels = sorted(labels)
        if kind in (OBS_PT_RANK, OBS_DR_HARDEST):
            pts = np.array([np.sqrt(p[1, q + 2] ** 2 + p[2, q + 2] ** 2) for q in labels])  # [m][n]
            # stable order: p_T descending, lower label first on equal p_T
            order = np.argsort(-pts, axis=0, kind="stable")
            if kind == OBS_PT_RANK:
                out[j] = np.take_along_axis(pts, order[rank:rank + 1], axis=0)[0] if rank < len(labels) else 0.0
                continue
            a = np.array(labels)[order[0]]
            b = np.array(labels)[order[1]]
            idx = np.arange(n)

            def eta(q):
                px, py, pz = p[1, q + 2, idx], p[2, q + 2, idx], p[3, q + 2, idx]
                return np.arcsinh(pz / np.sqrt(px * px + py * py))

            dphi = np.abs(np.arctan2(p[2, a + 2, idx], p[1, a + 2, idx]) - np.arctan2(p[2, b + 2, idx], p[1, b + 2, idx]))
            dphi = np.where(dphi > np.pi, 2.0 * np.pi - dphi, dphi)
            deta = eta(a) - eta(b)
            out[j] = np.sqrt(deta * deta + dphi * dphi)
            continue
        E = np.zeros(n)
        X = np.zeros(n)
        Y = np.zeros(n)
        Z = np.zeros(n)
        for q in labels:
            E = E + p[0, q + 2]
            X = X + p[1, q + 2]
            Y = Y + p[2, q + 2]
            Z = Z + p[3, q + 2]
        pt = np.sqrt(X * X + Y * Y)
        if kind == OBS_E:
            out[j] = E
        elif kind == OBS_PT:
            out[j] = pt
        elif kind == OBS_ETA:
            out[j] = np.arcsinh(Z / pt)
        elif kind == OBS_PHI:
            out[j] = np.arctan2(Y, X)
        else:
            out[j] = np.sqrt(np.maximum(E * E - X * X - Y * Y - Z * Z, 0.0))
    return out


def cut(x: np.ndarray, lo, hi, w: np.ndarray) -> np.ndarray:
    """w with every event outside lo[j] <= x[j] < hi[j] (any j) set to 0."""
    x = np.asarray(x, np.float64)
    keep = np.all((x >= np.asarray(lo)[:, None]) & (x < np.asarray(hi)[:, None]), axis=0)
    return np.where(keep, w, 0.0)


def histogram(x: np.ndarray, w: np.ndarray, bins: int, lo: float, hi: float) -> np.ndarray:
    """[2][bins]: sum w and sum w^2 per equal bin of [lo, hi), bin =
    floor((x - lo) bins / (hi - lo)); events outside [lo, hi) not counted."""
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    inside = (x >= lo) & (x < hi)
    scale = bins / (hi - lo)
    b = np.clip(np.floor((x[inside] - lo) * scale).astype(np.int64), 0, bins - 1)
    wi = w[inside]
    return np.stack([np.bincount(b, weights=wi, minlength=bins), np.bincount(b, weights=wi * wi, minlength=bins)])


def unweight(w: np.ndarray, w_max: float, u: np.ndarray) -> dict:
    """Hit-or-miss unweighting (section 3.4.1): event i is kept when
    u_i w_max < w_i (u: the uniforms drawn for the decision, passed in) and
    carries the unit weight max(1, w_i / w_max).  Returns the kept indices in
    increasing order and their unit weights."""
    w = np.asarray(w, np.float64)
    keep = np.nonzero(u * w_max < w)[0]
    return {"keep": keep, "uw": np.maximum(1.0, w[keep] / w_max)}


class _Channel(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("root", C.c_int32), ("n_sorder", C.c_int32),
                ("n_dec", C.c_int32),
                ("kind", C.c_void_p), ("particle", C.c_void_p), ("parent", C.c_void_p),
                ("child_start", C.c_void_p), ("child_count", C.c_void_p), ("children", C.c_void_p),
                ("mass", C.c_void_p), ("width", C.c_void_p), ("nu", C.c_void_p),
                ("t_order", C.c_char_p), ("s_order", C.c_void_p), ("dec_order", C.c_void_p),
                ("rambo", C.c_void_p), ("chili", C.c_int32), ("st", C.c_int32)]


class _Process(C.Structure):
    _fields_ = [("hadronic", C.c_int32), ("n_final", C.c_int32), ("s_lab", C.c_double),
                ("shat_min", C.c_double), ("nu", C.c_double), ("reg_a", C.c_double),
                ("mass", C.c_void_p),
                ("pdf", C.c_int32), ("pdf_a", C.c_double), ("pdf_b", C.c_double),
                ("pt_min", C.c_double), ("ang", C.c_int32), ("n_prop", C.c_int32),
                ("prop_t", C.c_void_p), ("prop_set", C.c_void_p), ("prop_bw", C.c_void_p),
                ("prop_m", C.c_void_p), ("prop_w", C.c_void_p), ("prop_mu", C.c_void_p),
                ("n_chan", C.c_int32), ("alpha_mu", C.c_double), ("ch_start", C.c_void_p),
                ("chp_t", C.c_void_p), ("chp_set", C.c_void_p), ("chp_m", C.c_void_p),
                ("chp_w", C.c_void_p), ("ch_prior", C.c_void_p)]


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p) if a.size else None


class ChannelTree:
    """One channel as a node tree (the oracle's own channel compiler).

    Node 0 is the root: the effective t-node with the spine legs as children
    (t-channel topologies), or the cluster decaying at s-hat (pure s-channel)."""

    def __init__(self, chan: dict, masses, nu: float):
        self.kind, self.particle, self.parent, self.children = [], [], [], []
        self.mass, self.width, self.nu, self.order = [], [], [], []
        self.rambo = []  # FastRambo clusters: their particle count - 1, else 0
        self.chili = bool(chan.get("chili"))
        # t-chain blocks after the first in the (s~, t) parametrisation
        self.st = bool(chan.get("st"))
        if self.chili:
            # Chili (section 2.4): no tree, 3 random numbers per particle but
            # the last, which takes only its rapidity
            self.n_final = len(masses)
            self.t_order, self.s_order, self.dec_order, self.kappa = "", [], [], 0
            return

        def add(leg, parent):
            idx = len(self.kind)
            self.parent.append(parent)
            self.children.append([])
            if isinstance(leg, (int, np.integer)):
                lab = int(leg)
                if not 1 <= lab <= len(masses):
                    raise ValueError(f"particle label {lab} out of range")
                self.kind.append(LEAF)
                self.particle.append(lab - 1)
                self.mass.append(float(masses[lab - 1]))
                self.width.append(0.0)
                self.nu.append(nu)
                self.order.append(None)
                self.rambo.append(0)
            else:
                kids = leg["d"]
                if len(kids) not in (2, 3):
                    raise ValueError("a cluster decays into two or three children")
                if len(kids) == 3 and leg.get("rambo"):
                    raise ValueError("a FastRambo cluster decays into two children")
                self.kind.append(CLUSTER)
                self.particle.append(-1)
                self.mass.append(float(leg.get("m", 0.0)))
                self.width.append(float(leg.get("w", 0.0)))
                self.nu.append(float(leg.get("nu", nu)))
                self.order.append(leg.get("order"))
                self.rambo.append(-1 if leg.get("rambo") else 0)
                for kid in kids:
                    self.children[idx].append(add(kid, idx))
            if self.rambo[idx] < 0:
                self.rambo[idx] = len(self.particles(idx)) - 1
            return idx

        if "t_chain" in chan:
            legs = chan["t_chain"]
            if len(legs) < 2:
                raise ValueError("a t-channel spine needs at least two legs")
            self.kind.append(TNODE)
            self.particle.append(-1)
            self.parent.append(-1)
            self.children.append([])
            self.mass.append(0.0)
            self.width.append(0.0)
            self.nu.append(nu)
            self.order.append(None)
            self.rambo.append(0)
            for leg in legs:
                self.children[0].append(add(leg, 0))
            self.t_order = chan.get("t_order", "")
            kappa = len(legs) - 1
            if len(self.t_order) != kappa - 1 or any(c not in "AB" for c in self.t_order):
                raise ValueError("t_order needs kappa-1 letters from {A, B}")
        else:
            add(chan["s"], -1)
            if self.kind[0] != CLUSTER:
                raise ValueError("a pure s-channel root must be a cluster")
            self.t_order = ""
        leaves = sorted(self.particle[j] for j in range(len(self.kind)) if self.kind[j] == LEAF)
        if leaves != list(range(len(masses))):
            raise ValueError("every final-state particle must appear exactly once")
        clusters = [j for j in range(len(self.kind)) if self.kind[j] == CLUSTER and j != 0]
        # sampling order: explicit "order" keys first, then depth-first order
        self.s_order = sorted(clusters, key=lambda j: (self.order[j] is None,
                                                       self.order[j] if self.order[j] is not None else 0, j))
        self.dec_order = [j for j in range(len(self.kind)) if self.kind[j] == CLUSTER]
        self.kappa = len(self.children[0]) - 1 if self.kind[0] == TNODE else 0

    def particles(self, j):
        if self.kind[j] == LEAF:
            return [self.particle[j]]
        out = []
        for c in self.children[j]:
            out += self.particles(c)
        return out

    def dims(self, hadronic: bool) -> int:
        if self.chili:
            if not hadronic:
                raise ValueError("a Chili channel samples x1, x2 from the momenta: hadronic beams only")
            return 3 * self.n_final - 2
        # (phi, theta) per two-body decay, (E1, E2, phi, theta, beta) per 1 -> 3
        dec = sum(5 if len(self.children[j]) == 3 else 2 for j in self.dec_order)
        d = len(self.s_order) + max(self.kappa - 1, 0) + 2 * self.kappa + dec
        return d + (2 if hadronic else 0)

    def propagators(self):
        """(t_type, particle set, mass, width) of every internal line."""
        out = []
        if self.chili:
            return out
        if self.kind[0] == TNODE:
            acc = []
            for leg in self.children[0][:-1]:
                acc = acc + self.particles(leg)
                out.append((1, _mask(acc), 0.0, 0.0))
        for j in range(len(self.kind)):
            if self.kind[j] == CLUSTER:
                out.append((0, _mask(self.particles(j)), self.mass[j], self.width[j]))
        return out

    def struct(self):
        n = len(self.kind)
        starts, counts, flat = [], [], []
        for j in range(n):
            starts.append(len(flat))
            counts.append(len(self.children[j]))
            flat += self.children[j]
        self._keep = dict(
            kind=np.array(self.kind, np.int32), particle=np.array(self.particle, np.int32),
            parent=np.array(self.parent, np.int32), child_start=np.array(starts, np.int32),
            child_count=np.array(counts, np.int32), children=np.array(flat + [0], np.int32),
            mass=np.array(self.mass, np.float64), width=np.array(self.width, np.float64),
            nu=np.array(self.nu, np.float64), s_order=np.array(self.s_order + [0], np.int32),
            dec_order=np.array(self.dec_order + [0], np.int32),
            t_order=self.t_order.encode() + b"\0", rambo=np.array(self.rambo, np.int32))
        k = self._keep
        return _Channel(n, 0, len(self.s_order), len(self.dec_order),
                        _ptr(k["kind"]), _ptr(k["particle"]), _ptr(k["parent"]),
                        _ptr(k["child_start"]), _ptr(k["child_count"]), _ptr(k["children"]),
                        _ptr(k["mass"]), _ptr(k["width"]), _ptr(k["nu"]), k["t_order"],
                        _ptr(k["s_order"]), _ptr(k["dec_order"]), _ptr(k["rambo"]), int(self.chili),
                        int(self.st))


def _mask(parts):
    m = 0
    for p in parts:
        m |= 1 << p
    return m


class Process:
    """A process description compiled for the oracle."""

    def __init__(self, desc: dict):
        self.desc = desc
        self.masses = [float(m) for m in desc["masses"]]
        self.n = len(self.masses)
        self.hadronic = desc.get("beams", "hadronic") == "hadronic"
        self.s_lab = float(desc["sqrt_s"]) ** 2
        self.nu = float(desc.get("nu", 0.8))
        self.reg_a = float(desc.get("regulator", 1e-3))
        self.nbins = int(desc.get("vegas_bins", 64))
        self.channels = [ChannelTree(c, self.masses, self.nu) for c in desc["channels"]]
        self.dims = [c.dims(self.hadronic) for c in self.channels]
        ig = desc.get("integrand", {})
        pdf = ig.get("pdf")
        props = ig.get("props", [])
        self._k = dict(
            mass=np.array(self.masses, np.float64),
            prop_t=np.array([1 if p.get("t") else 0 for p in props] + [0], np.int32),
            prop_set=np.array([_mask([q - 1 for q in p["particles"]]) for p in props] + [0], np.uint32),
            prop_bw=np.array([1 if p.get("bw") else 0 for p in props] + [0], np.int32),
            prop_m=np.array([float(p.get("m", 0.0)) for p in props] + [0], np.float64),
            prop_w=np.array([float(p.get("w", 0.0)) for p in props] + [0], np.float64),
            prop_mu=np.array([float(p.get("mu", 0.0)) for p in props] + [0], np.float64),
        )
        chp, start = [], [0]
        for c in self.channels:
            chp += c.propagators()
            start.append(len(chp))
        self._k.update(
            ch_start=np.array(start, np.int32),
            chp_t=np.array([q[0] for q in chp] + [0], np.int32),
            chp_set=np.array([q[1] for q in chp] + [0], np.uint32),
            chp_m=np.array([q[2] for q in chp] + [0], np.float64),
            chp_w=np.array([q[3] for q in chp] + [0], np.float64),
            ch_prior=np.array([1 if c.chili else 0 for c in self.channels], np.int32))
        k = self._k
        n_chan = len(self.channels) if "alpha_mu" in desc else 1
        self._proc = _Process(
            1 if self.hadronic else 0, self.n, self.s_lab, float(desc.get("shat_min", 0.0)),
            self.nu, self.reg_a, _ptr(k["mass"]),
            1 if pdf else 0, float(pdf[0]) if pdf else 0.0, float(pdf[1]) if pdf else 0.0,
            float(ig.get("pt_min", 0.0)), int(ig["ang"]) - 1 if "ang" in ig else -1, len(props),
            _ptr(k["prop_t"]), _ptr(k["prop_set"]), _ptr(k["prop_bw"]), _ptr(k["prop_m"]),
            _ptr(k["prop_w"]), _ptr(k["prop_mu"]), n_chan, float(desc.get("alpha_mu", 0.0)),
            _ptr(k["ch_start"]), _ptr(k["chp_t"]), _ptr(k["chp_set"]), _ptr(k["chp_m"]),
            _ptr(k["chp_w"]), _ptr(k["ch_prior"]))
        self._chs = [c.struct() for c in self.channels]

    def uniform_grid(self, chan: int) -> np.ndarray:
        nb = self.nbins
        e = np.arange(nb + 1, dtype=np.float64) / nb
        return np.tile(e, (self.dims[chan], 1))

    def map(self, chan: int, y: np.ndarray, grid: np.ndarray | None = None,
            nthreads: int = 0, want_inv: bool = False, variant: str = "ref") -> dict:
        """Run the per-event chain on uniforms y [dims][n] through the VEGAS grid
        [dims][nb+1] (None: no VEGAS step).  Returns p [4][n+2][N] (lab frame,
        incoming a, b first), x1x2 [2][N], jac, w, alpha, f (and inv when asked)."""
        d = self.dims[chan]
        y = np.ascontiguousarray(y, dtype=np.float64)
        if y.ndim != 2 or y.shape[0] != d:
            raise ValueError(f"y must be [{d}][n]")
        n = y.shape[1]
        np_ = self.n + 2
        out = dict(p=np.empty((4, np_, n)), x1x2=np.empty((2, n)), jac=np.empty(n),
                   w=np.empty(n), alpha=np.empty(n), f=np.empty(n))
        if want_inv:
            out["inv"] = np.empty((len(self.channels[chan].kind), n))
            out["tabs"] = np.empty((self.channels[chan].kappa, n))
        g = None
        if grid is not None:
            g = np.ascontiguousarray(grid, dtype=np.float64)
            if g.shape != (d, self.nbins + 1):
                raise ValueError("grid shape mismatch")
        nt = nthreads if nthreads > 0 else (os.cpu_count() or 1)
        dp = lambda a: a.ctypes.data_as(C.c_void_p) if a is not None else None
        rc = lib(variant).orc_map(C.byref(self._proc), C.byref(self._chs[chan]), C.c_int32(chan),
                           C.c_int32(d), C.c_int64(n), dp(y), dp(g), C.c_int32(self.nbins),
                           dp(out["p"]), dp(out["x1x2"]), dp(out["jac"]), dp(out["w"]),
                           dp(out["alpha"]), dp(out["f"]), dp(out.get("inv")),
                           dp(out.get("tabs")), C.c_int32(nt))
        if rc != 0:
            raise ValueError("oracle rejected the sizes")
        return out

    def inverse(self, chan: int, p: np.ndarray, x1x2: np.ndarray | None, grid: np.ndarray | None = None,
                nthreads: int = 0, variant: str = "ref") -> dict:
        """Inverse of map(): the uniforms y [dims][N] that the channel maps to the
        lab-frame momenta p [4][n+2][N] and x1x2 [2][N], through the inverse
        VEGAS grid when given, and jac [N] = the forward Jacobian at y (the
        channel density of the event is 1/jac)."""
        d = self.dims[chan]
        p = np.ascontiguousarray(p, dtype=np.float64)
        n = p.shape[2]
        if p.shape != (4, self.n + 2, n):
            raise ValueError("p shape mismatch")
        x = None if x1x2 is None else np.ascontiguousarray(x1x2, dtype=np.float64)
        if self.hadronic and (x is None or x.shape != (2, n)):
            raise ValueError("x1x2 [2][n] required")
        g = None
        if grid is not None:
            g = np.ascontiguousarray(grid, dtype=np.float64)
            if g.shape != (d, self.nbins + 1):
                raise ValueError("grid shape mismatch")
        y, jac = np.empty((d, n)), np.empty(n)
        nt = nthreads if nthreads > 0 else (os.cpu_count() or 1)
        dp = lambda a: a.ctypes.data_as(C.c_void_p) if a is not None else None
        rc = lib(variant).orc_inverse(C.byref(self._proc), C.byref(self._chs[chan]), C.c_int32(chan),
                                      C.c_int32(d), C.c_int64(n), dp(p), dp(x), dp(g), C.c_int32(self.nbins),
                                      dp(y), dp(jac), C.c_int32(nt))
        if rc != 0:
            raise ValueError("oracle rejected the sizes")
        return {"y": y, "jac": jac}

    def inverse_forward_error(self, chan: int, p, x1x2, grid=None, ref: dict | None = None) -> dict:
        """Forward-error estimate of inverse(): the largest deviation from the
        reference among the x87 build and the builds with every libm / sqrt
        result and every input momentum moved by one ulp."""
        ref = ref if ref is not None else self.inverse(chan, p, x1x2, grid)
        alts = [self.inverse(chan, p, x1x2, grid, variant=v) for v in ("x87", "up", "down")]
        den = np.where(ref["jac"] != 0.0, np.abs(ref["jac"]), 1.0)
        return {"y": np.max([np.abs(o["y"] - ref["y"]).max(axis=0) for o in alts], axis=0),
                "jac": np.max([np.abs(o["jac"] - ref["jac"]) / den for o in alts], axis=0)}

    def multichannel_density(self, p: np.ndarray, x1x2: np.ndarray | None, alpha, grids=None,
                             variant: str = "ref") -> np.ndarray:
        """Global multichannel density g(p) = sum_c alpha_c / J_c(y_c(p)) over
        this process's channels (section 2.1, Kleiss-Pittau form): each
        channel's inverse map gives y_c and the forward Jacobian there; a
        channel whose chain cuts the event (J = 0) contributes 0."""
        g = np.zeros(p.shape[2])
        for c in range(len(self.channels)):
            inv = self.inverse(c, p, x1x2, None if grids is None else grids[c], variant=variant)
            j = inv["jac"]
            g += np.where(j > 0, alpha[c] / np.where(j > 0, j, 1.0), 0.0)
        return g

    def weight(self, chan: int, p: np.ndarray, x1x2: np.ndarray | None, jac: np.ndarray,
               nthreads: int = 0, variant: str = "ref") -> dict:
        """w = alpha_c f jac from lab-frame momenta p [4][n+2][N], x1x2 [2][N]
        and jac [N]; returns w and alpha."""
        p = np.ascontiguousarray(p, dtype=np.float64)
        jac = np.ascontiguousarray(jac, dtype=np.float64)
        n = jac.size
        if p.shape != (4, self.n + 2, n):
            raise ValueError("p shape mismatch")
        x = None if x1x2 is None else np.ascontiguousarray(x1x2, dtype=np.float64)
        if self.hadronic and (x is None or x.shape != (2, n)):
            raise ValueError("x1x2 [2][n] required")
        w, a = np.empty(n), np.empty(n)
        nt = nthreads if nthreads > 0 else (os.cpu_count() or 1)
        dp = lambda arr: arr.ctypes.data_as(C.c_void_p) if arr is not None else None
        rc = lib(variant).orc_weight(C.byref(self._proc), C.c_int32(chan), C.c_int64(n), dp(p), dp(x),
                                     dp(jac), dp(w), dp(a), C.c_int32(nt))
        if rc != 0:
            raise ValueError("oracle rejected the sizes")
        return {"w": w, "alpha": a}

    def weight_forward_error(self, chan: int, p, x1x2, jac, ref: dict | None = None) -> dict:
        """Forward-error estimate of weight(): largest deviation from the
        reference among the x87 and the one-ulp perturbation builds."""
        ref = ref if ref is not None else self.weight(chan, p, x1x2, jac)
        a = ref["w"]
        den = np.where(a != 0.0, np.abs(a), 1.0)
        alts = [self.weight(chan, p, x1x2, jac, variant=v) for v in ("x87", "up", "down")]
        return {"w": np.max([np.abs(o["w"] - a) / den for o in alts], axis=0),
                "cut_ambiguous": np.any([(o["w"] == 0.0) != (a == 0.0) for o in alts], axis=0)}

    def forward_error(self, chan: int, y: np.ndarray, grid: np.ndarray | None = None,
                      ref: dict | None = None) -> dict:
        """Per-event estimate of the FP64 forward error of the reference
        evaluation: the largest deviation from it among the x87 build, the
        builds with every libm result moved one ulp up / down, and the
        reference build on inputs moved by one ulp up / down.
        Returns relative deviations of w and jac, and momentum deviations in
        units of the event's largest energy."""
        ref = ref if ref is not None else self.map(chan, y, grid)
        y = np.asarray(y, np.float64)
        alts = [self.map(chan, y, grid, variant="x87"),
                self.map(chan, y, grid, variant="up"),
                self.map(chan, y, grid, variant="down"),
                self.map(chan, np.nextafter(y, 1.0), grid),
                self.map(chan, np.nextafter(y, 0.0), grid)]
        emax = np.abs(ref["p"][0]).max(axis=0)
        out = {}
        for key in ("w", "jac"):
            a = ref[key]
            den = np.where(a != 0.0, np.abs(a), 1.0)
            out[key] = np.max([np.abs(o[key] - a) / den for o in alts], axis=0)
        out["p"] = np.max([np.abs(o["p"] - ref["p"]).max(axis=(0, 1)) / np.where(emax > 0, emax, 1.0)
                           for o in alts], axis=0)
        # events that some rounding variant keeps while the reference cuts them
        # (or the reverse): a cut decided within rounding
        out["cut_ambiguous"] = np.any([(o["w"] == 0.0) != (ref["w"] == 0.0) for o in alts], axis=0)
        return out


# ---------------------------------------------------------------------------
# VEGAS (Lepage 1978; "VEGAS enhanced" 2021), cited by the paper for its
# adaptive grids; the paper gives no formulas, the classic algorithm is used.
# ---------------------------------------------------------------------------

def vegas_histogram(y: np.ndarray, w: np.ndarray, nbins: int) -> np.ndarray:
    """d[k][i] = sum of w^2 over events whose uniform y_k lies in bin i."""
    y = np.asarray(y, np.float64)
    w2 = np.asarray(w, np.float64) ** 2
    out = np.zeros((y.shape[0], nbins))
    for k in range(y.shape[0]):
        b = np.minimum(np.floor(y[k] * nbins).astype(np.int64), nbins - 1)
        out[k] = np.bincount(b, weights=w2, minlength=nbins)
    return out


def vegas_refine(edges: np.ndarray, d: np.ndarray, alpha: float) -> np.ndarray:
    """One grid refinement per dimension: smooth the accumulated d_i with
    weights (1,6,1)/8 ((7,1)/8 at the ends), normalise, damp with
    omega_i = ((1 - d_i)/ln(1/d_i))^alpha, then move the edges so that every
    new bin holds the same share of sum(omega), linearly inside old bins."""
    edges = np.array(edges, np.float64, copy=True)
    d = np.asarray(d, np.float64)
    nb = d.shape[1]
    for k in range(edges.shape[0]):
        dk = d[k]
        if dk.sum() <= 0.0:
            continue
        sm = np.empty(nb)
        if nb == 1:
            sm[0] = dk[0]
        else:
            sm[0] = (7.0 * dk[0] + dk[1]) / 8.0
            sm[-1] = (dk[-2] + 7.0 * dk[-1]) / 8.0
            for i in range(1, nb - 1):
                sm[i] = (dk[i - 1] + 6.0 * dk[i] + dk[i + 1]) / 8.0
        sm = sm / sm.sum()
        om = np.empty(nb)
        for i in range(nb):
            if sm[i] <= 0.0:
                om[i] = 0.0
            elif sm[i] >= 1.0:
                om[i] = 1.0
            else:
                om[i] = ((1.0 - sm[i]) / math.log(1.0 / sm[i])) ** alpha
        total = om.sum()
        if total <= 0.0:
            continue
        share = total / nb
        old = edges[k].copy()
        new = np.empty(nb + 1)
        new[0], new[nb] = 0.0, 1.0
        i, acc = 0, 0.0  # acc: omega collected from old bins before bin i
        for j in range(1, nb):
            target = j * share
            while i < nb - 1 and acc + om[i] < target:
                acc += om[i]
                i += 1
            frac = (target - acc) / om[i] if om[i] > 0.0 else 0.0
            frac = min(max(frac, 0.0), 1.0)
            new[j] = old[i] + (old[i + 1] - old[i]) * frac
        edges[k] = new
    return edges


# ---------------------------------------------------------------------------
# Statistics and unweighting
# ---------------------------------------------------------------------------

def channel_stats(w: np.ndarray) -> np.ndarray:
    """[sum w, sum w^2, n, n with w == 0, max w] of one channel's weights."""
    w = np.asarray(w, np.float64)
    return np.array([w.sum(), (w * w).sum(), float(w.size), float((w == 0.0).sum()),
                     w.max() if w.size else 0.0])


def integral(stats: np.ndarray):
    """Multichannel estimate I = sum_c <w>_c and its error, stats [C][5]."""
    tot, var = 0.0, 0.0
    for s1, s2, n, _, _ in stats:
        if n <= 0:
            continue
        mean = s1 / n
        tot += mean
        if n > 1:
            var += max(s2 / n - mean * mean, 0.0) / (n - 1)
    return tot, math.sqrt(var)


def unweighting_efficiency(w: np.ndarray, overweight: float = 1e-3):
    """Smallest W with sum_i max(0, w_i - W) <= overweight * sum_i w_i; returns
    (mean(w)/W, W).  Computed exactly from the sorted weights: between two
    consecutive sorted weights the overweight sum is linear in W."""
    w = np.sort(np.asarray(w, np.float64))[::-1]
    n = w.size
    if n == 0:
        return 0.0, 0.0
    total = w.sum()
    if total <= 0.0:
        return 0.0, 0.0
    target = overweight * total
    csum = np.cumsum(w)
    # with the k largest weights at or above W, excess(W) = csum[k-1] - k W on
    # [w[k], w[k-1]]; the first interval whose lower end reaches the target
    # holds the crossing
    k = np.arange(1, n + 1, dtype=np.float64)
    lo = np.append(w[1:], 0.0)
    ex_lo = csum - k * lo
    kk = int(np.argmax(ex_lo >= target))
    W = (csum[kk] - target) / (kk + 1)
    W = max(W, 0.0)
    return (total / n) / W if W > 0 else 0.0, W
