"""Host-side checks of the C ABI: the library loads, exports every entry point
that include/msx.h declares, and rejects bad arguments synchronously (no GPU
needed: argument and description errors are caught before any device call)."""
import ctypes as C
import json
import os
import re

import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    import paper_2602_06895_amd as pkg

    if not os.path.exists(pkg.LIB_PATH):
        from paper_2602_06895_amd import build

        build.build()
    return pkg.load_library()


def declared_symbols():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            names |= set(re.findall(r"\b(msx_[a-z_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_binding_exports():
    import paper_2602_06895_amd as pkg

    assert declared_symbols() == sorted(pkg.EXPORTS)


def test_every_declared_symbol_is_exported(L):
    for name in declared_symbols():
        assert hasattr(L, name), name


def _create(L, text, precision=0):
    h = C.c_void_p()
    st = L.msx_create_channels(text.encode() if text is not None else None, precision, 0, C.byref(h))
    return st, h


@pytest.mark.parametrize("text,needle", [
    ("{", "JSON"),
    ("[1, 2]", "object"),
    (json.dumps({"sqrt_s": 100.0}), "masses"),
    (json.dumps({**W.c2_pp4j(), "channels": []}), "channels"),
    (json.dumps({**W.c2_pp4j(), "channels": [{"t_chain": [1, 2, 3, 4], "t_order": "A"}]}), "kappa-1"),
    (json.dumps({**W.c2_pp4j(), "channels": [{"t_chain": [1, 2, 3, 3], "t_order": "AA"}]}), "exactly once"),
    (json.dumps({**W.c2_pp4j(), "channels": [{"s": {"d": [1, 2, 3, 4]}}]}), "[child, child]"),
    (json.dumps({**W.c2_pp4j(), "vegas_bins": 1000}), "vegas_bins"),
    (json.dumps({**W.volume_process(3), "channels": [{"chili": True}]}), "hadronic beams"),
    (json.dumps({**W.c2_pp4j(), "channels": [{"chili": False}]}), "\"chili\" must be true"),
    (json.dumps({**W.volume_process(3), "channels": [{"s": {"d": [1, 2, 3], "rambo": True}}]}),
     "FastRambo cluster decays into two"),
    (json.dumps({**W.c1_ee_mumu(), "beams": "hadronic"}), "ang"),
    (json.dumps({**W.c2_pp4j(), "masses": [0.0] * 9, "channels": [{"t_chain": list(range(1, 10)),
                                                                     "t_order": "A" * 7}]}), "8 final"),
])
def test_bad_descriptions_are_rejected(L, text, needle):
    st, h = _create(L, text)
    assert st == 1 and not h.value
    assert needle in L.msx_last_error(None).decode()


def test_null_and_precision_errors(L):
    st, _ = _create(L, None)
    assert st == 1
    st, _ = _create(L, json.dumps(W.c1_ee_mumu()), precision=7)
    assert st == 1 and "precision" in L.msx_last_error(None).decode()
    assert L.msx_create_channels(b"{}", 0, 0, None) == 1


def test_calls_on_null_context_fail_cleanly(L):
    v = C.c_int64()
    assert L.msx_get_meta(None, 0, 0, C.byref(v)) == 1
    assert L.msx_map(None, 0, 10, None, None, None, None, None, None) == 1
    assert L.msx_sample(None, None, 0, 0, 0, 0, None, None, None, None, None) == 1
    assert L.msx_vegas_adapt(None, 10, 1, 0.5, 1, 0, 0, None, None) == 1
    assert L.msx_vegas_update(None, 0.5, None) == 1
    assert L.msx_destroy(None) == 0
    assert L.msx_last_error(None).decode() != ""


def test_valid_description_reaches_the_device_check(L):
    """Without a GPU a valid description compiles and fails only at the device."""
    import torch

    st, h = _create(L, json.dumps(W.c3_ttbar6()))
    if torch.cuda.is_available():
        assert st == 0
        L.msx_destroy(h)
    else:
        assert st == 2 and "device" in L.msx_last_error(None).decode()


def test_allocate_counts_is_neyman(L):
    """msx_allocate_counts (host only): counts proportional to each channel's
    weight standard deviation above a floor, summing to the total."""
    import numpy as np

    rng = np.random.default_rng(3)
    for C_ in (1, 3, 8, 24):
        n = rng.integers(100, 10000, C_).astype(float)
        mean = rng.random(C_)
        sd = rng.random(C_) * 2.0
        if C_ > 1:
            sd[0] = 0.0
        stats = np.stack([mean * n, (sd ** 2 + mean ** 2) * n, n, np.zeros(C_), np.ones(C_)], axis=1)
        total, floor = 1_000_003, 0.01
        out = np.zeros(C_, dtype=np.int64)
        assert L.msx_allocate_counts(C_, stats.ctypes.data, total, floor, out.ctypes.data) == 0
        assert out.sum() == total and (out >= int(floor * total)).all()
        rest = total - int(floor * total) * C_
        got = sd / sd.sum()
        share = (out - int(floor * total)) / rest
        assert np.abs(share - got).max() <= C_ / rest + 1e-9
    # degenerate: every channel flat -> equal shares
    stats = np.tile([2.0, 4.0, 2.0, 0.0, 1.0], (4, 1))
    out = np.zeros(4, dtype=np.int64)
    assert L.msx_allocate_counts(4, stats.ctypes.data, 10, 0.0, out.ctypes.data) == 0
    assert out.tolist() == [4, 2, 2, 2]
    assert L.msx_allocate_counts(4, stats.ctypes.data, -1, 0.0, out.ctypes.data) == 1
    assert L.msx_allocate_counts(4, stats.ctypes.data, 10, 0.5, out.ctypes.data) == 1
