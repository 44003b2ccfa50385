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
    assert L.msx_sample(None, None, 0, 0, 0, None, None, None, None, None) == 1
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
