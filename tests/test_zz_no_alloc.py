"""msx_sample_noalloc (the allocation-free variant of msx_sample, its tile
statistics in the library's fixed device scratch) against msx_sample, through
the C ABI: bit-identical events, weights, channel ids and momentum fractions,
and the same statistics, on two calls in a row, the second smaller (the
scratch keeps the first call's contents); sizes beyond the scratch are
refused before any launch."""
import ctypes as C

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t

    if not t.cuda.is_available():
        pytest.skip("needs a GPU")
    return t


def _call(ctx, fn, counts, seed, sid, off, out):
    s = ctx._stream()
    c = np.ascontiguousarray(counts, dtype=np.int64)
    p, x, w, ch = (out[k].data_ptr() if out[k] is not None else None for k in ("p", "x1x2", "w", "chan"))
    if fn == "sample":
        return ctx.L.msx_sample(ctx.h, c.ctypes.data, seed, sid, off, 0, p, x, w, ch, s)
    return ctx.L.msx_sample_noalloc(ctx.h, c.ctypes.data, seed, sid, off, p, x, w, ch, s)


@pytest.mark.parametrize("cfg,ept", [("c2", 4), ("c2", 1), ("c3", 2)])
def test_noalloc_equals_sample(torch, cfg, ept):
    from paper_2602_06895_amd import Context

    desc = {"c2": W.c2_pp4j, "c3": W.c3_ttbar6}[cfg]()
    a, b = Context(desc), Context(desc)
    for ctx in (a, b):
        ctx.set_launch(ept, 0)
    C_ = a.n_channels
    calls = ([np.array([40000, 3, 0, 25000, 1025, 1, 77777, 6000])[:C_] if C_ > 1 else np.array([150001]),
              np.array([100, 0, 0, 0, 257, 1, 0, 2])[:C_] if C_ > 1 else np.array([1023])])
    for i, counts in enumerate(calls):
        N = int(counts.sum())
        oa, ob = a.sample_buffers(N), b.sample_buffers(N)
        a.reset_stats()
        b.reset_stats()
        assert _call(a, "sample", counts, 7 + i, 1, 1000 * i, oa) == 0, a.L.msx_last_error(a.h)
        assert _call(b, "noalloc", counts, 7 + i, 1, 1000 * i, ob) == 0, b.L.msx_last_error(b.h)
        torch.cuda.synchronize()
        for k in ("p", "w", "chan", "x1x2"):
            if oa[k] is not None:
                assert torch.equal(oa[k], ob[k]), f"call {i}: {k} differs"
        sa, sb = a.stats(), b.stats()
        assert np.array_equal(sa, sb), f"call {i}: statistics differ"
        assert np.array_equal(sa[:, 2], counts.astype(float))
    a.close()
    b.close()


def test_noalloc_refuses_beyond_scratch(torch):
    from paper_2602_06895_amd import Context

    ctx = Context(W.c2_pp4j())
    ctx.set_launch(1, 0)
    counts = np.zeros(8, dtype=np.int64)
    counts[0] = 256 * (1 << 17) + 1  # one tile more than the scratch holds
    # full-size buffers: the refusal is a host check, but a launch would stay in bounds
    out = ctx.sample_buffers(int(counts.sum()), want_chan=False)
    assert _call(ctx, "noalloc", counts, 1, 0, 0, out) == 1
    assert b"fixed scratch" in ctx.L.msx_last_error(ctx.h)
    ctx.close()
