"""The allocation-free crop gather (lbsg_gather_noalloc) against lbsg_gather: the same
crops, bit for bit, on two calls in a row (the second smaller, so stale scratch contents
from the first call would show), and its size limit."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _call(name, field, h, w, yx, crop, cond, x, y, stream):
    from paper_2501_03759_amd import lbsg
    L = lbsg._bind()
    k = yx.shape[0]
    nc = 0 if cond is None else cond.shape[1]
    cp = None if cond is None else cond.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    return getattr(L, name)(ctypes.c_void_p(field.data_ptr()), h, w, yx.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                            k, crop, cp, nc, ctypes.c_void_p(x.data_ptr()) if x is not None else None,
                            ctypes.c_void_p(y.data_ptr()) if y is not None else None,
                            ctypes.c_void_p(stream.cuda_stream))


def test_noalloc_gather_matches_gather_on_two_calls():
    import torch
    from paper_2501_03759_amd import lbch
    stream = torch.cuda.Stream()
    rng = np.random.default_rng(17)
    h, w = 96, 160
    field = torch.tensor(rng.normal(size=(h, w)).astype(np.float32), device="cuda")
    # call 1: 700 crops of 40 x 40 with 4 conditioning values; call 2: 90 crops of 24 x 24 with 2
    for k, crop, nc in ((700, 40, 4), (90, 24, 2)):
        print(f"case noalloc gather k={k} crop={crop} ncond={nc}", flush=True)
        yx = np.ascontiguousarray(np.stack([rng.integers(-h, 2 * h, size=k), rng.integers(-w, 2 * w, size=k)], 1),
                                  dtype=np.int32)
        cond = np.ascontiguousarray(rng.normal(size=(k, nc)), dtype=np.float32)
        outs = {}
        for name in ("lbsg_gather", "lbsg_gather_noalloc"):
            x = torch.full((k, crop, crop, 1 + nc), float("nan"), device="cuda")
            y = torch.full((k, crop, crop), float("nan"), device="cuda")
            assert _call(name, field, h, w, yx, crop, cond, x, y, stream) == lbch.OK, lbch.lib().lbch_last_error().decode()
            torch.cuda.synchronize()
            outs[name] = (x.cpu(), y.cpu())
        (xa, ya), (xb, yb) = outs["lbsg_gather"], outs["lbsg_gather_noalloc"]
        assert torch.equal(xa, xb) and torch.equal(ya, yb)
        # and against the definition: periodic crops of the field
        f = field.cpu().numpy()
        q = k // 2
        rows = (yx[q, 0] + np.arange(crop)) % h
        cols = (yx[q, 1] + np.arange(crop)) % w
        assert np.array_equal(yb[q].numpy(), f[np.ix_(rows, cols)])
        assert np.array_equal(xb[q, 0, 0, 1:].numpy(), cond[q])


def test_noalloc_gather_rejects_more_crops_than_its_scratch_holds():
    import torch
    from paper_2501_03759_amd import lbch
    stream = torch.cuda.Stream()
    field = torch.zeros((32, 32), device="cuda")
    k = 16385
    yx = np.zeros((k, 2), dtype=np.int32)
    y = torch.empty((k, 2, 2), device="cuda")
    assert _call("lbsg_gather_noalloc", field, 32, 32, yx, 2, None, None, y, stream) == lbch.E_INVALID
    assert "16384" in lbch.lib().lbch_last_error().decode()
