"""Spatial subdivision (row bands) against the oracle and the single-context
composite (GPU)."""

import numpy as np
import pytest
import torch

import oracle
from paper_2104_14667_amd import synth
from paper_2104_14667_amd.subdivide import composite_banded

from gpu_common import say

pytestmark = pytest.mark.gpu

ALL = ("count", "sum", "max")


@pytest.mark.parametrize("band_rows", [1, 7, 64, 1000])
def test_banded_equals_oracle(band_rows):
    W, H, n = 300, 130, 13
    stack = synth.random_members(band_rows, n, H, W)
    exp = oracle.narrow(oracle.accumulate(list(stack), shape=(H, W)), 32)
    host = torch.from_numpy(stack).pin_memory()
    got = composite_banded([host[i] for i in range(n)], W, H, band_rows, ALL, 32, chunk_depth=4)
    for k in ALL:
        assert np.array_equal(got[k], exp[k]), k


def test_banded_pageable_sources_u16():
    W, H, n = 64, 50, 9
    stack = synth.random_members(3, n, H, W)
    exp = oracle.narrow(oracle.accumulate(list(stack), shape=(H, W), outputs=("count",)), 16)
    got = composite_banded([stack[i] for i in range(n)], W, H, 16, ("count",), 16,
                           pageable_host=1, chunk_depth=2)
    assert np.array_equal(got["count"], exp["count"])


def test_banded_into_pinned_outputs_reusing_contexts():
    """Six bands of 20 rows and a ragged one of 10: the two contexts of the
    full band are used in turn, each cleared and reused twice while the other
    band's read-back runs, and the last band gets its own.  The outputs are
    page-locked, prefilled with garbage, and written by the copy engine
    directly; a second call into the same outputs gives the same."""
    W, H, n = 200, 130, 11
    stack = synth.random_members(40, n, H, W)
    exp = oracle.narrow(oracle.accumulate(list(stack), shape=(H, W)), 32)
    host = torch.from_numpy(stack).pin_memory()
    out = {"count": torch.empty((H, W), dtype=torch.int32, pin_memory=True).numpy().view(np.uint32),
           "sum": torch.empty((H, W), dtype=torch.int32, pin_memory=True).numpy().view(np.uint32),
           "max": torch.empty((H, W), dtype=torch.uint8, pin_memory=True).numpy()}
    for rep in range(2):
        for a in out.values():
            a.fill(0xAB)
        got = composite_banded([host[i] for i in range(n)], W, H, 20, ALL, 32, out=out,
                               pinned=True, chunk_depth=3)
        for k in ALL:
            assert got[k] is out[k]
            assert np.array_equal(got[k], exp[k]), (rep, k)
    with pytest.raises(ValueError):
        composite_banded([host[i] for i in range(n)], W, H, 48, ("count",), 32,
                         out={"count": np.empty((H, W), dtype=np.uint16)})


def _hashed_rows(W, y0, y1):
    """Hashed elevation of rows [y0, y1) of a W-wide raster, on the device."""
    xx = torch.arange(W, device="cuda", dtype=torch.int64)[None, :]
    yy = torch.arange(y0, y1, device="cuda", dtype=torch.int64)[:, None]
    return ((((xx * 2654435761 + yy * 40503 + (xx ^ yy) * 97) & 0xFFFFFFFF) >> 24)
            .to(torch.uint8))


def test_banded_raster_beyond_one_context():
    """65536 x 65600 pixels (2^32 + 2^22), more than one context accepts:
    two members (a mask and a depth map, 4.3 GB each in pinned host memory)
    composited in four bands of 16384 rows and one of 64.  Every pixel of
    count (u16) and max is compared on the device with the members' closed
    form, and sampled pixels, the last ones included, with the oracle."""
    from paper_2104_14667_amd.composite import Composite, CompositeError
    W, H, LM, LD = 65536, 65600, 120, 170
    npix = W * H
    assert npix > 2**32 - 16
    with pytest.raises(CompositeError):
        Composite(W, H, ("count",), 16)
    say("banded beyond one context", W, H)
    host = [torch.empty(npix, dtype=torch.uint8, pin_memory=True) for _ in range(2)]
    for y0 in range(0, H, 4096):
        y1 = min(H, y0 + 4096)
        e = _hashed_rows(W, y0, y1).to(torch.int16)
        host[0][y0 * W:y1 * W].copy_((e < LM).to(torch.uint8).reshape(-1))
        host[1][y0 * W:y1 * W].copy_((LD - e).clamp(0, 255).to(torch.uint8).reshape(-1))
    torch.cuda.synchronize()
    got = composite_banded(host, W, H, 16384, ("count", "max"), 16, chunk_depth=2)
    for y0 in range(0, H, 4096):
        y1 = min(H, y0 + 4096)
        e = _hashed_rows(W, y0, y1).to(torch.int16)
        m, d = (e < LM).to(torch.int32), (LD - e).clamp(0, 255).to(torch.int32)
        cnt = torch.from_numpy(got["count"][y0:y1].astype(np.int32)).cuda()
        mx = torch.from_numpy(got["max"][y0:y1]).cuda().to(torch.int32)
        assert torch.equal(cnt, m + (d > 0).to(torch.int32)), y0
        assert torch.equal(mx, torch.maximum(m, d)), y0
    rng = np.random.default_rng(11)
    idx = np.concatenate([rng.integers(0, npix, 500), np.arange(npix - 20, npix), [0, W - 1, W]])
    ys, xs = idx // W, idx % W
    e = ((((xs * 2654435761 + ys * 40503 + (xs ^ ys) * 97) & 0xFFFFFFFF) >> 24)
         .astype(np.int16))
    ms = [(e < LM).astype(np.uint8), np.clip(LD - e, 0, 255).astype(np.uint8)]
    exp = oracle.narrow(oracle.accumulate(ms, shape=e.shape, outputs=("count", "max")), 16)
    assert np.array_equal(got["count"].reshape(-1)[idx], exp["count"])
    assert np.array_equal(got["max"].reshape(-1)[idx], exp["max"])
