"""Spatial subdivision (row bands) against the oracle and the single-context
composite (GPU)."""

import numpy as np
import pytest
import torch

import oracle
from paper_2104_14667_amd import synth
from paper_2104_14667_amd.subdivide import composite_banded

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
