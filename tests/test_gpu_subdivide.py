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
