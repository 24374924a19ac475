"""Overlap-class histogram and the tiled repack, through the C ABI (GPU)."""

import numpy as np
import pytest
import torch

import oracle
from paper_2104_14667_amd import synth
from paper_2104_14667_amd.composite import (Composite, composite_repack_tiled,
                                            composite_tiled_bytes)

from gpu_common import dev_of

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("W,H,n,bits", [(512, 512, 16, 16), (37, 11, 9, 32), (4097, 3, 300, 32),
                                        (8, 1, 5, 16), (1, 7, 2, 32)])
def test_histogram_matches_oracle(W, H, n, bits):
    stack = synth.random_members(W + n, n, H, W)
    count = oracle.accumulate(list(stack), shape=(H, W), outputs=("count",))["count"]
    dev = dev_of(stack)
    with Composite(W, H, ("count",), bits) as c:
        c.add_device([dev[i] for i in range(n)])
        for nbins in (n + 1, max(1, n // 2), 1, 10000):
            got, over = c.histogram(nbins)
            exp = oracle.overlap_histogram(np.minimum(count, nbins), nbins + 1)
            assert np.array_equal(got, exp[:nbins]), nbins
            assert over == int(exp[nbins]), nbins


def test_histogram_of_full_plain_workload():
    ens = synth.PLAIN_SMALL
    e = ens.elevation()
    stack = synth.members(e, ens.levels(), "mask")
    count = oracle.accumulate(list(stack), shape=e.shape, outputs=("count",))["count"]
    dev = dev_of(stack)
    with Composite(ens.W, ens.H, ("count",), 16) as c:
        c.add_device([dev[i] for i in range(ens.N)])
        got, over = c.histogram(ens.N + 1)
    assert np.array_equal(got, oracle.overlap_histogram(count, ens.N + 1)) and over == 0


def tiled_reference(a, tw, th):
    """The tiled layout written from its definition: pad to whole tiles with
    zeros, tiles in row-major tile order, each tile row-major."""
    H, W = a.shape
    nty, ntx = -(-H // th), -(-W // tw)
    p = np.zeros((nty * th, ntx * tw), dtype=a.dtype)
    p[:H, :W] = a
    out = []
    for ty in range(nty):
        for tx in range(ntx):
            out.append(p[ty * th:(ty + 1) * th, tx * tw:(tx + 1) * tw].ravel())
    return np.concatenate(out)


@pytest.mark.parametrize("W,H,tw,th", [(64, 64, 64, 64), (48, 33, 16, 7), (4096, 9, 128, 4),
                                       (160, 100, 32, 128), (16, 1, 16, 1), (100, 100, 64, 64),
                                       (1, 1, 16, 1), (4097, 3, 128, 2), (1856, 17, 64, 64),
                                       # tiles taller than one workgroup's 32 rows, the last
                                       # row group of each tile row partial
                                       (1100, 70, 16, 40), (2100, 45, 64, 33)])
def test_repack_matches_layout_definition(W, H, tw, th):
    n = 3
    stack = synth.random_members(W * H, n, H, W)
    src = dev_of(stack)
    tb = composite_tiled_bytes(W, H, tw, th)
    dst = torch.full((n, tb), 7, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    composite_repack_tiled(src, W * H, dst, tb, n, W, H, tw, th)
    torch.cuda.synchronize()
    got = dst.cpu().numpy()
    for i in range(n):
        assert np.array_equal(got[i], tiled_reference(stack[i], tw, th)), i
