"""Device allocations through the caller's allocator hooks (cmp_opts.dev_alloc
/ dev_free), through the C ABI (GPU): every allocation is returned, results
equal the oracle's."""

import numpy as np
import pytest
import torch

from paper_2104_14667_amd import synth
from paper_2104_14667_amd.composite import CMP_ENOMEM, CMP_TILED, Composite, CompositeError

from gpu_common import check_full, dev_of, expect_oracle, pinned_copy, say

pytestmark = pytest.mark.gpu

ALL = ("count", "sum", "max")


@pytest.mark.parametrize("layout", ["linear", "tiled"])
def test_torch_caching_allocator_hooks(layout):
    say("allocator hooks", layout)
    W, H = 160, 33
    A = synth.random_members(51, 6, H, W)
    dA = dev_of(A)
    hA = pinned_copy(torch.from_numpy(A))
    live, calls = {}, {"alloc": 0, "free": 0}

    def alloc(n):
        p = int(torch.cuda.caching_allocator_alloc(int(n), 0))
        assert p % 256 == 0
        live[p] = n
        calls["alloc"] += 1
        return p

    def free(p):
        assert p in live, "freed an address the hook did not return"
        del live[p]
        calls["free"] += 1
        torch.cuda.caching_allocator_delete(p)

    kw = dict(layout=CMP_TILED, tile_w=32, tile_h=8) if layout == "tiled" else {}
    with Composite(W, H, ("count", "sum"), 32, allocator=(alloc, free), verify_members=1,
                   pingpong=1, **kw) as c:
        c.add([hA[i] for i in range(3)], ids=[0, 1, 2])              # staging, fingerprints
        if layout == "linear":
            c.add_device([dA[i] for i in range(3, 6)], ids=[3, 4, 5])
            exp = A
        else:
            c.add([hA[i] for i in range(3, 6)], ids=[3, 4, 5])
            exp = A
        check_full(c, expect_oracle(exp, ("count", "sum"), 32))
        bins, over = c.histogram(8)
        assert bins.sum() + over == W * H
        assert calls["alloc"] >= 6 and live
    assert calls["free"] == calls["alloc"] and not live


def test_allocator_failure_reports_enomem():
    calls = {"n": 0}

    def alloc(n):
        calls["n"] += 1
        return 0                                                       # always fails

    with pytest.raises(CompositeError) as ei:
        Composite(64, 8, ALL, 32, allocator=(alloc, lambda p: None))
    assert ei.value.status == CMP_ENOMEM and calls["n"] == 1


def test_torch_allocator_shorthand():
    W, H = 96, 17
    A = synth.random_members(52, 4, H, W)
    dA = dev_of(A)
    with Composite(W, H, ALL, 16, allocator="torch", retain_members=1) as c:
        c.add_device([dA[i] for i in range(4)], ids=[0, 1, 2, 3])
        c.remove(ids=[2])
        check_full(c, expect_oracle(A[[0, 1, 3]], ALL, 16))
