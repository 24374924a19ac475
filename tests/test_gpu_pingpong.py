"""Two accumulators used in turn (cmp_opts.pingpong) and tiled device-resident
members, through the C ABI (GPU), against the oracle.  Tolerance zero."""

import numpy as np
import pytest
import torch

from paper_2104_14667_amd import synth
from paper_2104_14667_amd.composite import (CMP_EINVAL, CMP_TILED, Composite, CompositeError,
                                            composite_repack_tiled, composite_tiled_bytes)

from gpu_common import check_full, dev_of, expect_oracle, pinned_copy, say

pytestmark = pytest.mark.gpu

ALL = ("count", "sum", "max")


def tiled_copies(A: np.ndarray, tw: int, th: int) -> torch.Tensor:
    """Device copies of the rasters of A in the tiled layout, one per row."""
    n, H, W = A.shape
    tb = composite_tiled_bytes(W, H, tw, th)
    src = dev_of(A.reshape(n, -1))
    dst = torch.zeros((n, tb), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    composite_repack_tiled(src, H * W, dst, tb, n, W, H, tw, th)
    torch.cuda.synchronize()
    return dst


# linear with a ragged 16-pixel tail; tiled with partial edge tiles
@pytest.mark.parametrize("layout,W,H", [("linear", 130, 21), ("tiled", 144, 37)])
@pytest.mark.parametrize("count_bits", [16, 32])
@pytest.mark.parametrize("pingpong", [0, 1])
def test_accumulators_in_turn_equal_in_place(layout, W, H, count_bits, pingpong):
    say("pingpong", layout, W, H, count_bits, pingpong)
    A = synth.random_members(31, 7, H, W)
    B = synth.random_members(32, 5, H, W)
    kw = dict(retain_members=1, pingpong=pingpong, chunk_depth=3)
    if layout == "tiled":
        kw.update(layout=CMP_TILED, tile_w=32, tile_h=8)
        dA = tiled_copies(A, 32, 8)
    else:
        dA = dev_of(A)
    hB = pinned_copy(torch.from_numpy(B))
    outs = ALL if count_bits == 32 else ("count", "max")
    with Composite(W, H, outs, count_bits, **kw) as c:
        c.add_device([dA[i] for i in range(7)], ids=list(range(7)))
        check_full(c, expect_oracle(A, outs, count_bits))
        c.add_device([dA[i] for i in range(3)], ids=[0, 1, 2])       # duplicates
        check_full(c, expect_oracle(np.concatenate([A, A[:3]]), outs, count_bits))
        c.remove(ids=[0, 1, 2, 5])                                    # retained rasters, max rebuilt
        keep = A[[0, 1, 2, 3, 4, 6]]
        check_full(c, expect_oracle(keep, outs, count_bits))
    # streamed adds and removes (no max: host rasters cannot rebuild it)
    so = ("count", "sum") if count_bits == 32 else ("count",)
    kw.pop("retain_members")
    with Composite(W, H, so, count_bits, **kw) as c:
        c.add([hB[i] for i in range(5)])
        c.add_device([dA[i] for i in range(7)])
        check_full(c, expect_oracle(np.concatenate([B, A]), so, count_bits))
        c.remove(maps=[hB[1], hB[3]])
        check_full(c, expect_oracle(np.concatenate([B[[0, 2, 4]], A]), so, count_bits))
        c.clear()
        c.add([hB[0]])
        check_full(c, expect_oracle(B[:1], so, count_bits))


def test_tiled_device_members_and_verification():
    """A tiled context takes device rasters in the tiled layout; fingerprints
    are over the tiled bytes, so a raster added from host memory is removable
    as its tiled device copy and the other way round."""
    W, H = 160, 50
    A = synth.random_members(33, 4, H, W)
    dA = tiled_copies(A, 64, 16)
    hA = pinned_copy(torch.from_numpy(A))
    with Composite(W, H, ("count", "sum"), 32, layout=CMP_TILED, tile_w=64, tile_h=16,
                   verify_members=1, pingpong=1) as c:
        c.add([hA[0], hA[1]], ids=[0, 1])
        c.add_device([dA[2], dA[3]], ids=[2, 3])
        check_full(c, expect_oracle(A, ("count", "sum"), 32))
        c.remove(maps=[dA[0]], ids=[0], on_device=True)               # added from host
        c.remove(maps=[hA[3]], ids=[3])                               # added as tiled device copy
        check_full(c, expect_oracle(A[[1, 2]], ("count", "sum"), 32))
        with pytest.raises(CompositeError) as ei:
            c.remove(maps=[dA[2]], ids=[1], on_device=True)           # wrong id
        assert ei.value.status == CMP_EINVAL
        check_full(c, expect_oracle(A[[1, 2]], ("count", "sum"), 32))


def test_pingpong_full_depth_workload_sampled():
    """The depth workload at full size through both accumulators, against the
    closed form (every pixel) and sampled oracle pixels."""
    from gpu_common import check_closed_form_and_samples, device_members, elevation_of
    ens = synth.DEPTH
    e = elevation_of(ens)
    lv = ens.levels()
    dev = device_members(ens, e, lv)
    with Composite(ens.W, ens.H, ens.outputs, ens.count_bits, pingpong=1) as c:
        c.add_device([dev[i] for i in range(ens.N)])
        check_closed_form_and_samples(c, ens, e, lv)
        c.clear()                    # clears the accumulators the first add wrote
        c.add_device([dev[i] for i in range(ens.N)])
        check_closed_form_and_samples(c, ens, e, lv)
