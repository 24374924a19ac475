"""Member verification (cmp_opts.verify_members) through the C ABI (GPU): a
remove is accepted only for rasters whose fingerprint is held under their id,
and a refused remove changes nothing."""

import numpy as np
import pytest
import torch

from paper_2104_14667_amd import synth
from paper_2104_14667_amd.composite import (CMP_EINVAL, CMP_ENOTMEMBER, CMP_TILED, Composite,
                                            CompositeError)

from fingerprint_ref import colliding, tile, untile
from gpu_common import check_full, dev_of, expect_oracle, pinned_copy, say

pytestmark = pytest.mark.gpu

CS = ("count", "sum")


def _refused(fn, status=CMP_EINVAL):
    with pytest.raises(CompositeError) as ei:
        fn()
    assert ei.value.status == status


def _snapshot(c):
    return {k: c.read(k).copy() for k in c.outputs}


def _same(c, snap):
    for k, v in snap.items():
        assert np.array_equal(c.read(k), v), k


# sizes: ragged tail, one workgroup, several workgroups per member
@pytest.mark.parametrize("W,H", [(37, 29), (64, 16), (700, 900)])
def test_added_rasters_are_accepted_across_upload_paths(W, H):
    say("verify accept", W, H)
    A = synth.random_members(21, 5, H, W)
    dA = dev_of(A)
    hA = pinned_copy(torch.from_numpy(A))
    with Composite(W, H, CS, 32, verify_members=1) as c:
        c.add_device([dA[0], dA[1]], ids=[0, 1])
        c.add([hA[2], hA[3], hA[4]], ids=[2, 3, 4])
        check_full(c, expect_oracle(A, CS, 32))
        # device-added rasters removed from host copies and the other way round
        c.remove(maps=[hA[1]], ids=[1])
        c.remove(maps=[dA[3]], ids=[3], on_device=True)
        check_full(c, expect_oracle(A[[0, 2, 4]], CS, 32))
        c.remove(maps=[dA[0], dA[2], dA[4]], ids=[0, 2, 4], on_device=True)
        assert c.members() == 0
        assert not c.read("count").any() and not c.read("sum").any()


@pytest.mark.parametrize("on_device", [False, True])
def test_changed_raster_is_refused(on_device):
    W, H = 701, 899                            # 630199 px, a 7-byte tail
    say("verify refuse", on_device)
    A = synth.random_members(22, 3, H, W)
    dA = dev_of(A)
    hA = pinned_copy(torch.from_numpy(A))
    with Composite(W, H, CS, 32, verify_members=1) as c:
        c.add_device([dA[i] for i in range(3)], ids=[0, 1, 2])
        snap = _snapshot(c)
        npix = W * H
        for pos in (0, 17, npix // 2, (npix // 16) * 16 - 1, npix - 1):
            bad = A[1].copy().ravel()
            bad[pos] ^= 0x40
            bad = bad.reshape(H, W)
            m = dev_of(bad) if on_device else pinned_copy(torch.from_numpy(bad))
            _refused(lambda: c.remove(maps=[m], ids=[1], on_device=on_device))
            _same(c, snap)
            assert c.members() == 3
        # the right raster under the wrong id, and a mix with one bad raster
        m = dA[2] if on_device else hA[2]
        _refused(lambda: c.remove(maps=[m], ids=[1], on_device=on_device))
        ok = dA[0] if on_device else hA[0]
        _refused(lambda: c.remove(maps=[ok, m], ids=[0, 1], on_device=on_device))
        _same(c, snap)
        # the same rasters are still removable
        c.remove(maps=[dA[1]], ids=[1], on_device=True)
        check_full(c, expect_oracle(A[[0, 2]], CS, 32))


def test_anonymous_members_and_multiplicity():
    W, H = 130, 21
    A = synth.random_members(23, 3, H, W)
    dA = dev_of(A)
    with Composite(W, H, CS, 16, verify_members=1) as c:
        c.add_device([dA[0], dA[0], dA[1]])                  # no ids
        snap = _snapshot(c)
        _refused(lambda: c.remove(maps=[dA[2]], on_device=True))
        _same(c, snap)
        c.remove(maps=[dA[0]], on_device=True)
        c.remove(maps=[dA[0]], on_device=True)
        _refused(lambda: c.remove(maps=[dA[0]], on_device=True))
        check_full(c, expect_oracle(A[[1]], CS, 16))
        c.add_device([dA[2], dA[2]], ids=[5, 5])
        c.remove(maps=[dA[2], dA[2]], ids=[5, 5], on_device=True)
        _refused(lambda: c.remove(maps=[dA[2]], ids=[5], on_device=True), CMP_ENOTMEMBER)
        check_full(c, expect_oracle(A[[1]], CS, 16))


def test_retained_raster_changed_in_place_is_refused():
    W, H = 96, 40
    A = synth.random_members(24, 2, H, W)
    dA = dev_of(A)
    with Composite(W, H, ("count", "sum", "max"), 32, retain_members=1, verify_members=1) as c:
        c.add_device([dA[0], dA[1]], ids=[0, 1])
        snap = _snapshot(c)
        dA[1, 3, 5] ^= 1
        torch.cuda.synchronize()
        _refused(lambda: c.remove(ids=[1]))
        _same(c, snap)
        dA[1, 3, 5] ^= 1                        # restored: max is rebuilt from it
        torch.cuda.synchronize()
        c.remove(ids=[0])
        check_full(c, expect_oracle(A[[1]], ("count", "sum", "max"), 32))


@pytest.mark.parametrize("layout", ["linear", "tiled"])
def test_fingerprint_is_the_documented_sum(layout):
    """A raster built to collide under the documented definition is accepted
    (the fingerprint detects mistakes, not forgeries); the same change without
    its compensating word is refused.  The two words are far apart (a wrong
    weight or word index anywhere between them shows).  In a tiled context the
    fingerprint is over the tiled layout, so the words are chosen there."""
    W, H, tw, th = 256, 37, 64, 64                # 9472 px; tiled: 4 tiles of 64x64
    A = synth.random_members(25, 1, H, W)[0].copy()
    if layout == "linear":
        flat = A.ravel().copy()
        j, k = 3, flat.size // 4 - 1              # first row, x 12..15; last word
        to_raster = lambda f: f.reshape(H, W)
    else:
        flat = tile(A, tw, th)
        j, k = 3, (36 * tw + 60) // 4            # tile 0: row 0 x 12..15; row 36 x 60..63
        to_raster = lambda f: untile(f, W, H, tw, th)
    flat[4 * j:4 * j + 4] = 0                     # word j zero
    flat[4 * k:4 * k + 4] = 255                   # word k all ones
    A = to_raster(flat)
    Bf = colliding(flat, j, k)
    Cf = Bf.copy()
    Cf[4 * k:4 * k + 4] = 255                     # uncompensated change
    B, C = to_raster(Bf), to_raster(Cf)
    assert not np.array_equal(A, B) and not np.array_equal(A, C)
    kw = {"layout": CMP_TILED, "tile_w": tw, "tile_h": th} if layout == "tiled" else {}
    hA = pinned_copy(torch.from_numpy(A))
    hB = pinned_copy(torch.from_numpy(B))
    hC = pinned_copy(torch.from_numpy(C))
    with Composite(W, H, CS, 32, verify_members=1, **kw) as c:
        c.add([hA], ids=[9])
        _refused(lambda: c.remove(maps=[hC], ids=[9]))
        assert c.members() == 1
        c.remove(maps=[hB], ids=[9])
        assert c.members() == 0
