"""HIP compositing path against the oracle, through the C ABI (GPU).

Small and ragged cases compare every pixel with the oracle; full-size
workloads compare every pixel with the closed form and sampled pixels with
the oracle.  Tolerance is zero everywhere: the outputs are integers."""

import numpy as np
import pytest
import torch

import oracle
from paper_2104_14667_amd import synth
from paper_2104_14667_amd.composite import (CMP_ENOTMEMBER, CMP_ERANGE, CMP_EINVAL,
                                            CMP_EUNSUPPORTED, CMP_TILED, Composite,
                                            CompositeError)

from gpu_common import (check_closed_form_and_samples, check_full, dev_of, device_members,
                        elevation_of, expect_oracle, pinned_copy, say)

pytestmark = pytest.mark.gpu

ALL = ("count", "sum", "max")


def _random_stack(seed, n, H, W):
    return synth.random_members(seed, n, H, W)


# ---------------------------------------------------------------- small, exact

def test_plain_small_resident_and_streamed():
    ens = synth.PLAIN_SMALL
    say("plain-small", ens.N, ens.H, ens.W)
    e = elevation_of(ens)
    lv = ens.levels()
    stack = synth.members(e, lv, "mask")
    exp = expect_oracle(stack, ("count",), 16)
    dev = dev_of(stack)
    with Composite(ens.W, ens.H, ("count",), 16) as c:
        c.add_device([dev[i] for i in range(ens.N)])
        check_full(c, exp)
    host = pinned_copy(torch.from_numpy(stack))
    for nbuf in (1, 2):
        with Composite(ens.W, ens.H, ("count",), 16, nbuf=nbuf, chunk_depth=3) as c:
            c.add([host[i] for i in range(ens.N)])
            check_full(c, exp)


SHAPES = [(1, 1), (15, 1), (1, 17), (17, 3), (33, 65), (4095, 3), (4097, 5), (64, 48), (512, 7)]


@pytest.mark.parametrize("W,H", SHAPES)
@pytest.mark.parametrize("count_bits", [16, 32])
def test_ragged_resident_unaligned(W, H, count_bits):
    # members are slices of one (N, H, W) tensor: for odd W*H every member
    # but the first starts at an address that is not 16-byte aligned
    for n in (0, 1, 3, 7):
        say("ragged resident", W, H, n, count_bits)
        stack = _random_stack(W * 1000 + H + n, n, H, W)
        exp = expect_oracle(stack, ALL, count_bits)
        dev = dev_of(stack)
        with Composite(W, H, ALL, count_bits) as c:
            c.add_device([dev[i] for i in range(n)])
            check_full(c, exp)
            assert c.members() == n


@pytest.mark.parametrize("W,H", SHAPES)
@pytest.mark.parametrize("nbuf,depth", [(1, 1), (2, 1), (2, 3), (1, 8), (2, 8)])
def test_ragged_streamed(W, H, nbuf, depth):
    n = 11
    say("ragged streamed", W, H, nbuf, depth)
    stack = _random_stack(W * 7 + H * 3 + depth, n, H, W)
    exp = expect_oracle(stack, ALL, 32)
    host = pinned_copy(torch.from_numpy(stack))
    for paced, streams in ((1, 0), (0, 0), (0, 2)):
        if streams == 2 and nbuf != 2:
            continue
        with Composite(W, H, ALL, 32, nbuf=nbuf, chunk_depth=depth, host_paced=paced,
                       copy_streams=streams) as c:
            c.add([host[i] for i in range(n)])
            check_full(c, exp)


def test_streamed_from_pageable_numpy():
    W, H, n = 100, 37, 9
    stack = _random_stack(5, n, H, W)
    exp = expect_oracle(stack, ALL, 32)
    for nbuf in (1, 2):
        with Composite(W, H, ALL, 32, chunk_depth=4, nbuf=nbuf, pageable_host=1) as c:
            c.add([stack[i] for i in range(n)])
            check_full(c, exp)
        with Composite(W, H, ("count", "sum"), 32, chunk_depth=2, nbuf=nbuf,
                       pageable_host=1) as c:
            c.add([stack[i] for i in range(n)])
            c.remove([stack[i] for i in range(3, n)])
            check_full(c, expect_oracle(stack[:3], ("count", "sum"), 32))


@pytest.mark.parametrize("depth", [1, 3, 8, 255, 256])
def test_chunking_and_group_boundaries(depth):
    # 300 members cross the 256-member group of the kernels' 16-bit lanes,
    # with values up to 255 the sum lanes are exercised at their limit
    W, H, n = 64, 24, 300
    say("chunking", depth)
    stack = _random_stack(depth, n, H, W)
    stack[:, 0, :] = 255
    exp = expect_oracle(stack, ALL, 32)
    dev = dev_of(stack)
    with Composite(W, H, ALL, 32) as c:
        c.add_device([dev[i] for i in range(n)])
        check_full(c, exp)
    host = pinned_copy(torch.from_numpy(stack))
    with Composite(W, H, ALL, 32, chunk_depth=depth) as c:
        c.add([host[i] for i in range(n)])
        check_full(c, exp)
    # several calls accumulate into the same composite
    with Composite(W, H, ALL, 32, chunk_depth=depth) as c:
        c.add_device([dev[i] for i in range(0, 100)])
        c.add([host[i] for i in range(100, 250)])
        c.add_device([dev[i] for i in range(250, n)])
        check_full(c, exp)


@pytest.mark.parametrize("W,H,tw,th", [(64, 64, 64, 64), (96, 50, 32, 16), (4096, 9, 128, 4),
                                       (48, 33, 16, 7), (512, 300, 64, 64)])
def test_tiled_layout(W, H, tw, th):
    n = 13
    stack = _random_stack(W + H + tw, n, H, W)
    exp = expect_oracle(stack, ALL, 32)
    host = pinned_copy(torch.from_numpy(stack))
    for nbuf in (1, 2):
        with Composite(W, H, ALL, 32, nbuf=nbuf, chunk_depth=4, layout=CMP_TILED,
                       tile_w=tw, tile_h=th) as c:
            c.add([host[i] for i in range(n)])
            check_full(c, exp)


def test_poisoned_staging_stays_exact():
    W, H, n = 256, 40, 29
    stack = _random_stack(9, n, H, W)
    exp = expect_oracle(stack, ALL, 32)
    host = pinned_copy(torch.from_numpy(stack))
    for layout in (0, CMP_TILED):
        for paced in (1, 0):
            with Composite(W, H, ALL, 32, chunk_depth=3, debug_poison=1, layout=layout,
                           host_paced=paced) as c:
                c.add([host[i] for i in range(n)])
                check_full(c, exp)


# ---------------------------------------------------------------- add / remove

def test_add_then_remove_restores():
    W, H = 130, 21
    A = _random_stack(1, 6, H, W)
    B = _random_stack(2, 5, H, W)
    dA = dev_of(A)
    dB = dev_of(B)
    hB = pinned_copy(torch.from_numpy(B))
    with Composite(W, H, ALL, 32, retain_members=1) as c:
        c.add_device([dA[i] for i in range(6)], ids=list(range(6)))
        before = {k: c.read(k).copy() for k in ALL}
        c.add_device([dB[i] for i in range(5)], ids=list(range(10, 15)))
        c.remove(ids=list(range(10, 15)))            # retained rasters, max rebuilt
        for k in ALL:
            assert np.array_equal(c.read(k), before[k]), k
        assert c.members() == 6
        # remove a subset by id with the device rasters given explicitly
        c.remove(maps=[dA[1], dA[4]], ids=[1, 4], on_device=True)
        exp = expect_oracle(A[[0, 2, 3, 5]], ALL, 32)
        check_full(c, exp)
    with Composite(W, H, ("count", "sum"), 16) as c:
        c.add_device([dA[i] for i in range(6)])
        c.add([hB[i] for i in range(5)])
        c.remove(maps=[hB[i] for i in range(5)])      # streamed removal
        check_full(c, expect_oracle(A, ("count", "sum"), 16))


def test_remove_errors_leave_state_unchanged():
    W, H = 48, 10
    A = _random_stack(3, 4, H, W)
    dA = dev_of(A)
    hA = pinned_copy(torch.from_numpy(A))
    with Composite(W, H, ALL, 32, retain_members=1) as c:
        c.add_device([dA[i] for i in range(4)], ids=[7, 7, 8, 9])
        before = {k: c.read(k).copy() for k in ALL}
        with pytest.raises(CompositeError) as ei:
            c.remove(ids=[7, 7, 7])
        assert ei.value.status == CMP_ENOTMEMBER
        with pytest.raises(CompositeError) as ei:
            c.remove(ids=[42])
        assert ei.value.status == CMP_ENOTMEMBER
        for k in ALL:
            assert np.array_equal(c.read(k), before[k])
        assert c.members() == 4
        c.remove(ids=[7])                                # one of two copies
        check_full(c, expect_oracle(A[[1, 2, 3]], ALL, 32))
    with Composite(W, H, ALL, 32) as c:                  # max without retained members
        c.add([hA[i] for i in range(4)])
        with pytest.raises(CompositeError) as ei:
            c.remove(maps=[hA[0]])
        assert ei.value.status == CMP_EUNSUPPORTED
        check_full(c, expect_oracle(A, ALL, 32))


def test_range_guard_refuses_overflow():
    W, H = 16, 1
    m = torch.full((H, W), 255, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    with Composite(W, H, ("count",), 16) as c:
        c.add_device([m] * 65535)
        with pytest.raises(CompositeError) as ei:
            c.add_device([m])
        assert ei.value.status == CMP_ERANGE
        assert c.members() == 65535
        assert np.all(c.read("count") == 65535)


def test_read_windows_and_device_destination():
    W, H, n = 300, 77, 5
    stack = _random_stack(4, n, H, W)
    full = oracle.narrow(oracle.accumulate(list(stack), shape=(H, W)), 32)
    dev = dev_of(stack)
    with Composite(W, H, ALL, 32) as c:
        c.add_device([dev[i] for i in range(n)])
        for (x0, y0, w, h) in [(0, 0, W, H), (3, 5, 17, 9), (W - 1, H - 1, 1, 1), (0, 10, W, 1)]:
            for k in ALL:
                got = c.read(k, (x0, y0, w, h))
                assert np.array_equal(got, oracle.window(full[k], x0, y0, w, h)), (k, x0, y0)
                dst = torch.zeros((h, w + 3), dtype={"max": torch.uint8}.get(k, torch.int32),
                                  device="cuda")
                torch.cuda.synchronize()
                c.read_device(k, dst, (x0, y0, w, h), pitch_bytes=dst.stride(0) * dst.element_size())
                torch.cuda.synchronize()
                gd = dst[:, :w].cpu().numpy().view(got.dtype)
                assert np.array_equal(gd, got)
        with pytest.raises(CompositeError) as ei:
            c.read("count", (W - 2, 0, 3, 1))
        assert ei.value.status == CMP_EINVAL
        # page-locked destination written by the copy engine directly
        for k in ALL:
            dt = {"max": torch.uint8}.get(k, torch.int32)
            pin = torch.zeros((H - 3, W - 5), dtype=dt, pin_memory=True)
            arr = pin.numpy().view(full[k].dtype)
            c.read(k, (2, 1, W - 5, H - 3), out=arr, pinned=True)
            assert np.array_equal(arr, oracle.window(full[k], 2, 1, W - 5, H - 3))


@pytest.mark.parametrize("count_bits", [16, 32])
def test_read_device_windows_vector_and_element_paths(count_bits):
    """Windows read into device memory: 16-byte moves where every source and
    destination row starts on a 16-byte boundary (with the row's ragged end
    element by element), one element per thread otherwise."""
    W, H, n = 320, 40, 4
    stack = _random_stack(9, n, H, W)
    full = oracle.narrow(oracle.accumulate(list(stack), shape=(H, W)), count_bits)
    dev = dev_of(stack)
    elem = {"count": count_bits // 8, "sum": 4, "max": 1}
    with Composite(W, H, ALL, count_bits) as c:
        c.add_device([dev[i] for i in range(n)])
        for (x0, y0, w, h) in [(0, 0, W, H), (16, 3, 37, 5), (4, 2, 50, 7), (5, 1, 19, 3), (304, 39, 16, 1)]:
            for k in ALL:
                e = elem[k]
                want = oracle.window(full[k], x0, y0, w, h)
                for pitch in (-(-w * e // 64) * 64, w * e + e):   # aligned rows; rows off 16 B
                    buf = torch.full((h * pitch + 64,), 0x5A, dtype=torch.uint8, device="cuda")
                    torch.cuda.synchronize()
                    c.read_device(k, buf, (x0, y0, w, h), pitch_bytes=pitch)
                    torch.cuda.synchronize()
                    b = buf.cpu().numpy()
                    got = np.stack([b[r * pitch:r * pitch + w * e].view(want.dtype) for r in range(h)])
                    assert np.array_equal(got, want), (k, x0, y0, w, h, pitch)
                    # nothing written between rows or after the last one
                    for r in range(h):
                        assert (b[r * pitch + w * e:(r + 1) * pitch] == 0x5A).all(), (k, r, pitch)
                    assert (b[h * pitch:] == 0x5A).all()


def test_clear_forgets_members():
    W, H = 32, 32
    stack = _random_stack(8, 3, H, W)
    dev = dev_of(stack)
    with Composite(W, H, ALL, 32) as c:
        c.add_device([dev[i] for i in range(3)])
        c.clear()
        assert c.members() == 0
        for k in ALL:
            assert not c.read(k).any()


# ---------------------------------------------------------------- full size

def test_full_streamed_mask_4096_n256():
    ens = synth.STREAMED
    say("full streamed", ens.name)
    e = elevation_of(ens)
    lv = ens.levels()
    host = pinned_copy(device_members(ens, e, lv))
    for layout in (0, CMP_TILED):
        with Composite(ens.W, ens.H, ens.outputs, ens.count_bits, nbuf=2, chunk_depth=8,
                       layout=layout) as c:
            c.add([host[i] for i in range(ens.N)])
            check_closed_form_and_samples(c, ens, e, lv)
    del host


@pytest.mark.parametrize("mode", ["resident", "streamed"])
def test_full_depth_8192_n128(mode):
    ens = synth.DEPTH
    say("full depth", ens.name, mode)
    e = elevation_of(ens)
    lv = ens.levels()
    dev = device_members(ens, e, lv)
    with Composite(ens.W, ens.H, ens.outputs, ens.count_bits, chunk_depth=8) as c:
        if mode == "resident":
            c.add_device([dev[i] for i in range(ens.N)])
        else:
            host = pinned_copy(dev)
            del dev
            torch.cuda.empty_cache()
            c.add([host[i] for i in range(ens.N)])
        check_closed_form_and_samples(c, ens, e, lv)


def test_full_depth_remove_half_and_reads():
    """The resident depth workload (128 x 8192x8192, count+sum+max) with
    retained members: removing 64 of them (count and sum decremented, max
    rebuilt from the 64 kept) leaves the composite of the rest, checked per
    pixel against the closed form and at sampled pixels against the oracle;
    windows read to pinned host and to device memory equal the full read."""
    ens = synth.DEPTH
    say("full depth remove", ens.name)
    e = elevation_of(ens)
    lv = ens.levels()
    dev = device_members(ens, e, lv)
    n = len(lv)
    ids = list(range(n))
    with Composite(ens.W, ens.H, ens.outputs, ens.count_bits, retain_members=1) as c:
        c.add_device([dev[i] for i in range(n)], ids)
        c.remove(None, ids[: n // 2])
        assert c.members() == n - n // 2
        check_closed_form_and_samples(c, ens, e, lv[n // 2:])
        full = c.read("count")
        x0, y0, v = ens.W - 1024 - 3, 777, 1024
        win = torch.empty((v, v), dtype=torch.int32, pin_memory=True)
        c.read("count", window=(x0, y0, v, v), out=win.numpy().view(np.uint32), pinned=True)
        assert np.array_equal(win.numpy().view(np.uint32), full[y0:y0 + v, x0:x0 + v])
        dwin = torch.empty((v, v + 5), dtype=torch.int32, device="cuda:0")
        c.read_device("count", dwin, window=(x0, y0, v, v), pitch_bytes=4 * (v + 5))
        got = dwin.cpu().numpy().view(np.uint32)[:, :v]
        assert np.array_equal(got, full[y0:y0 + v, x0:x0 + v])


def test_repeated_and_alternating_member_tables():
    """Calls that repeat the previous call's rasters reuse its device table;
    alternating and repeated tables give the oracle's composite."""
    W, H = 200, 9
    A = _random_stack(41, 3, H, W)
    B = _random_stack(42, 2, H, W)
    dA, dB = dev_of(A), dev_of(B)
    a = [dA[i] for i in range(3)]
    b = [dB[i] for i in range(2)]
    with Composite(W, H, ALL, 32, retain_members=1) as c:
        for maps in (a, a, b, a, b, b, a[:2], a[:2]):
            c.add_device(maps)
        stack = np.concatenate([A, A, B, A, B, B, A[:2], A[:2]])
        check_full(c, expect_oracle(stack, ALL, 32))
        c.remove(maps=b, on_device=True)
        c.remove(maps=b, on_device=True)
        check_full(c, expect_oracle(np.concatenate([A, A, B, A, A[:2], A[:2]]), ("count", "sum"), 32)
                   | {"max": expect_oracle(stack, ("max",), 32)["max"]})
