"""Batched crop requests against a device pool, through the C ABI (GPU).

Every output is compared with the oracle's batched composite (small pools,
every pixel) or with the closed form per request plus sampled pixels of the
oracle (the full pool of 2048 maps of 2048x2048).  Tolerance zero."""

import numpy as np
import pytest
import torch

import oracle
from paper_2104_14667_amd import synth
from paper_2104_14667_amd.composite import (CMP_BATCH_MATRIX, CMP_BATCH_PER_REQUEST,
                                            CMP_BATCH_PERSISTENT, CMP_BATCH_SHARED, CMP_EINVAL,
                                            CMP_ORDER_COST,
                                            CMP_ORDER_ROWS, CompositeError, Pool, make_tune)
from paper_2104_14667_amd.tune import autotune

from gpu_common import say

pytestmark = pytest.mark.gpu


def _pool_tensor(stack: np.ndarray):
    """Contiguous device copy with 64 bytes of slack after the last raster."""
    P, H, W = stack.shape
    buf = torch.zeros(P * H * W + 64, dtype=torch.uint8, device="cuda")
    buf[: P * H * W].copy_(torch.from_numpy(stack.reshape(-1)))
    torch.cuda.synchronize()
    return buf


def _outs(reqs, pad=0):
    for r in reqs:
        r["out"] = torch.full((r["h"], r["w"] + pad), -1, dtype=torch.int32, device="cuda")
        r["pitch"] = r["w"] + pad
    torch.cuda.synchronize()


def _got(r):
    return r["out"][:, : r["w"]].cpu().numpy().view(np.uint32).astype(np.int64)


TUNES = [make_tune(CMP_BATCH_PERSISTENT, 64, 1, 0, CMP_ORDER_COST, 1),
         make_tune(CMP_BATCH_PERSISTENT, 1024, 8, 1, CMP_ORDER_COST, 0),
         make_tune(CMP_BATCH_PERSISTENT, 256, 3, 1, CMP_ORDER_ROWS, 0),
         make_tune(CMP_BATCH_PERSISTENT, 64, 16, 1, CMP_ORDER_ROWS, 1),
         make_tune(CMP_BATCH_PER_REQUEST, stream_loads=1),
         make_tune(CMP_BATCH_PER_REQUEST, stream_loads=0)]


def _small_case(seed):
    rng = np.random.default_rng(seed)
    P, H, W = 37, 45, 77
    stack = synth.random_members(seed, P, H, W)
    reqs = [dict(ids=[], x0=0, y0=0, w=W, h=H),                       # empty set
            dict(ids=[3], x0=W - 1, y0=H - 1, w=1, h=1),               # last pixel
            dict(ids=[5, 5, 5], x0=1, y0=2, w=17, h=3),                 # repeats
            dict(ids=list(range(P)), x0=0, y0=0, w=W, h=H)]             # everything
    for _ in range(12):
        w = int(rng.integers(1, W + 1))
        h = int(rng.integers(1, H + 1))
        n = int(rng.integers(0, 300))
        reqs.append(dict(ids=rng.integers(0, P, n).tolist(), x0=int(rng.integers(0, W - w + 1)),
                         y0=int(rng.integers(0, H - h + 1)), w=w, h=h))
    return stack, reqs


@pytest.mark.parametrize("ti", range(len(TUNES)))
def test_small_pool_all_tunes(ti):
    stack, reqs = _small_case(ti + 1)
    P, H, W = stack.shape
    exp = oracle.batch(stack, reqs)
    buf = _pool_tensor(stack)
    with Pool(buf, P, W, H, H * W, buf.numel()) as pool:
        for pad in (0, 5):
            _outs(reqs, pad)
            pool.run(reqs, TUNES[ti])
            for k, (r, e) in enumerate(zip(reqs, exp)):
                assert np.array_equal(_got(r), e), f"request {k}"
            # a second run of the same pool and tune (graph replay) is identical
            _outs(reqs, pad)
            pool.run(reqs, TUNES[ti])
            for k, (r, e) in enumerate(zip(reqs, exp)):
                assert np.array_equal(_got(r), e), f"replay, request {k}"


def test_varying_batches_reuse_one_graph():
    stack, reqs = _small_case(9)
    P, H, W = stack.shape
    buf = _pool_tensor(stack)
    tune = make_tune(CMP_BATCH_PERSISTENT, 128, 2, 1)
    with Pool(buf, P, W, H, H * W, buf.numel()) as pool:
        for k in range(1, len(reqs) + 1, 3):
            sub = [dict(r) for r in reqs[:k]]
            _outs(sub)
            pool.run(sub, tune)
            for r, e in zip(sub, oracle.batch(stack, sub)):
                assert np.array_equal(_got(r), e)
            torch.cuda.synchronize()          # eager work between replays


def test_invalid_requests_launch_nothing():
    stack, reqs = _small_case(4)
    P, H, W = stack.shape
    buf = _pool_tensor(stack)
    with Pool(buf, P, W, H, H * W, buf.numel()) as pool:
        good = [dict(reqs[2])]
        bads = [dict(good[0], ids=[P]), dict(good[0], ids=[-1]), dict(good[0], x0=W - 3, w=4),
                dict(good[0], h=0)]
        for bad in bads:
            batch = [dict(good[0]), bad]
            _outs(batch)
            with pytest.raises(CompositeError) as ei:
                pool.run(batch)
            assert ei.value.status == CMP_EINVAL
            assert (batch[0]["out"] == -1).all()      # nothing ran
        bad = dict(good[0])
        _outs([bad])
        bad["pitch"] = bad["w"] - 1
        with pytest.raises(CompositeError):
            pool.run([bad])
    with pytest.raises(CompositeError):
        Pool(buf, P, W, H, H * W, P * H * W)          # no slack after the last raster


def _set_requests(rng, P, H, W, nreq):
    """Requests whose ids are distinct (sets), plus the edge cases."""
    reqs = [dict(ids=[], x0=0, y0=0, w=W, h=H),
            dict(ids=[P - 1], x0=W - 1, y0=H - 1, w=1, h=1),
            dict(ids=list(range(P)), x0=0, y0=0, w=W, h=H)]
    for _ in range(nreq - len(reqs)):
        w = int(rng.integers(1, W + 1))
        h = int(rng.integers(1, H + 1))
        n = int(rng.integers(0, P + 1))
        reqs.append(dict(ids=rng.choice(P, n, replace=False).tolist(),
                         x0=int(rng.integers(0, W - w + 1)), y0=int(rng.integers(0, H - h + 1)),
                         w=w, h=h))
    return reqs


# (P, H, W, requests): one partial tile; several tiles per row with a ragged
# last one; exactly one tile; more than 64 requests, so more than one pass of
# 32 per tile and more than one ballot chunk
@pytest.mark.parametrize("P,H,W,nreq", [(37, 45, 77, 16), (23, 6, 2501, 40), (16, 9, 1024, 24),
                                        (29, 4, 3000, 150)])
@pytest.mark.parametrize("graph,nt,bpc", [(1, 0, 2), (0, 1, 1), (1, 1, 4)])
def test_shared_mode_small(P, H, W, nreq, graph, nt, bpc):
    rng = np.random.default_rng(P * W + nreq)
    stack = synth.random_members(P + H, P, H, W)
    reqs = _set_requests(rng, P, H, W, nreq)
    exp = oracle.batch(stack, reqs)
    buf = _pool_tensor(stack)
    say("shared", P, H, W, nreq, graph, nt, bpc)
    tune = make_tune(CMP_BATCH_SHARED, 1024, bpc, graph, CMP_ORDER_ROWS, nt)
    with Pool(buf, P, W, H, H * W, buf.numel()) as pool:
        for rep in range(2):                          # the second run replays the graph
            _outs(reqs, pad=3 * rep)
            pool.run(reqs, tune)
            ms, items, mode = pool.last()
            assert mode == CMP_BATCH_SHARED and items == H * ((W + 1023) // 1024)
            for k, (r, e) in enumerate(zip(reqs, exp)):
                assert np.array_equal(_got(r), e), f"run {rep}, request {k}"


def test_shared_mode_falls_back_on_repeated_ids():
    stack, reqs = _small_case(11)                     # has a request with ids [5, 5, 5]
    P, H, W = stack.shape
    exp = oracle.batch(stack, reqs)
    buf = _pool_tensor(stack)
    with Pool(buf, P, W, H, H * W, buf.numel()) as pool:
        _outs(reqs)
        pool.run(reqs, make_tune(CMP_BATCH_SHARED, 256, 2, 1))
        assert pool.last()[2] == CMP_BATCH_PERSISTENT
        for k, (r, e) in enumerate(zip(reqs, exp)):
            assert np.array_equal(_got(r), e), f"request {k}"
        sets = [dict(r, ids=sorted(set(r["ids"]))) for r in reqs]
        _outs(sets)
        pool.run(sets, make_tune(CMP_BATCH_SHARED, 256, 2, 1))
        assert pool.last()[2] == CMP_BATCH_SHARED
        for k, (r, e) in enumerate(zip(sets, oracle.batch(stack, sets))):
            assert np.array_equal(_got(r), e), f"set request {k}"


# (P, H, W, requests): one partial tile narrower than a wave's 128 pixels;
# several tiles per row with a ragged last one; exactly two tiles; three
# blocks of 64 requests, the last partial; pools ending in a partial chunk of
# 32 members, and spanning ten chunks
@pytest.mark.parametrize("P,H,W,nreq", [(37, 45, 77, 16), (23, 6, 2501, 40), (16, 9, 1024, 24),
                                        (29, 4, 3000, 150), (70, 5, 640, 70), (300, 3, 130, 20),
                                        (1, 7, 1, 5)])
@pytest.mark.parametrize("graph,nt,bpc", [(1, 0, 2), (0, 1, 1), (1, 1, 2)])
def test_matrix_mode_small(P, H, W, nreq, graph, nt, bpc):
    rng = np.random.default_rng(P * W + nreq + 1)
    stack = synth.random_members(P + H + 1, P, H, W)
    reqs = _set_requests(rng, P, H, W, nreq)
    exp = oracle.batch(stack, reqs)
    buf = _pool_tensor(stack)
    say("matrix", P, H, W, nreq, graph, nt, bpc)
    tune = make_tune(CMP_BATCH_MATRIX, 1024, bpc, graph, CMP_ORDER_ROWS, nt)
    with Pool(buf, P, W, H, H * W, buf.numel()) as pool:
        for rep in range(2):                          # the second run replays the graph
            _outs(reqs, pad=3 * rep)
            pool.run(reqs, tune)
            ms, items, mode = pool.last()
            assert mode == CMP_BATCH_MATRIX
            assert items == (nreq + 63) // 64 * H * ((W + 511) // 512)
            for k, (r, e) in enumerate(zip(reqs, exp)):
                assert np.array_equal(_got(r), e), f"run {rep}, request {k}"


def test_matrix_mode_tile_edges():
    """Windows that start, end or sit exactly at the 512-pixel tile edges and
    one pixel either side of them, single-row windows at the first and last
    rows, and 65 requests, so that the second block of 64 holds one."""
    P, H, W = 45, 6, 1536
    stack = synth.random_members(31, P, H, W)
    rng = np.random.default_rng(8)
    edges = [(0, 512), (512, 512), (511, 2), (1023, 2), (1024, 512), (1535, 1), (0, W),
             (510, 3), (1022, 4), (513, 510)]
    reqs = []
    for k in range(65):
        x0, w = edges[k % len(edges)]
        y0 = [0, H - 1, 2, 0][k % 4]
        h = 1 if k % 4 < 2 else H - y0
        reqs.append(dict(ids=rng.choice(P, int(rng.integers(0, P + 1)), replace=False).tolist(),
                         x0=x0, y0=y0, w=w, h=h))
    exp = oracle.batch(stack, reqs)
    buf = _pool_tensor(stack)
    with Pool(buf, P, W, H, H * W, buf.numel()) as pool:
        for bpc, nt in ((1, 0), (2, 1)):
            say("matrix tile edges", P, H, W, len(reqs), bpc, nt)
            _outs(reqs, pad=bpc)
            pool.run(reqs, make_tune(CMP_BATCH_MATRIX, 1024, bpc, 1, CMP_ORDER_ROWS, nt))
            assert pool.last()[2] == CMP_BATCH_MATRIX
            for k, (r, e) in enumerate(zip(reqs, exp)):
                assert np.array_equal(_got(r), e), f"bpc {bpc}, request {k}"


def test_matrix_mode_nonzero_values_and_dense_sets():
    """Members with every byte value (the nonzero test, not a mask), and
    requests holding every member of a pool of 96 (three full chunks)."""
    P, H, W = 96, 3, 515
    rng = np.random.default_rng(5)
    stack = rng.integers(0, 256, (P, H, W), dtype=np.uint8)
    stack[:, :, ::3] = 0                              # zeros at known places
    stack[5] = np.arange(H * W, dtype=np.int64).reshape(H, W) % 256
    reqs = [dict(ids=list(range(P)), x0=0, y0=0, w=W, h=H),
            dict(ids=list(range(P - 1, -1, -2)), x0=3, y0=1, w=W - 7, h=2),
            dict(ids=[5], x0=0, y0=0, w=W, h=H)]
    exp = oracle.batch(stack, reqs)
    buf = _pool_tensor(stack)
    with Pool(buf, P, W, H, H * W, buf.numel()) as pool:
        _outs(reqs)
        pool.run(reqs, make_tune(CMP_BATCH_MATRIX, 1024, 1, 1, CMP_ORDER_ROWS, 0))
        assert pool.last()[2] == CMP_BATCH_MATRIX
        for k, (r, e) in enumerate(zip(reqs, exp)):
            assert np.array_equal(_got(r), e), f"request {k}"


def test_matrix_mode_falls_back():
    """Repeated ids run in the persistent mode; a stride the matrix mode
    cannot address runs in the shared mode; both exact."""
    stack, reqs = _small_case(12)                     # has a request with ids [5, 5, 5]
    P, H, W = stack.shape
    buf = _pool_tensor(stack)
    tune = make_tune(CMP_BATCH_MATRIX, 256, 2, 1)
    with Pool(buf, P, W, H, H * W, buf.numel()) as pool:
        _outs(reqs)
        pool.run(reqs, tune)
        assert pool.last()[2] == CMP_BATCH_PERSISTENT
        for k, (r, e) in enumerate(zip(reqs, oracle.batch(stack, reqs))):
            assert np.array_equal(_got(r), e), f"request {k}"
    # one raster with a stride of 2^28 bytes: 31 strides exceed 32-bit offsets
    one = stack[:1]
    reqs1 = [dict(ids=[0], x0=0, y0=0, w=W, h=H), dict(ids=[], x0=2, y0=3, w=5, h=4)]
    buf1 = _pool_tensor(one)
    with Pool(buf1, 1, W, H, 1 << 28, buf1.numel()) as pool:
        _outs(reqs1)
        pool.run(reqs1, tune)
        assert pool.last()[2] == CMP_BATCH_SHARED
        for k, (r, e) in enumerate(zip(reqs1, oracle.batch(one, reqs1))):
            assert np.array_equal(_got(r), e), f"request {k}"


def test_matrix_mode_large_pool_uses_more_than_64k_lds():
    """8192 rasters, the limit: M of a request block takes 64 KiB of LDS,
    which with the union bytes and chunk list (65.5 KiB in all) is above the
    64 KiB a launch gets by default."""
    P, H, W = 8192, 2, 9
    stack = synth.random_members(78, P, H, W)
    rng = np.random.default_rng(4)
    reqs = [dict(ids=rng.choice(P, int(rng.integers(1, 3000)), replace=False).tolist(),
                 x0=int(rng.integers(0, 5)), y0=int(rng.integers(0, 2)), w=4, h=1) for _ in range(70)]
    reqs.append(dict(ids=list(range(P)), x0=0, y0=0, w=W, h=H))
    exp = oracle.batch(stack, reqs)
    buf = _pool_tensor(stack)
    with Pool(buf, P, W, H, H * W, buf.numel()) as pool:
        _outs(reqs)
        pool.run(reqs, make_tune(CMP_BATCH_MATRIX, 256, 2, 1, CMP_ORDER_ROWS, 1))
        assert pool.last()[2] == CMP_BATCH_MATRIX
        for k, (r, e) in enumerate(zip(reqs, exp)):
            assert np.array_equal(_got(r), e), f"request {k}"


def test_matrix_mode_pool_above_limit_runs_shared():
    P, H, W = 8193, 2, 9
    stack = synth.random_members(77, P, H, W)
    rng = np.random.default_rng(3)
    reqs = [dict(ids=rng.choice(P, 40, replace=False).tolist(), x0=1, y0=0, w=7, h=2),
            dict(ids=[P - 1, 0], x0=0, y0=1, w=W, h=1)]
    buf = _pool_tensor(stack)
    with Pool(buf, P, W, H, H * W, buf.numel()) as pool:
        _outs(reqs)
        pool.run(reqs, make_tune(CMP_BATCH_MATRIX, 256, 2, 1))
        assert pool.last()[2] == CMP_BATCH_SHARED
        for k, (r, e) in enumerate(zip(reqs, oracle.batch(stack, reqs))):
            assert np.array_equal(_got(r), e), f"request {k}"


def _closed_form_counts(levels_sorted, e_crop):
    # count of levels L > e, for members e < L of one shared elevation field
    return len(levels_sorted) - np.searchsorted(levels_sorted, e_crop, side="right")


def test_full_batched_pool_2048():
    wl = synth.BATCHED
    say("full batched", wl.name)
    e = wl.elevation()
    lv = wl.levels()
    et = torch.from_numpy(e).cuda()
    plane = wl.H * wl.W
    buf = torch.empty(wl.pool * plane + 64, dtype=torch.uint8, device="cuda")
    for i, L in enumerate(lv):
        synth.member_torch(et, int(L), "mask", out=buf[i * plane:(i + 1) * plane].view(wl.H, wl.W))
    torch.cuda.synchronize()
    reqs = wl.requests()
    rng = np.random.default_rng(0)
    _outs(reqs)
    with Pool(buf, wl.pool, wl.W, wl.H, plane, buf.numel()) as pool:
        best = autotune(pool, reqs[:16], reps=1)
        say("autotuned", best)
        per = best["by_mode"][str(CMP_BATCH_PERSISTENT)]
        for tune in (make_tune(best["mode"], best["tile_vecs"], best["blocks_per_cu"], 1,
                               best["order"], best["stream_loads"], best["slots"]),
                     make_tune(CMP_BATCH_PERSISTENT, per["tile_vecs"], per["blocks_per_cu"], 1,
                               per["order"], per["stream_loads"]),
                     make_tune(CMP_BATCH_SHARED, 1024, 2, 1, CMP_ORDER_ROWS, 1, 16),
                     make_tune(CMP_BATCH_MATRIX, 1024, 2, 1, CMP_ORDER_ROWS, 0),
                     make_tune(CMP_BATCH_MATRIX, 1024, 1, 0, CMP_ORDER_ROWS, 1),
                     make_tune(CMP_BATCH_PER_REQUEST)):
            _outs(reqs)
            pool.run(reqs, tune)
            assert pool.last()[2] == tune.mode
            for k, r in enumerate(reqs):
                got = _got(r)
                ec = e[r["y0"]:r["y0"] + r["h"], r["x0"]:r["x0"] + r["w"]]
                exp = _closed_form_counts(np.sort(lv[r["ids"]]), ec)
                assert np.array_equal(got, exp), f"request {k} vs closed form"
                # sampled pixels against the oracle, members rebuilt on the host
                ys = rng.integers(0, r["h"], 16)
                xs = rng.integers(0, r["w"], 16)
                es = ec[ys, xs]
                o = oracle.accumulate([synth.mask(es, int(lv[i])) for i in r["ids"]],
                                      shape=es.shape, outputs=("count",))["count"]
                assert np.array_equal(got[ys, xs], o), f"request {k} vs oracle samples"
