"""Served sessions through the C ABI (GPU): every viewport returned in the
concurrent mix equals the oracle's replay of that session alone.  Tolerance
zero."""

import numpy as np
import pytest
import torch

import oracle
from paper_2104_14667_amd import synth
from paper_2104_14667_amd.composite import (CMP_EINVAL, CMP_ENOTMEMBER, CMP_OP_ADD,
                                            CMP_OP_REMOVE, CompositeError, Pool, Server)

from gpu_common import say

pytestmark = pytest.mark.gpu


def _pool(stack):
    P, H, W = stack.shape
    buf = torch.zeros(P * H * W + 64, dtype=torch.uint8, device="cuda")
    buf[: P * H * W].copy_(torch.from_numpy(stack.reshape(-1)))
    torch.cuda.synchronize()
    return buf


def _small(seed=0, sessions=5, pool=40, H=48, W=64, n=160):
    wl = synth.ServeWorkload(sessions=sessions, pool=pool, H=H, W=W, sigma=4.0, view=16,
                             k_lo=1, k_hi=6, seed=seed)
    e = wl.elevation()
    lv = wl.levels()
    stack = np.stack([synth.depth(e, int(L)) for L in lv])
    return wl, stack, wl.schedule(n)


def _run_mix(srv, wl, sched, view_dims=None):
    sids = [srv.open() for _ in range(wl.sessions)]
    outs, tickets = [], []
    for r in sched:
        dst = torch.full((r["vh"], r["vw"]), -1, dtype=torch.int32, pin_memory=True)
        op = CMP_OP_ADD if r["op"] == "add" else CMP_OP_REMOVE
        tickets.append(srv.submit(sids[r["sid"]], op, r["ids"],
                                  (r["vx0"], r["vy0"], r["vw"], r["vh"]), dst))
        outs.append(dst)
    for t in tickets:
        srv.wait(t)
    return sids, outs


def _check_alone(wl, stack, sched, outs):
    for sid in range(wl.sessions):
        idx = [i for i, r in enumerate(sched) if r["sid"] == sid]
        views = oracle.replay_session(stack, [sched[i] for i in idx])
        for i, v in zip(idx, views):
            got = outs[i].numpy().view(np.uint32).astype(np.int64)
            assert np.array_equal(got, v["count"]), f"request {i} (session {sid})"


# remat: 0 copies every evicted non-empty composite to host memory and back, 65535
# drops and rebuilds every one, 4 drops sessions of at most 4 members only
# bpc: persistent workgroups per CU, or 0 for one workgroup per work item
@pytest.mark.parametrize("max_batch,overlap,budget_slots,remat,bpc", [
    (1, 0, 8, 0, 2), (4, 1, 4, 0, 2), (64, 1, 64, 512, 2), (3, 0, 3, 65535, 2), (8, 1, 10, 4, 2),
    (4, 1, 4, 512, 2), (1, 0, 3, 4, 2), (64, 1, 64, 512, 0), (4, 1, 4, 65535, 0)])
def test_mix_equals_alone(max_batch, overlap, budget_slots, remat, bpc):
    wl, stack, sched = _small(seed=max_batch + 10 * overlap + remat % 7)
    P, H, W = stack.shape
    say("serve mix", max_batch, overlap, budget_slots, remat, bpc)
    buf = _pool(stack)
    with Pool(buf, P, W, H, H * W, buf.numel()) as pool:
        with Server(pool, max_batch=max_batch, overlap=overlap,
                    hbm_budget_bytes=budget_slots * H * W * 4, max_view_pixels=16 * 16,
                    tile_vecs=64, blocks_per_cu=bpc, remat_max_members=remat) as srv:
            sids, outs = _run_mix(srv, wl, sched)
            st = srv.stats()
            assert st["requests"] == len(sched)
            assert st["max_step"] <= max_batch
            if budget_slots < wl.sessions:
                if remat == 0:
                    assert st["spills"] > 0 and st["restores"] > 0
                elif remat >= P * 8:
                    assert st["drops"] > 0 and st["rebuilds"] > 0 and st["spills"] == 0
                else:
                    assert st["drops"] > 0 and st["spills"] > 0
            else:
                assert st["spills"] == st["drops"] == 0
    _check_alone(wl, stack, sched, outs)


def test_submit_validation():
    wl, stack, sched = _small(seed=3, n=10)
    P, H, W = stack.shape
    buf = _pool(stack)
    dst = torch.zeros((16, 16), dtype=torch.int32, pin_memory=True)
    with Pool(buf, P, W, H, H * W, buf.numel()) as pool:
        with Server(pool, max_batch=4, hbm_budget_bytes=8 * H * W * 4, max_view_pixels=256,
                    max_sessions=2) as srv:
            a = srv.open()
            b = srv.open()
            with pytest.raises(CompositeError):
                srv.open()                                   # max_sessions
            t = srv.submit(a, CMP_OP_ADD, [1, 2, 2], (0, 0, 16, 16), dst)
            for bad in [dict(op=CMP_OP_REMOVE, ids=[3]), dict(op=CMP_OP_REMOVE, ids=[2, 2, 2])]:
                with pytest.raises(CompositeError) as ei:
                    srv.submit(a, bad["op"], bad["ids"], (0, 0, 16, 16), dst)
                assert ei.value.status == CMP_ENOTMEMBER
            for vp in [(W - 15, 0, 16, 16), (0, 0, 17, 16), (0, H, 1, 1)]:
                with pytest.raises(CompositeError) as ei:
                    srv.submit(a, CMP_OP_ADD, [1], vp, dst)
                assert ei.value.status == CMP_EINVAL
            with pytest.raises(CompositeError):
                srv.submit(a, CMP_OP_ADD, [P], (0, 0, 16, 16), dst)
            srv.wait(t)
            t2 = srv.submit(a, CMP_OP_REMOVE, [2, 2, 1], (0, 0, 16, 16), dst)   # valid now
            srv.wait(t2)
            assert not dst.numpy().any()                     # empty again
            srv.close_session(b)
            c = srv.open()
            assert c not in (a, b)


@pytest.mark.parametrize("bpc", [0, 3])
def test_heavy_requests_automatic_launch(bpc):
    """Requests of 70-120 members: with blocks_per_cu 0 their steps average
    more than 64 members and run on the persistent grid; both launch forms
    equal the oracle's replay of each session alone."""
    wl = synth.ServeWorkload(sessions=3, pool=260, H=40, W=80, sigma=4.0, view=16,
                             k_lo=70, k_hi=120, seed=21)
    e = wl.elevation()
    lv = wl.levels()
    stack = np.stack([synth.depth(e, int(L)) for L in lv])
    sched = wl.schedule(24)
    P, H, W = stack.shape
    say("serve heavy", bpc)
    buf = _pool(stack)
    with Pool(buf, P, W, H, H * W, buf.numel()) as pool:
        with Server(pool, max_batch=2, overlap=1, hbm_budget_bytes=2 * H * W * 4,
                    max_view_pixels=16 * 16, tile_vecs=64, blocks_per_cu=bpc) as srv:
            sids, outs = _run_mix(srv, wl, sched)
            assert srv.stats()["requests"] == len(sched)
    _check_alone(wl, stack, sched, outs)


def test_replay_small_open_loop():
    wl, stack, sched = _small(seed=5, n=300)
    P, H, W = stack.shape
    buf = _pool(stack)
    ring = [torch.zeros((16, 16), dtype=torch.int32, pin_memory=True) for _ in range(8)]
    with Pool(buf, P, W, H, H * W, buf.numel()) as pool:
        with Server(pool, max_batch=16, hbm_budget_bytes=16 * H * W * 4, max_view_pixels=256,
                    tile_vecs=64, blocks_per_cu=2) as srv:
            sids = [srv.open() for _ in range(wl.sessions)]
            sched = [dict(r, t=r["t"] * 0.25) for r in sched]      # 8000 req/s offered
            lat = srv.replay(sched, sids, ring, 16)
            assert lat.shape == (len(sched),) and (lat > 0).all()
            assert srv.stats()["requests"] == len(sched)


@pytest.mark.parametrize("remat", [2048, 0])
def test_full_served_shape_bursts(remat):
    """Sessions of 4096x4096 over a pool of 1024 depth maps, half of them
    resident; bursts of 64 requests are checked against the closed form of
    each session's ids.  Evicted composites are rebuilt from their members
    (remat 2048) or copied to host memory and back (remat 0)."""
    wl = synth.SERVED
    say("full served", wl.name, remat)
    e = wl.elevation()
    lv = wl.levels()
    et = torch.from_numpy(e).cuda()
    plane = wl.H * wl.W
    buf = torch.empty(wl.pool * plane + 64, dtype=torch.uint8, device="cuda")
    for i, L in enumerate(lv):
        synth.member_torch(et, int(L), "depth", out=buf[i * plane:(i + 1) * plane].view(wl.H, wl.W))
    torch.cuda.synchronize()
    sched = wl.schedule(256)
    held = [[] for _ in range(wl.sessions)]
    with Pool(buf, wl.pool, wl.W, wl.H, plane, buf.numel()) as pool:
        with Server(pool, max_batch=64, hbm_budget_bytes=128 * plane * 4,
                    remat_max_members=remat) as srv:
            sids = [srv.open() for _ in range(wl.sessions)]
            for b0 in range(0, len(sched), 64):
                burst = sched[b0:b0 + 64]
                outs, tickets = [], []
                for r in burst:
                    dst = torch.empty((r["vh"], r["vw"]), dtype=torch.int32, pin_memory=True)
                    op = CMP_OP_ADD if r["op"] == "add" else CMP_OP_REMOVE
                    tickets.append(srv.submit(sids[r["sid"]], op, r["ids"],
                                              (r["vx0"], r["vy0"], r["vw"], r["vh"]), dst))
                    outs.append(dst)
                for t in tickets:
                    srv.wait(t)
                for r, dst in zip(burst, outs):
                    if r["op"] == "add":
                        held[r["sid"]] += [int(i) for i in r["ids"]]
                    else:
                        for i in r["ids"]:
                            held[r["sid"]].remove(int(i))
                    lvs = np.sort(lv[held[r["sid"]]])
                    ev = e[r["vy0"]:r["vy0"] + r["vh"], r["vx0"]:r["vx0"] + r["vw"]]
                    exp = len(lvs) - np.searchsorted(lvs, ev, side="right")
                    assert np.array_equal(dst.numpy().view(np.uint32), exp)
            st = srv.stats()
            assert st["requests"] == len(sched)
            if remat:
                assert st["drops"] > 0 and st["spills"] == 0
            else:
                assert st["spills"] > 0                     # only empty sessions are dropped


def test_threaded_submitters_and_close_semantics():
    """Several host threads submit to their own sessions at once; each result
    equals the session replayed alone.  A close races with in-flight work only
    as EBUSY; freeing the server drains what was submitted."""
    import threading
    from paper_2104_14667_amd.composite import CMP_EBUSY
    wl, stack, sched = _small(seed=21, sessions=6, n=240)
    P, H, W = stack.shape
    buf = _pool(stack)
    outs = [None] * len(sched)
    with Pool(buf, P, W, H, H * W, buf.numel()) as pool:
        srv = Server(pool, max_batch=8, hbm_budget_bytes=8 * H * W * 4, max_view_pixels=256,
                     tile_vecs=64, blocks_per_cu=2)
        sids = [srv.open() for _ in range(wl.sessions)]
        errors = []

        def run(sid_idx):
            try:
                tickets = []
                for i, r in enumerate(sched):
                    if r["sid"] != sid_idx:
                        continue
                    dst = torch.full((r["vh"], r["vw"]), -1, dtype=torch.int32, pin_memory=True)
                    op = CMP_OP_ADD if r["op"] == "add" else CMP_OP_REMOVE
                    tickets.append(srv.submit(sids[sid_idx], op, r["ids"],
                                              (r["vx0"], r["vy0"], r["vw"], r["vh"]), dst))
                    outs[i] = dst
                for t in tickets[: len(tickets) // 2]:
                    srv.wait(t)
            except Exception as ex:          # surfaced below
                errors.append(ex)

        th = [threading.Thread(target=run, args=(k,)) for k in range(wl.sessions)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        assert not errors, errors
        try:
            srv.close_session(sids[0])
            closed = True
        except CompositeError as ex:
            assert ex.status == CMP_EBUSY
            closed = False
        srv.close()                          # drains every submitted request
        assert closed in (True, False)
    _check_alone(wl, stack, sched, outs)
