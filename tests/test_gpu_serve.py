"""Served sessions through the C ABI (GPU): every viewport returned in the
concurrent mix equals the oracle's replay of that session alone.  Tolerance
zero."""

import numpy as np
import pytest
import torch

import oracle
from paper_2104_14667_amd import synth
from paper_2104_14667_amd.composite import (CMP_EBUSY, CMP_EINVAL, CMP_ENOMEM, CMP_ENOTMEMBER,
                                            CMP_ERANGE, CMP_OP_ADD, CMP_OP_REMOVE, CompositeError,
                                            Pool, Server)

from gpu_common import say

pytestmark = pytest.mark.gpu


def _pool(stack):
    P, H, W = stack.shape
    buf = torch.zeros(P * H * W + 64, dtype=torch.uint8, device="cuda")
    buf[: P * H * W].copy_(torch.from_numpy(stack.reshape(-1)))
    torch.cuda.synchronize()
    return buf


def _vbuf(cb, shape, fill=0):
    """Page-locked host buffer for viewport counts of a server whose session
    composites hold cb bits (viewports come back in that width)."""
    return torch.full(shape, fill, dtype=torch.int16 if cb == 16 else torch.int32, pin_memory=True)


def _counts(t):
    """Viewport counts of a buffer made by _vbuf, as int64."""
    return t.numpy().view(np.uint16 if t.dtype == torch.int16 else np.uint32).astype(np.int64)


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
        dst = _vbuf(srv.opts.count_bits, (r["vh"], r["vw"]), -1)
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
            got = _counts(outs[i])
            assert np.array_equal(got, v["count"]), f"request {i} (session {sid})"


# remat: 0 copies every evicted non-empty composite to host memory and back, 65535
# drops and rebuilds every one, 4 drops sessions of at most 4 members only
# bpc: persistent workgroups per CU, or 0 for one workgroup per work item;
# cb: bits of the session composites.  Budgets below the 5 sessions admit
# them by oversubscription (they live by eviction)
# bpc 0 steps launch the viewport rows and, beside them on a second stream,
# the other rows (ordered after the step's spill and restore copies); vg: row
# blocks per workgroup of the viewport launch (0: the library's choice)
@pytest.mark.parametrize("max_batch,overlap,budget_slots,remat,bpc,cb,vg", [
    (1, 0, 8, 0, 2, 32, 0), (4, 1, 4, 0, 2, 32, 0), (64, 1, 64, 512, 2, 32, 0),
    (3, 0, 3, 65535, 2, 32, 0), (8, 1, 10, 4, 2, 32, 0), (4, 1, 4, 512, 2, 32, 0),
    (1, 0, 3, 4, 2, 32, 0), (64, 1, 64, 512, 0, 32, 0), (4, 1, 4, 65535, 0, 32, 0),
    (4, 1, 4, 0, 2, 16, 0), (3, 0, 3, 65535, 2, 16, 0), (64, 1, 64, 512, 0, 16, 0),
    (8, 1, 10, 4, 2, 16, 0), (4, 1, 4, 0, 0, 32, 0), (4, 1, 4, 0, 0, 16, 3),
    (8, 1, 10, 4, 0, 16, 2), (1, 0, 3, 0, 0, 32, 0), (2, 1, 3, 4, 0, 32, 5)])
def test_mix_equals_alone(max_batch, overlap, budget_slots, remat, bpc, cb, vg):
    wl, stack, sched = _small(seed=max_batch + 10 * overlap + remat % 7 + cb + vg)
    P, H, W = stack.shape
    say("serve mix", max_batch, overlap, budget_slots, remat, bpc, cb, vg)
    buf = _pool(stack)
    with Pool(buf, P, W, H, H * W, buf.numel()) as pool:
        with Server(pool, max_batch=max_batch, overlap=overlap,
                    hbm_budget_bytes=budget_slots * H * W * cb // 8, max_view_pixels=16 * 16,
                    tile_vecs=64, blocks_per_cu=bpc, remat_max_members=remat, count_bits=cb,
                    oversubscribe_pct=100, view_group=vg) as srv:
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
    dst = _vbuf(32, (16, 16), 0)
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
                    max_view_pixels=16 * 16, tile_vecs=64, blocks_per_cu=bpc,
                    oversubscribe_pct=100) as srv:
            sids, outs = _run_mix(srv, wl, sched)
            assert srv.stats()["requests"] == len(sched)
    _check_alone(wl, stack, sched, outs)


@pytest.mark.parametrize("cb", [32, 16])
def test_replay_small_open_loop(cb):
    wl, stack, sched = _small(seed=5, n=300)
    P, H, W = stack.shape
    buf = _pool(stack)
    ring = [_vbuf(cb, (16, 16), 0) for _ in range(8)]
    with Pool(buf, P, W, H, H * W, buf.numel()) as pool:
        with Server(pool, max_batch=16, hbm_budget_bytes=16 * H * W * 4, max_view_pixels=256,
                    tile_vecs=64, blocks_per_cu=2, count_bits=cb) as srv:
            sids = [srv.open() for _ in range(wl.sessions)]
            sched = [dict(r, t=r["t"] * 0.25) for r in sched]      # 8000 req/s offered
            lat = srv.replay(sched, sids, ring, 16)
            assert lat.shape == (len(sched),) and (lat > 0).all()
            assert srv.stats()["requests"] == len(sched)


@pytest.mark.parametrize("remat,cb", [(2048, 32), (0, 32), (0, 16)])
def test_full_served_shape_bursts(remat, cb):
    """Sessions of 4096x4096 over a pool of 1024 depth maps, half of them
    resident (admitted by oversubscription); bursts of 64 requests are checked
    against the closed form of each session's ids.  Evicted composites are
    rebuilt from their members (remat 2048) or copied to host memory and back
    (remat 0); uint32 or uint16 composites."""
    wl = synth.SERVED
    say("full served", wl.name, remat, cb)
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
        with Server(pool, max_batch=64, hbm_budget_bytes=128 * plane * cb // 8,
                    remat_max_members=remat, count_bits=cb, oversubscribe_pct=100) as srv:
            sids = [srv.open() for _ in range(wl.sessions)]
            for b0 in range(0, len(sched), 64):
                burst = sched[b0:b0 + 64]
                outs, tickets = [], []
                for r in burst:
                    dst = _vbuf(cb, (r["vh"], r["vw"]), 0)
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
                    assert np.array_equal(_counts(dst), exp)
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
                    dst = _vbuf(32, (r["vh"], r["vw"]), -1)
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


def _expect_view(stack, held, r):
    """The oracle's count over the window of the members held (id -> multiplicity)."""
    x0, y0, w, h = r["vx0"], r["vy0"], r["vw"], r["vh"]
    crops = (oracle.window(stack[i], x0, y0, w, h) for i, k in held.items() for _ in range(k))
    return oracle.accumulate(crops, shape=(h, w), outputs=("count",))["count"]


@pytest.mark.parametrize("cb,pct", [(32, 0), (16, 0), (32, 100)])
def test_admission_refuses_with_state_unchanged(cb, pct):
    """The HBM budget holds 3 composites: sessions beyond 3 (plus pct percent
    by oversubscription) are refused with CMP_ENOMEM, nothing changes, the
    admitted sessions still serve exact viewports, and a close makes room."""
    wl, stack, sched = _small(seed=31, sessions=3, n=40)
    P, H, W = stack.shape
    say("serve admission", cb, pct)
    buf = _pool(stack)
    limit = 3 + 3 * pct // 100
    with Pool(buf, P, W, H, H * W, buf.numel()) as pool:
        with Server(pool, max_batch=2, hbm_budget_bytes=3 * H * W * cb // 8 + H * W * cb // 16,
                    max_view_pixels=256, tile_vecs=64, count_bits=cb, oversubscribe_pct=pct) as srv:
            sids = [srv.open() for _ in range(limit)]
            st0 = srv.stats()
            for k in range(2):
                with pytest.raises(CompositeError) as ei:
                    srv.open()
                assert ei.value.status == CMP_ENOMEM
                assert srv.try_open() is None
            st1 = srv.stats()
            assert st1["refused_sessions"] == st0["refused_sessions"] + 4
            assert {k: v for k, v in st1.items() if k != "refused_sessions"} == \
                   {k: v for k, v in st0.items() if k != "refused_sessions"}
            # every admitted session serves, in the mix, what it serves alone
            outs = []
            for r in sched:
                dst = _vbuf(cb, (r["vh"], r["vw"]), -1)
                op = CMP_OP_ADD if r["op"] == "add" else CMP_OP_REMOVE
                outs.append((srv.submit(sids[r["sid"]], op, r["ids"],
                                        (r["vx0"], r["vy0"], r["vw"], r["vh"]), dst), dst))
            for t, _ in outs:
                srv.wait(t)
            _check_alone(wl, stack, sched, [d for _, d in outs])
            srv.close_session(sids[0])
            sid = srv.open()                                   # room again
            assert sid not in sids
            with pytest.raises(CompositeError) as ei:
                srv.open()
            assert ei.value.status == CMP_ENOMEM
            dst = _vbuf(cb, (16, 16), -1)
            srv.wait(srv.submit(sid, CMP_OP_ADD, [0, 1], (0, 0, 16, 16), dst))
            held = {0: 1, 1: 1}
            exp = _expect_view(stack, held, dict(vx0=0, vy0=0, vw=16, vh=16))
            assert np.array_equal(_counts(dst), exp)


def test_queue_bound_refuses_busy_with_state_unchanged():
    """With the server paused, max_queue requests wait; the next submit is
    refused with CMP_EBUSY and changes nothing (its ids are not held
    afterwards); after resuming every accepted request completes exactly."""
    wl, stack, sched = _small(seed=41, sessions=2, n=4)
    P, H, W = stack.shape
    say("serve queue bound")
    buf = _pool(stack)
    with Pool(buf, P, W, H, H * W, buf.numel()) as pool:
        with Server(pool, max_batch=2, hbm_budget_bytes=4 * H * W * 4, max_view_pixels=256,
                    tile_vecs=64, max_queue=4) as srv:
            a, b = srv.open(), srv.open()
            srv.pause(True)
            plan = [(a, CMP_OP_ADD, [1, 2]), (b, CMP_OP_ADD, [3]), (a, CMP_OP_ADD, [4]),
                    (b, CMP_OP_REMOVE, [3])]
            views, tickets = [], []
            for sid, op, ids in plan:
                dst = _vbuf(32, (16, 16), -1)
                tickets.append(srv.submit(sid, op, ids, (0, 0, 16, 16), dst))
                views.append(dst)
            spare = _vbuf(32, (16, 16), -7)
            with pytest.raises(CompositeError) as ei:
                srv.submit(a, CMP_OP_ADD, [5], (0, 0, 16, 16), spare)
            assert ei.value.status == CMP_EBUSY
            st = srv.stats()
            assert st["refused_busy"] == 1 and st["queue_peak"] == 4 and st["requests"] == 0
            srv.pause(False)
            for t in tickets:
                srv.wait(t)
            assert (spare.numpy() == -7).all()                 # never written
            with pytest.raises(CompositeError) as ei:          # 5 was never added
                srv.submit(a, CMP_OP_REMOVE, [5], (0, 0, 16, 16), spare)
            assert ei.value.status == CMP_ENOTMEMBER
            held = {a: {}, b: {}}
            for (sid, op, ids), dst in zip(plan, views):
                for i in ids:
                    held[sid][i] = held[sid].get(i, 0) + (1 if op == CMP_OP_ADD else -1)
                exp = _expect_view(stack, held[sid], dict(vx0=0, vy0=0, vw=16, vh=16))
                assert np.array_equal(_counts(dst), exp)
            assert srv.stats()["requests"] == len(plan)


def test_uint16_sessions_at_their_limit():
    """A uint16 session holds up to 65535 members: 65535 copies of one raster
    give 65535 where it is nonzero; one more member is refused with
    CMP_ERANGE and changes nothing; after a remove it is accepted."""
    rng = np.random.default_rng(5)
    P, H, W = 3, 2, 32
    stack = rng.integers(0, 3, size=(P, H, W), dtype=np.uint8)
    say("serve u16 limit")
    buf = _pool(stack)
    with Pool(buf, P, W, H, H * W, buf.numel()) as pool:
        with Server(pool, max_batch=1, hbm_budget_bytes=H * W * 2, max_view_pixels=H * W,
                    tile_vecs=64, count_bits=16) as srv:
            sid = srv.open()
            dst = _vbuf(16, (H, W), -1)
            vp = (0, 0, W, H)
            srv.wait(srv.submit(sid, CMP_OP_ADD, [0] * 65535, vp, dst))
            held = {0: 65535}
            assert np.array_equal(_counts(dst),
                                  _expect_view(stack, held, dict(vx0=0, vy0=0, vw=W, vh=H)))
            with pytest.raises(CompositeError) as ei:
                srv.submit(sid, CMP_OP_ADD, [1], vp, dst)
            assert ei.value.status == CMP_ERANGE
            srv.wait(srv.submit(sid, CMP_OP_REMOVE, [0], vp, dst))
            srv.wait(srv.submit(sid, CMP_OP_ADD, [1], vp, dst))
            held = {0: 65534, 1: 1}
            assert np.array_equal(_counts(dst),
                                  _expect_view(stack, held, dict(vx0=0, vy0=0, vw=W, vh=H)))
            with pytest.raises(CompositeError) as ei:
                srv.submit(sid, CMP_OP_ADD, [2], vp, dst)
            assert ei.value.status == CMP_ERANGE


@pytest.mark.parametrize("cb", [32, 16])
def test_replay_records_refusals_and_goes_on(cb):
    """An open-loop replay into a server whose queue holds one request: some
    submits are refused (CMP_EBUSY, or CMP_ENOTMEMBER for removes of ids only
    a refused add would have held); the replay records them and goes on, and
    the final composite of every session equals the members of its accepted
    requests."""
    wl, stack, sched = _small(seed=51, sessions=4, n=200)
    P, H, W = stack.shape
    say("serve replay refusals")
    buf = _pool(stack)
    ring = [_vbuf(cb, (16, 16), 0) for _ in range(8)]
    sched = [dict(r, t=r["t"] * 0.01) for r in sched]          # a burst: 200 requests in ~1 ms
    with Pool(buf, P, W, H, H * W, buf.numel()) as pool:
        with Server(pool, max_batch=1, overlap=0, hbm_budget_bytes=4 * H * W * 4,
                    max_view_pixels=H * W, tile_vecs=64, max_queue=1, count_bits=cb) as srv:
            sids = [srv.open() for _ in range(wl.sessions)]
            lat, status = srv.replay(sched, sids, ring, 16, with_status=True)
            ok = status == 0
            assert ok.any() and (~ok).any()
            assert set(status[~ok].tolist()) <= {CMP_EBUSY, CMP_ENOTMEMBER}
            assert (lat[ok] > 0).all() and (lat[~ok] == -1).all()
            st = srv.stats()
            assert st["requests"] == int(ok.sum())
            assert st["refused_busy"] == int((status == CMP_EBUSY).sum())
            dst = _vbuf(cb, (H, W), -1)
            for k, sid in enumerate(sids):
                held = {}
                for r, good in zip(sched, ok):
                    if good and r["sid"] == k:
                        for i in r["ids"]:
                            held[int(i)] = held.get(int(i), 0) + (1 if r["op"] == "add" else -1)
                srv.wait(srv.submit(sid, CMP_OP_ADD, [], (0, 0, W, H), dst))
                exp = _expect_view(stack, held, dict(vx0=0, vy0=0, vw=W, vh=H))
                assert np.array_equal(_counts(dst), exp), k


@pytest.mark.parametrize("cb,vg", [(32, 0), (16, 0), (16, 3)])
def test_viewport_edges_and_destination_layout(cb, vg):
    """The kernel writes each viewport straight into the caller's page-locked
    buffer, 16 bytes at a time from the destination's first 16-byte boundary:
    viewports at every column phase, of widths around the vector width, into
    destinations at every element offset and with wider pitches, in work
    items of several rows and in one row split over chunks, and (vg 3) in
    viewport work items of three row blocks.  Each equals the oracle's
    window, and no count outside it is touched."""
    rng = np.random.default_rng(61 + cb)
    for (P, H, W, tv) in [(6, 40, 96, 64), (4, 5, 4608, 256)]:
        stack = rng.integers(0, 3, size=(P, H, W), dtype=np.uint8)
        buf = _pool(stack)
        say("serve viewport edges", cb, vg, H, W, tv)
        with Pool(buf, P, W, H, H * W, buf.numel()) as pool:
            with Server(pool, max_batch=4, hbm_budget_bytes=4 * H * W * 4, max_view_pixels=H * W,
                        tile_vecs=tv, count_bits=cb, view_group=vg) as srv:
                sid = srv.open()
                held = {1: 2, 3: 1, 2: 1}
                srv.wait(srv.submit(sid, CMP_OP_ADD, [1, 1, 3, 2], (0, 0, 16, 1), _vbuf(cb, (1, 16), 0)))
                cases = []
                for vx0 in list(range(0, 17)) + [W - 33, W - 9]:
                    for vw in (1, 7, 8, 9, 16, 17, 33):
                        if vx0 + vw <= W:
                            cases.append((vx0, vw))
                cases.append((0, W))
                for c, (vx0, vw) in enumerate(cases):
                    vy0 = int(rng.integers(0, H))
                    vh = int(rng.integers(1, H - vy0 + 1))
                    off = c % 9                                   # destination element offset
                    pitch = vw + (0, 1, 3, 8)[c % 4]
                    dst = _vbuf(cb, (off + vh * pitch + 8,), -1)
                    el = 2 if cb == 16 else 4
                    srv.wait(srv.submit(sid, CMP_OP_ADD, [], (vx0, vy0, vw, vh),
                                        dst.data_ptr() + off * el, pitch))
                    got = _counts(dst)
                    sent = 65535 if cb == 16 else 2 ** 32 - 1     # -1 in the buffer's width
                    inside = np.zeros(got.shape, bool)
                    for y in range(vh):
                        inside[off + y * pitch: off + y * pitch + vw] = True
                    assert (got[~inside] == sent).all(), (vx0, vw, off, pitch)
                    view = np.stack([got[off + y * pitch: off + y * pitch + vw] for y in range(vh)])
                    exp = _expect_view(stack, held, dict(vx0=vx0, vy0=vy0, vw=vw, vh=vh))
                    assert np.array_equal(view, exp), (vx0, vy0, vw, vh, off, pitch)


def test_submit_refuses_destinations_the_kernel_cannot_write():
    """dst must be page-locked memory the device can address and aligned to a
    count: pageable memory and a misaligned address are refused with
    CMP_EINVAL, nothing changes, and the session serves on."""
    wl, stack, sched = _small(seed=71, n=10)
    P, H, W = stack.shape
    buf = _pool(stack)
    with Pool(buf, P, W, H, H * W, buf.numel()) as pool:
        with Server(pool, max_batch=2, hbm_budget_bytes=2 * H * W * 2, max_view_pixels=256,
                    tile_vecs=64, count_bits=16) as srv:
            sid = srv.open()
            pageable = np.zeros((16, 16), np.uint16)
            pinned = _vbuf(16, (16 * 16 + 1,), -1)
            for bad in (pageable, pinned.data_ptr() + 1):
                with pytest.raises(CompositeError) as ei:
                    srv.submit(sid, CMP_OP_ADD, [2], (0, 0, 16, 16), bad)
                assert ei.value.status == CMP_EINVAL
            assert srv.stats()["requests"] == 0
            torch.cuda.synchronize()                           # no error left behind
            srv.wait(srv.submit(sid, CMP_OP_ADD, [2], (0, 0, 16, 16), pinned))
            exp = _expect_view(stack, {2: 1}, dict(vx0=0, vy0=0, vw=16, vh=16))
            assert np.array_equal(_counts(pinned)[:256].reshape(16, 16), exp)


@pytest.mark.parametrize("cb,remat,vg", [(32, 0, 0), (16, 0, 2), (32, 4, 0), (16, 65535, 0)])
def test_split_steps_with_evictions(cb, remat, vg):
    """At most two requests outstanding against a step size of four: no step
    finds a backlog, so every step launches its viewport rows and, beside
    them on the second stream, the other rows, while sessions are evicted
    (copied out and back with remat 0, dropped and rebuilt with 65535, both
    with 4).  Each viewport equals the oracle's replay of its session alone."""
    wl, stack, sched = _small(seed=81 + cb + remat % 11 + vg, sessions=5, n=120)
    P, H, W = stack.shape
    say("serve split evictions", cb, remat, vg)
    buf = _pool(stack)
    with Pool(buf, P, W, H, H * W, buf.numel()) as pool:
        with Server(pool, max_batch=4, overlap=1, hbm_budget_bytes=4 * H * W * cb // 8,
                    max_view_pixels=16 * 16, tile_vecs=64, remat_max_members=remat, count_bits=cb,
                    oversubscribe_pct=100, view_group=vg) as srv:
            sids = [srv.open() for _ in range(wl.sessions)]
            outs, pending = [], []
            for r in sched:
                dst = _vbuf(cb, (r["vh"], r["vw"]), -1)
                op = CMP_OP_ADD if r["op"] == "add" else CMP_OP_REMOVE
                pending.append(srv.submit(sids[r["sid"]], op, r["ids"],
                                          (r["vx0"], r["vy0"], r["vw"], r["vh"]), dst))
                outs.append(dst)
                if len(pending) == 2:
                    srv.wait(pending.pop(0))
            for t in pending:
                srv.wait(t)
            st = srv.stats()
            assert st["requests"] == len(sched) and st["max_step"] <= 2
            if remat == 0:
                assert st["spills"] > 0 and st["restores"] > 0
            elif remat >= 65535:
                assert st["drops"] > 0 and st["spills"] == 0
            else:
                assert st["drops"] + st["spills"] > 0
    _check_alone(wl, stack, sched, outs)


@pytest.mark.parametrize("cb,vg", [(16, 0), (32, 0), (16, 3)])
def test_one_step_of_mixed_viewports(cb, vg):
    """Requests queued while the server is paused form one step: sessions whose
    viewports differ in size and place (one pixel, one row, one column, a
    square, the whole raster) are updated by one viewport launch and one
    launch of the other rows, the requests' items found by the kernel's
    search over unequal counts.  Each viewport equals the oracle's window."""
    rng = np.random.default_rng(91 + cb + vg)
    P, H, W = 8, 40, 96
    stack = rng.integers(0, 3, size=(P, H, W), dtype=np.uint8)
    buf = _pool(stack)
    views = [(5, 7, 1, 1), (0, 13, W, 1), (50, 0, 1, H), (17, 9, 33, 21), (0, 0, W, H), (80, 39, 16, 1)]
    say("serve one step mixed", cb, vg)
    with Pool(buf, P, W, H, H * W, buf.numel()) as pool:
        with Server(pool, max_batch=8, hbm_budget_bytes=8 * H * W * 4, max_view_pixels=H * W,
                    tile_vecs=64, count_bits=cb, view_group=vg) as srv:
            sids = [srv.open() for _ in views]
            held = [{} for _ in views]
            for rnd in range(3):
                srv.pause(True)
                tickets, outs = [], []
                for k, (sid, v) in enumerate(zip(sids, views)):
                    ids = [int(i) for i in rng.integers(0, P, size=1 + (k + rnd) % 5)]
                    for i in ids:
                        held[k][i] = held[k].get(i, 0) + 1
                    dst = _vbuf(cb, (v[3], v[2]), -1)
                    tickets.append(srv.submit(sid, CMP_OP_ADD, ids, v, dst))
                    outs.append(dst)
                steps0 = srv.stats()["steps"]
                srv.pause(False)
                for t in tickets:
                    srv.wait(t)
                assert srv.stats()["steps"] == steps0 + 1          # one step held them all
                for k, v in enumerate(views):
                    exp = _expect_view(stack, held[k], dict(vx0=v[0], vy0=v[1], vw=v[2], vh=v[3]))
                    assert np.array_equal(_counts(outs[k]), exp), (rnd, k, v)
