"""The seeded input generators (CPU)."""

import numpy as np
import pytest
import torch

from paper_2104_14667_amd import synth


def test_elevation_is_deterministic_and_spans_uint8():
    a = synth.elevation(5, 64, 96, 4.0)
    b = synth.elevation(5, 64, 96, 4.0)
    c = synth.elevation(6, 64, 96, 4.0)
    assert a.dtype == np.uint8 and a.shape == (64, 96)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert a.min() == 0 and a.max() == 255


def test_elevation_is_smooth():
    e = synth.elevation(1, 256, 256, 16.0).astype(np.int64)
    # neighbouring pixels of a field smoothed over 16 px differ by little
    assert np.abs(np.diff(e, axis=1)).mean() < 4.0
    assert np.abs(np.diff(e, axis=0)).mean() < 4.0


def test_levels_range_and_spread():
    lv = synth.levels(0, 20000, 64, 192)
    assert lv.min() == 64 and lv.max() == 192
    assert abs(lv.mean() - 128.0) < 1.0


def test_members_match_definitions():
    e = synth.elevation(2, 32, 48, 3.0)
    for L in (0, 1, 64, 200, 255, 256):
        m = synth.mask(e, L)
        d = synth.depth(e, L)
        for y in range(0, 32, 5):
            for x in range(0, 48, 7):
                assert m[y, x] == (1 if int(e[y, x]) < L else 0)
                assert d[y, x] == min(max(L - int(e[y, x]), 0), 255)


@pytest.mark.parametrize("kind", ["mask", "depth"])
def test_torch_members_are_bit_identical(kind):
    e = synth.elevation(3, 40, 72, 5.0)
    et = torch.from_numpy(e)
    for L in (0, 64, 128, 224, 255):
        ref = synth.mask(e, L) if kind == "mask" else synth.depth(e, L)
        got = synth.member_torch(et, L, kind).numpy()
        assert np.array_equal(ref, got)


def test_batch_requests_fit_and_are_seeded():
    wl = synth.BATCHED
    r1 = wl.requests()
    r2 = wl.requests()
    assert len(r1) == 64
    for a, b in zip(r1, r2):
        assert np.array_equal(a["ids"], b["ids"]) and a["x0"] == b["x0"]
        assert 4 <= len(a["ids"]) <= 512 and len(set(a["ids"].tolist())) == len(a["ids"])
        assert 512 <= a["w"] == a["h"] <= 2048
        assert 0 <= a["x0"] and a["x0"] + a["w"] <= 2048
        assert 0 <= a["y0"] and a["y0"] + a["h"] <= 2048


def test_serve_schedule_is_valid():
    wl = synth.SERVED.scaled(sessions=64, pool=1024)
    sched = wl.schedule(2000)
    held = [set() for _ in range(64)]
    t_prev = 0.0
    nadd = 0
    for r in sched:
        assert r["t"] > t_prev
        t_prev = r["t"]
        ids = [int(i) for i in r["ids"]]
        assert len(ids) >= 1 and len(set(ids)) == len(ids)
        if r["op"] == "add":
            nadd += 1
            assert not (set(ids) & held[r["sid"]])
            held[r["sid"]].update(ids)
        else:
            assert set(ids) <= held[r["sid"]]
            held[r["sid"]] -= set(ids)
        assert 0 <= r["vx0"] <= 4096 - 1024 and 0 <= r["vy0"] <= 4096 - 1024
    # roughly Poisson at the offered rate, roughly 60% adds
    assert abs(len(sched) / sched[-1]["t"] - 2000.0) < 150.0
    assert 0.55 < nadd / len(sched) < 0.75


def test_serve_schedule_full_session_turns_add_into_remove():
    wl = synth.SERVED.scaled(sessions=2, pool=8, k_lo=4, k_hi=8, view=16, W=64, H=64)
    held = [set(), set()]
    for r in wl.schedule(300):
        ids = set(int(i) for i in r["ids"])
        assert ids
        if r["op"] == "add":
            assert not (ids & held[r["sid"]])
            held[r["sid"]] |= ids
        else:
            assert ids <= held[r["sid"]]
            held[r["sid"]] -= ids
