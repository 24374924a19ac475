"""Pins for the CPU oracle: checks against facts fixed by mathematics and by the
input recipe, not by the oracle itself.

Each ``pin_*`` takes an implementation object exposing the oracle's functions
(``accumulate``, ``narrow``, ``window``, ``Multiset``, ``batch``,
``replay_session``, ``overlap_histogram``) and raises AssertionError on a
mismatch.  The same pins run against the real oracle (they must pass) and
against oracles with planted mistakes (each must be caught by some pin).
"""

from __future__ import annotations

import itertools

import numpy as np

from paper_2104_14667_amd import synth


# ----------------------------------------------------------------------------
# Independent forms of the expected values.

def brute_force(stack, H, W):
    """Per-pixel scalar evaluation with Python integers: sort the member values
    of each pixel and read count, sum and max off the sorted list."""
    n = len(stack)
    cnt = [[0] * W for _ in range(H)]
    tot = [[0] * W for _ in range(H)]
    mx = [[0] * W for _ in range(H)]
    for y in range(H):
        for x in range(W):
            vals = sorted(int(stack[i][y][x]) for i in range(n))
            nonzero = [v for v in vals if v != 0]
            cnt[y][x] = len(nonzero)
            t = 0
            for v in vals:
                t += v
            tot[y][x] = t
            mx[y][x] = vals[-1] if vals else 0
    return cnt, tot, mx


def closed_form_lut(levels, kind):
    """Composite of members generated from one elevation field, as a function
    of the elevation value e alone (all members share the field):

    * mask members  m_i = [e < L_i]:           count = sum = #{i: L_i > e},
                                                max = [exists i: L_i > e]
    * depth members m_i = clamp(L_i - e, 0, 255): count = #{i: L_i > e},
                                                sum = sum_i clamp(L_i - e, 0, 255),
                                                max = clamp(max_i L_i - e, 0, 255)

    Built with Python integers over the 256 possible elevations."""
    cnt = np.zeros(256, dtype=np.int64)
    tot = np.zeros(256, dtype=np.int64)
    mx = np.zeros(256, dtype=np.int64)
    for e in range(256):
        above = [int(L) for L in levels if int(L) > e]
        cnt[e] = len(above)
        if kind == "mask":
            tot[e] = len(above)
            mx[e] = 1 if above else 0
        else:
            tot[e] = sum(min(L - e, 255) for L in above)
            mx[e] = min(max(above) - e, 255) if above else 0
    return cnt, tot, mx


def _as(a):
    return np.asarray(a, dtype=np.int64)


# ----------------------------------------------------------------------------
# Pins.

def pin_brute_force(impl, seed=11, cases=40):
    rng = np.random.default_rng(seed)
    for _ in range(cases):
        H = int(rng.integers(1, 18))
        W = int(rng.integers(1, 18))
        n = int(rng.integers(0, 7))
        stack = synth.random_members(int(rng.integers(1 << 30)), n, H, W)
        got = impl.accumulate(list(stack), shape=(H, W))
        c, s, m = brute_force(stack, H, W)
        assert np.array_equal(_as(got["count"]), _as(c)), "count vs brute force"
        assert np.array_equal(_as(got["sum"]), _as(s)), "sum vs brute force"
        assert np.array_equal(_as(got["max"]), _as(m)), "max vs brute force"


def pin_exhaustive_binary_2x2():
    """All 2**12 binary ensembles of three 2x2 members.  Member i's pixel j is
    bit 4*i + j of the enumeration index, so the count at pixel j is the
    population count of those three bits."""
    def check(impl):
        for code in range(1 << 12):
            bits = [(code >> b) & 1 for b in range(12)]
            stack = [np.array(bits[4 * i:4 * i + 4], dtype=np.uint8).reshape(2, 2)
                     for i in range(3)]
            got = impl.accumulate(stack, shape=(2, 2))
            for j in range(4):
                pc = bin(code & (0x111 << j)).count("1")
                y, x = divmod(j, 2)
                assert int(got["count"][y, x]) == pc
                assert int(got["sum"][y, x]) == pc
                assert int(got["max"][y, x]) == (1 if pc else 0)
    return check


def pin_library_routines(impl, seed=12):
    """numpy's own reductions over a stacked ensemble."""
    for n, H, W in [(1, 5, 7), (9, 33, 65), (40, 16, 48), (300, 3, 5)]:
        stack = synth.random_members(seed + n, n, H, W)
        got = impl.accumulate(list(stack), shape=(H, W))
        assert np.array_equal(_as(got["count"]), np.count_nonzero(stack, axis=0))
        assert np.array_equal(_as(got["sum"]), stack.sum(axis=0, dtype=np.uint64).astype(np.int64))
        assert np.array_equal(_as(got["max"]), stack.max(axis=0, initial=0).astype(np.int64))


def pin_closed_form(impl, ens: synth.Ensemble):
    """The oracle over a generated ensemble equals LUT[e] of the closed form."""
    e = ens.elevation()
    lv = ens.levels()
    c_lut, s_lut, m_lut = closed_form_lut(lv, ens.kind)
    members = (synth.mask(e, L) if ens.kind == "mask" else synth.depth(e, L) for L in lv)
    got = impl.accumulate(members, shape=e.shape)
    assert np.array_equal(_as(got["count"]), c_lut[e]), "count vs closed form"
    assert np.array_equal(_as(got["sum"]), s_lut[e]), "sum vs closed form"
    assert np.array_equal(_as(got["max"]), m_lut[e]), "max vs closed form"


def pin_invariants(impl, seed=13):
    rng = np.random.default_rng(seed)
    H, W = 13, 29
    A = synth.random_members(seed, 7, H, W)
    B = synth.random_members(seed + 1, 5, H, W)
    full = impl.accumulate(list(A) + list(B), shape=(H, W))
    # empty set
    z = impl.accumulate([], shape=(H, W))
    for k in ("count", "sum", "max"):
        assert not np.any(_as(z[k])), "empty set must give zeros"
    # permutation of members
    perm = rng.permutation(len(A) + len(B))
    allm = list(A) + list(B)
    p = impl.accumulate([allm[i] for i in perm], shape=(H, W))
    for k in ("count", "sum", "max"):
        assert np.array_equal(_as(p[k]), _as(full[k])), "order of members"
    # N identical members
    m = A[0]
    for N in (1, 2, 5):
        r = impl.accumulate([m] * N, shape=(H, W))
        assert np.array_equal(_as(r["count"]), N * (m != 0).astype(np.int64))
        assert np.array_equal(_as(r["sum"]), N * m.astype(np.int64))
        assert np.array_equal(_as(r["max"]), _as(m))
    # additivity over a disjoint union
    ra = impl.accumulate(list(A), shape=(H, W))
    rb = impl.accumulate(list(B), shape=(H, W))
    assert np.array_equal(_as(full["count"]), _as(ra["count"]) + _as(rb["count"]))
    assert np.array_equal(_as(full["sum"]), _as(ra["sum"]) + _as(rb["sum"]))
    assert np.array_equal(_as(full["max"]), np.maximum(_as(ra["max"]), _as(rb["max"])))
    # bounds
    c, s, mx = _as(full["count"]), _as(full["sum"]), _as(full["max"])
    assert np.all(c <= len(allm)) and np.all(c >= 0)
    assert np.all(c <= s) and np.all(s <= 255 * c)
    assert np.array_equal(mx == 0, c == 0)
    # 0/1 members: sum equals count
    bits = (A > 128).astype(np.uint8)
    rbits = impl.accumulate(list(bits), shape=(H, W))
    assert np.array_equal(_as(rbits["sum"]), _as(rbits["count"]))


def pin_multiset(impl, seed=14):
    """add then remove restores the previous state; duplicates are counted."""
    H, W = 9, 11
    R = synth.random_members(seed, 6, H, W)
    ms = impl.Multiset((H, W))
    ms.add([0, 1, 2], [R[0], R[1], R[2]])
    before = {k: _as(v).copy() for k, v in ms.composite().items()}
    ms.add([3, 4, 3], [R[3], R[4], R[3]])
    ms.remove([3, 4, 3])
    after = ms.composite()
    for k in before:
        assert np.array_equal(before[k], _as(after[k])), "add then remove"
    # duplicates: removing one copy keeps the other
    ms.add([5, 5], [R[5], R[5]])
    ms.remove([5])
    once = impl.accumulate([R[0], R[1], R[2], R[5]], shape=(H, W))
    got = ms.composite()
    for k in once:
        assert np.array_equal(_as(once[k]), _as(got[k])), "one of two copies removed"
    assert len(ms) == 4
    # removing an absent id is refused and changes nothing
    try:
        ms.remove([7])
        raise AssertionError("absent id accepted")
    except KeyError:
        pass
    assert len(ms) == 4


def pin_window(impl):
    """A raster whose value encodes its own row and column: the window at
    (x0, y0) of width w and height h starts at row y0, column x0."""
    H, W = 7, 12
    a = (np.arange(H)[:, None] * 16 + np.arange(W)[None, :]).astype(np.uint8)
    x0, y0, w, h = 3, 2, 5, 4
    win = np.asarray(impl.window(a, x0, y0, w, h))
    assert win.shape == (h, w)
    for yy in range(h):
        for xx in range(w):
            assert int(win[yy, xx]) == (y0 + yy) * 16 + (x0 + xx)


def pin_batch(impl, seed=15):
    """Crop of the composite equals the composite of the crops, checked
    against the brute force over the full raster."""
    pool = synth.random_members(seed, 10, 12, 20)
    reqs = [dict(ids=[0, 3, 3, 9], x0=2, y0=1, w=7, h=9),
            dict(ids=[5], x0=0, y0=0, w=20, h=12),
            dict(ids=[], x0=19, y0=11, w=1, h=1),
            dict(ids=[1, 2, 4, 6, 7, 8], x0=13, y0=3, w=6, h=2)]
    got = impl.batch(pool, reqs)
    for r, g in zip(reqs, got):
        c, _, _ = brute_force([pool[i] for i in r["ids"]], 12, 20)
        c = np.array(c, dtype=np.int64)
        exp = c[r["y0"]:r["y0"] + r["h"], r["x0"]:r["x0"] + r["w"]]
        assert np.array_equal(_as(g), exp), "batched crop"


def pin_replay(impl, seed=16):
    """A replayed session equals the closed form over the ids it holds."""
    wl = synth.ServeWorkload(sessions=3, pool=24, H=40, W=48, sigma=4.0,
                             view=16, k_lo=1, k_hi=6, seed=seed)
    e = wl.elevation()
    lv = wl.levels()
    pool = np.stack([synth.depth(e, L) for L in lv])
    sched = wl.schedule(60)
    for sid in range(wl.sessions):
        ops = [r for r in sched if r["sid"] == sid]
        views = impl.replay_session(pool, ops)
        held = []
        for op, v in zip(ops, views):
            if op["op"] == "add":
                held += [int(i) for i in op["ids"]]
            else:
                for i in op["ids"]:
                    held.remove(int(i))
            c_lut, _, _ = closed_form_lut([lv[i] for i in held], "depth")
            ev = e[op["vy0"]:op["vy0"] + op["vh"], op["vx0"]:op["vx0"] + op["vw"]]
            assert np.array_equal(_as(v["count"]), c_lut[ev]), "session replay"


def pin_narrow(impl):
    c = {"count": np.array([0, 65535], dtype=np.int64),
         "sum": np.array([0, (1 << 32) - 1], dtype=np.int64),
         "max": np.array([0, 255], dtype=np.uint8)}
    out = impl.narrow(c, 16)
    assert out["count"].dtype == np.uint16 and int(out["count"][1]) == 65535
    assert out["sum"].dtype == np.uint32 and int(out["sum"][1]) == (1 << 32) - 1
    for bad, bits in (({"count": np.array([65536])}, 16),
                      ({"count": np.array([1 << 32])}, 32),
                      ({"sum": np.array([1 << 32])}, 32),
                      ({"count": np.array([-1])}, 32)):
        try:
            impl.narrow(bad, bits)
            raise AssertionError("out-of-range value accepted")
        except impl.OracleRangeError:
            pass
    out32 = impl.narrow({"count": np.array([70000])}, 32)
    assert out32["count"].dtype == np.uint32 and int(out32["count"][0]) == 70000


def pin_histogram(impl, seed=17):
    """Histogram of the nested-mask count composite: pixels whose elevation e
    satisfies #{i: L_i > e} = k, counted from the histogram of e."""
    ens = synth.PLAIN_SMALL.scaled(N=12, H=64, W=96, sigma=6.0)
    e = ens.elevation()
    lv = ens.levels()
    c_lut, _, _ = closed_form_lut(lv, "mask")
    count = c_lut[e]
    hist = impl.overlap_histogram(count, len(lv) + 1)
    eh = [int(np.sum(e == v)) for v in range(256)]
    exp = [0] * (len(lv) + 1)
    for v in range(256):
        exp[int(c_lut[v])] += eh[v]
    assert [int(h) for h in hist] == exp
    rnd = np.random.default_rng(seed).integers(0, 9, size=(17, 5))
    assert np.array_equal(_as(impl.overlap_histogram(rnd, 9)), np.bincount(rnd.ravel(), minlength=9))


ALL_SMALL = [pin_brute_force, pin_library_routines, pin_invariants, pin_multiset,
             pin_window, pin_batch, pin_replay, pin_narrow, pin_histogram]
