"""The fingerprint reference used by the member-verification tests: checked
against hand-worked values and the algebra it relies on (CPU)."""

import numpy as np

from fingerprint_ref import colliding, fingerprint, weight


def test_weights_hand_worked():
    assert weight(0) == 1                      # lowbias32(0) = 0, low bit forced
    x = 1
    x ^= x >> 16
    x = (x * 0x7FEB352D) % 2**32               # 0x7feb352d
    assert x == 0x7FEB352D
    x ^= x >> 15                               # 0x7feb352d ^ 0xffd6
    assert x == 0x7FEBCAFB
    x = (x * 0x846CA68B) % 2**32
    x ^= x >> 16
    assert weight(1) == x | 1
    assert all(weight(j) & 1 for j in range(1000))


def test_fingerprint_small_cases():
    assert fingerprint(np.zeros(37, np.uint8)) == 0
    r = np.zeros(12, np.uint8)
    r[0] = 7                                   # word 0 = 7, weight 1
    assert fingerprint(r) == 7
    r[5] = 1                                   # word 1 = 0x100
    assert fingerprint(r) == 7 + 0x100 * weight(1)
    t = np.zeros(9, np.uint8)
    t[8] = 3                                   # ragged: word 2 = 3, zero-padded
    assert fingerprint(t) == 3 * weight(2)
    big = np.full(8, 255, np.uint8)            # exercises the mod 2^64 wrap
    assert fingerprint(big) == (0xFFFFFFFF * (weight(0) + weight(1))) % 2**64


def test_single_word_changes_always_detected():
    rng = np.random.default_rng(0)
    r = rng.integers(0, 256, 203, dtype=np.uint8)
    f = fingerprint(r)
    for pos in (0, 1, 100, 199, 200, 202):
        for delta in (1, 128, 255):
            s = r.copy()
            s[pos] = (int(s[pos]) + delta) % 256
            assert fingerprint(s) != f


def test_colliding_raster_is_different_with_equal_fingerprint():
    r = np.zeros(64, np.uint8)
    r[40:44] = 255                             # word 10 all ones
    c = colliding(r, 3, 10)
    assert not np.array_equal(c, r)
    assert fingerprint(c) == fingerprint(r)


def test_tile_layout_round_trip_and_order():
    from fingerprint_ref import tile, untile
    r = np.arange(37 * 70, dtype=np.int64).reshape(37, 70).astype(np.uint8)
    t = tile(r, 32, 16)                       # 3 x 3 tiles of 32x16
    assert t.size == 9 * 32 * 16
    assert np.array_equal(untile(t, 70, 37, 32, 16), r)
    assert np.array_equal(t[:32], r[0, :32])          # tile 0, row 0
    assert np.array_equal(t[32:64], r[1, :32])        # tile 0, row 1
    assert np.array_equal(t[512:544], r[0, 32:64])    # tile 1, row 0
    assert not t[2 * 512 + 6:2 * 512 + 32].any()       # tile 2, row 0: x 70..95 is padding
