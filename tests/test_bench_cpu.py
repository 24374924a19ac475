"""Host helpers of bench.py that its reported figures rest on (CPU)."""

import bench


def test_matrix_unique_bytes_by_hand():
    # tiles of 512 pixels: (y=0, x 0..511) is covered by both requests, whose
    # union is members 0..19; the other three tiles only by the second one
    # (members 5..19); outputs are 4 bytes per window pixel
    reqs = [dict(ids=list(range(10)), x0=0, y0=0, w=100, h=1),
            dict(ids=list(range(5, 20)), x0=500, y0=0, w=100, h=2)]
    reads, writes = bench.matrix_unique_bytes(reqs, W=1024, H=2, P=40)
    assert reads == (20 + 3 * 15) * 512
    assert writes == 4 * (100 * 1 + 100 * 2)


def test_matrix_unique_bytes_ragged_tile_and_uncovered_rows():
    # W = 600: the second tile is 88 pixels wide; the window x 500..599
    # touches both tiles of rows 0 and 1; row 2 is covered by nothing
    reqs = [dict(ids=[3, 1], x0=500, y0=0, w=100, h=2)]
    reads, writes = bench.matrix_unique_bytes(reqs, W=600, H=3, P=4)
    assert reads == 2 * 2 * (512 + 88)
    assert writes == 4 * 100 * 2
    # a window inside the second tile only reads that tile
    reqs = [dict(ids=[3, 1], x0=590, y0=0, w=10, h=2)]
    reads, _ = bench.matrix_unique_bytes(reqs, W=600, H=3, P=4)
    assert reads == 2 * 2 * 88
