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


def test_traffic_counters_match_the_kernel_sources(monkeypatch, tmp_path):
    """The committed counter summary carries the hash of the kernel sources it
    was taken on.  It must match the sources as they are: a change to the
    resident kernel's sources needs new FETCH_SIZE / WRITE_SIZE counters.  Its
    traffic figures are used while they match, and dropped (None) once they
    differ or the summary is malformed."""
    kv = {}
    for line in open(bench.TRAFFIC_FILE):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.split("#")[0].strip()
    for pre in ("", "incremental_"):
        assert int(kv[pre + "traffic_bytes"]) == (int(kv[pre + "traffic_read_bytes"])
                                                  + int(kv[pre + "traffic_write_bytes"]))
    assert kv["kernel_sources_sha256"] == bench.kernel_source_hash(), \
        "the resident kernel's sources changed since its HBM counters were taken: take them again"
    assert bench.measured_traffic() == int(kv["traffic_bytes"])
    assert bench.measured_traffic("incremental_traffic_bytes") == int(kv["incremental_traffic_bytes"])
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 64)
    assert bench.measured_traffic() is None
    monkeypatch.undo()
    bad = tmp_path / "traffic.txt"
    bad.write_text(f"kernel_sources_sha256 = {bench.kernel_source_hash()}\n")   # no traffic_bytes
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(bad))
    assert bench.measured_traffic() is None
