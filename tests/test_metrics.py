"""Units and the pipeline model against the paper's printed numbers (CPU)."""

import json
import os
from collections import defaultdict

import numpy as np
import pytest

from paper_2104_14667_amd import metrics

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_rates.json")))


@pytest.mark.parametrize("row", GOLD["rows"], ids=lambda r: f"{r['set']}-{r['alg']}-{r['N']}")
def test_rate_is_pixel_members_per_second(row):
    # The printed transfer rate is N*W*H one-byte pixels over the run time.
    W, H = GOLD["dims"][row["set"]]
    r = metrics.gpx_members_per_s(row["N"], W, H, row["time_us"] * 1e-6)
    assert abs(r - row["rate_gbs"]) <= 0.0006, (r, row["rate_gbs"])


def test_efficiency_is_rate_over_a_fixed_copy_rate():
    # Efficiency = rate / copy rate: the copy rate it implies is one number
    # per raster size, whatever the algorithm and N.
    implied = defaultdict(list)
    for row in GOLD["rows"]:
        implied[row["set"]].append(row["rate_gbs"] / (row["eff_pct"] / 100.0))
    for s, v in implied.items():
        v = np.array(v)
        assert v.max() / v.min() < 1.004, (s, v)
    # and the copy rate settles near the ~5.1 GB/s plateau of the copy test
    assert 4.6 < np.mean(implied["2k"]) < 4.8
    assert 5.2 < np.mean(implied["4k"]) < 5.4
    assert 5.5 < np.mean(implied["8k"]) < 5.7
    assert metrics.efficiency(4.887, 5.285) == pytest.approx(0.9247, abs=2e-4)


def test_kernel_table_is_self_consistent():
    kt = GOLD["kernel_table"]
    for r in kt["rows"]:
        assert abs(r["total_us"] / kt["runs"] - r["avg_us"]) < 0.5
    img = min(r["total_us"] for r in kt["rows"] if r["kernel"].startswith("image"))
    buf = min(r["total_us"] for r in kt["rows"] if r["kernel"].startswith("buffer"))
    # printed truncated to two decimals: 15.8956...% -> 15.89
    assert 0.0 <= 100.0 * (buf - img) / buf - kt["image_faster_pct"] < 0.01


def test_pipeline_model_special_cases():
    assert metrics.pipeline_time([], [], []) == 0.0
    # one item: copy, transform and process in sequence
    assert metrics.pipeline_time([3.0], [1.0], [2.0]) == 6.0
    # nothing to hide: the copies alone
    assert metrics.pipeline_time([2.0] * 5, [0.0] * 5, [0.0] * 5) == 10.0
    # compute-bound: first copy, then all the work
    assert metrics.pipeline_time([1.0] * 4, [0.5] * 4, [2.0] * 4) == 1.0 + 10.0


@pytest.mark.parametrize("seed", range(20))
def test_pipeline_model_matches_two_slot_simulation_for_uniform_stages(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 40))
    c = float(rng.uniform(0.1, 3.0))
    m = float(rng.uniform(0.0, 1.0))
    p = float(rng.uniform(0.0, 3.0))
    model = metrics.pipeline_time([c] * n, [m] * n, [p] * n)
    sim = metrics.simulate_staged([c] * n, [m] * n, [p] * n, nbuf=2)
    assert sim == pytest.approx(model, rel=1e-12)


@pytest.mark.parametrize("seed", range(20))
def test_pipeline_model_is_a_lower_bound(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(1, 30))
    c, m, p = (list(rng.uniform(0.0, 2.0, n)) for _ in range(3))
    for nbuf in (1, 2, 3):
        assert metrics.simulate_staged(c, m, p, nbuf) >= metrics.pipeline_time(c, m, p) - 1e-12


def test_single_slot_serialises():
    # one slot: copy i+1 waits for processing i, so nothing overlaps
    c, m, p = [2.0] * 6, [0.5] * 6, [1.0] * 6
    assert metrics.simulate_staged(c, m, p, 1) == pytest.approx(6 * 3.5)


def test_sweep_summary_on_a_synthetic_map():
    from paper_2104_14667_amd.experiments import summarize_sweep
    sides = list(range(128, 1025, 128))
    rate = [[(100.0 if W % 256 == 0 else 50.0) for W in sides] for H in sides]
    s = summarize_sweep({"sides": sides, "hi": 1024, "rate_GBps": rate})
    assert s["points"] == 64 and s["max"] == 100.0 and s["min"] == 50.0
    assert s["by_W_mod_256"] == {0: 100.0, 128: 50.0}


def test_bench_traffic_is_null_when_kernel_sources_change(tmp_path, monkeypatch):
    import bench
    f = tmp_path / "t.txt"
    f.write_text(f"# x\nkernel_sources_sha256 = {bench.kernel_source_hash()}   # c\ntraffic_bytes = 123\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic() == 123
    f.write_text("kernel_sources_sha256 = 00\ntraffic_bytes = 123\n")
    assert bench.measured_traffic() is None


def test_frame_budget_reproduces_the_papers_figures():
    """The paper's data-per-frame figures at 10 FPS (Section 7.1) follow from
    its dual-buffer ("2b final") rates at N=100 (its transfer-rate tables)
    within 3%: the budget is the rate times the frame time."""
    from paper_2104_14667_amd.metrics import frame_budget_mb
    fb = GOLD["frame_budget"]
    for size, mb in fb["mb_per_frame"].items():
        row = [r for r in GOLD["rows"] if r["set"] == size and r["alg"] == "2b final" and r["N"] == 100]
        assert len(row) == 1
        got = frame_budget_mb(row[0]["rate_gbs"], fb["fps"])
        assert abs(got - mb) / mb < 0.03, (size, got, mb)
    assert frame_budget_mb(56.0) == 5600.0
    assert frame_budget_mb(1.0, fps=20) == 50.0
