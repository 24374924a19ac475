"""Throughput units and the pipeline timing model.

* Throughput is counted in pixel-members: one pixel of one member raster.
  The paper's transfer-rate columns (Section 6.1, the ~4k transfer-rate table
  and the ~2k/~8k one) equal N * W * H bytes of 1-byte pixels divided by the
  run time, with GB = 1e9 bytes, so Gpixel-members/s is the same number as the
  paper's GB/s for uint8 rasters.
* Efficiency (Section 6.1) divides the time of a plain host-to-device copy of
  the same bytes by the pipeline's time, i.e. achieved rate over copy rate.
* The pipeline model of Section 7.1 bounds the time of a staged pipeline in
  which member i needs copy time c_i, transform time m_i and processing time
  p_i: the run takes at least max(c_1 + sum(m + p), sum(c) + m_n + p_n).
* The frame budget of Section 7.1 is the data a pipeline processes within one
  frame at an interactive rate: rate (GB/s) divided by the frame rate.
"""

from __future__ import annotations

from typing import Sequence


def gpx_members_per_s(n_members: int, W: int, H: int, seconds: float) -> float:
    """Gpixel-members per second."""
    return float(n_members) * float(W) * float(H) / float(seconds) / 1e9


def frame_budget_mb(rate_gbps: float, fps: float = 10.0) -> float:
    """MB (1e6 bytes) of 1-byte pixels processed per frame at `fps` frames/s."""
    return float(rate_gbps) * 1e3 / float(fps)


def efficiency(rate: float, copy_rate: float) -> float:
    """Achieved rate over the plain-copy rate of the same bytes."""
    return float(rate) / float(copy_rate)


def pipeline_time(c: Sequence[float], m: Sequence[float], p: Sequence[float]) -> float:
    """Section 7.1 lower bound on the time of the staged pipeline."""
    n = len(c)
    if n == 0:
        return 0.0
    if len(m) != n or len(p) != n:
        raise ValueError("c, m and p must have one entry per member")
    front = c[0] + sum(m) + sum(p)
    back = sum(c) + m[-1] + p[-1]
    return max(front, back)


def simulate_staged(c: Sequence[float], m: Sequence[float], p: Sequence[float],
                    nbuf: int) -> float:
    """Event-by-event time of the staged pipeline with ``nbuf`` staging slots:
    one copy engine, one compute engine; the copy of item i waits for the copy
    of item i-1 and for the release of its slot by item i-nbuf; the transform
    and processing of item i wait for its copy and for item i-1's processing."""
    n = len(c)
    copy_done = [0.0] * n
    proc_done = [0.0] * n
    for i in range(n):
        start = copy_done[i - 1] if i else 0.0
        if i >= nbuf:
            start = max(start, proc_done[i - nbuf])
        copy_done[i] = start + c[i]
        s = max(copy_done[i], proc_done[i - 1] if i else 0.0)
        proc_done[i] = s + m[i] + p[i]
    return proc_done[-1] if n else 0.0
