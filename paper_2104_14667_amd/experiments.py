"""The paper's experiments, re-run on MI355X through the C ABI.

* ``repack-sweep``: rate of the linear-to-tiled transform over a grid of
  raster dimensions (the buffer-to-image transform test of Section 5.2, whose
  result is the banded rate map of Figure 15): W and H from `lo` to `hi` in
  steps of `step`, one raster per measurement, `reps` timed repetitions.
* ``paper-table``: the dual- and single-buffer streaming runs of Section 5.1
  at the paper's raster sizes (~2k 1856x2208, ~4k 3712x4416, ~8k 7424x8832)
  and N = 10, 100, 1000, with the efficiency of Section 6.1 (rate over the
  rate of a plain host-to-device copy of the same bytes in the same pieces),
  from the best of `reps` timed passes after one warm-up pass, with the
  median and the slowest pass beside it.  With ``--sample-clocks`` each pass
  also reports the graphics and memory clock levels it ran at, as far as the
  driver's sysfs tables are readable.
  The paper's host kept a small set of images and sent them again (8 GB of
  host memory cannot hold 1000 ~8k images); here a ring of 16 distinct pinned
  rasters is sent round-robin.  Variants: "final" (pinned source, staged
  copy then transform to tiles, 1 or 2 staging slots, one raster per slot as
  in the paper), "initial" (pageable source: the host copies every raster
  into a pinned bounce buffer first, as the runtime did behind the paper's
  clWriteImage), and this library's default (linear layout, 8 rasters per
  slot).
* ``kernel-table``: the kernel-runtime comparison of Section 5.3 (its table of
  four kernels): one ~4k raster per launch, 10,000 launches each, timed with
  HIP events around every launch.  Image kernels read images and accumulate
  into two images used in turn; buffer-kernel 1 accumulates in place in one
  buffer, buffer-kernel 2 in two buffers used in turn.  Here: tiled or linear
  device-resident input, and one accumulator in place (cmp_opts.pingpong 0) or
  two used in turn (pingpong 1).  The paper's image-kernel 2 differs from
  image-kernel 1 only in taking the raster size as kernel arguments, which
  HIP kernels always do, so it is the same kernel here.
* ``repack-rate``: the linear-to-tiled transform at fixed shapes: the
  streamed path's chunk (8 rasters of 4096x4096), single rasters of
  8192x8192, and widths that are and are not multiples of 1024 bytes, each
  timed with HIP events over `reps` launches on the launch stream.  The rate
  counts the bytes read (W*H per raster) plus the bytes written (the padded
  tiled plane).  Every output is compared with the layout's definition (tile
  (tx, ty) holds rows ty*th .. and bytes tx*tw .. of the raster, row-major,
  zero past the edges) on sampled tiles.
* ``h2d-sweep``: the host-to-device copy rate of a plain copy from pinned
  memory as a function of buffer size, 64 KiB to 64 MiB in steps of 64 KiB
  (the copy baseline of Section 6, its buffer-size figure).
* ``subdivide``: spatial subdivision (Section 1) at the ~16k raster size the
  paper could not run (14848x17664, 262 MB per mask): N masks, taken
  round-robin from a ring of distinct pinned rasters, composited band by
  band for several band heights, the whole raster (one band) first, into
  pageable and then page-locked host outputs.  Each timing covers the whole
  job: contexts, uploads, compositing and the read-back of every band's count
  into host memory.  Every result is checked
  against its closed form (a pixel's count is the number of members whose
  level exceeds its elevation).

* ``member-layout``: the resident depth workload (N = 128 members of
  8192x8192, count + sum + max) with the members placed in one allocation at a
  stride of 8192^2 + pad bytes, for several pads: the compositing kernel's
  average launch time (HIP events) and the same-traffic reference kernel's
  best time on the same placement.  With pad 0 the same pixel of every member
  lies exactly 64 MiB apart.
* ``pool-layout``: the batched workload (64 crop requests over a pool of 2048
  masks of 2048x2048) with the pool's rasters at a stride of 2048^2 + pad
  bytes, for several pads: the median device time of the library's default
  tune (matrix mode, graph replay), every output checked against its closed
  form.  With pad 0 the same pixel of every raster lies exactly 4 MiB apart.
* ``serve-layout``: the served workload's continuous-batching run for a
  few seconds of its schedule with the pool's depth maps at a stride of
  4096^2 + pad bytes, for several pads, and with several sizes of the
  viewport launch's workgroups (view_group): device time per request, the
  viewport launch's time, p50, p99.
* ``tile-reads``: the batched matrix kernel's read pattern with trivial
  arithmetic over the batched pool's shape, rasters stored one after another
  or row-interleaved (row y of every raster side by side).
* ``two-phase``: the set pass's traffic with the whole grid's reads and
  writes kept apart band by band (grid-wide barriers of a cooperatively
  launched grid), against the same traffic interleaved.
* ``write-mix``: what the composite's read and write cost next to n member
  streams: the same-traffic reference kernel over n members of 8192x8192 with
  member reads only, plus the 9 B/px composite read, plus its write, plus both
  (read-modify-write), for several n, and the write-only mode again with
  each workgroup's member order rotated (starting at member blockIdx mod n),
  and phased: a grid of 2 or 4 workgroups per compute unit whose threads
  read all members for V = 2, 4 or 8 vectors before writing those vectors'
  composite, round after round, and with the members interleaved in 1 KiB
  blocks (a wave's loads of all members walk contiguous memory);
  and a plain fill and copy of the same composite bytes (torch) for scale.

Usage: python -m paper_2104_14667_amd.experiments
           {repack-sweep,repack-rate,paper-table,kernel-table,h2d-sweep,subdivide,
            member-layout,pool-layout,serve-layout,tile-reads,two-phase,write-mix}
           [--out FILE]
"""

from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

PAPER_SIZES = {"2k": (1856, 2208), "4k": (3712, 4416), "8k": (7424, 8832)}


def repack_sweep(lo: int, hi: int, step: int, reps: int, tile=(64, 64)) -> dict:
    import torch

    from .composite import composite_repack_tiled, composite_tiled_bytes
    tw, th = tile
    maxb = hi * hi
    src = torch.zeros(maxb + 64, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty(composite_tiled_bytes(hi, hi, tw, th) + 64, dtype=torch.uint8, device="cuda:0")
    s = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    sides = list(range(lo, hi + 1, step))
    rate = np.zeros((len(sides), len(sides)))
    t0 = time.perf_counter()
    for iy, H in enumerate(sides):
        for ix, W in enumerate(sides):
            tb = composite_tiled_bytes(W, H, tw, th)
            composite_repack_tiled(src, W * H, dst, tb, 1, W, H, tw, th, s)   # warm-up
            ev[0].record(s)
            for _ in range(reps):
                composite_repack_tiled(src, W * H, dst, tb, 1, W, H, tw, th, s)
            ev[1].record(s)
            ev[1].synchronize()
            ms = ev[0].elapsed_time(ev[1]) / reps
            rate[iy, ix] = W * H / (ms * 1e-3) / 1e9
    return {"lo": lo, "hi": hi, "step": step, "reps": reps, "tile": [tw, th],
            "seconds": time.perf_counter() - t0, "sides": sides, "rate_GBps": rate.tolist()}


REPACK_SHAPES = ((4096, 4096, 8), (8192, 8192, 1), (8192, 8192, 8), (8320, 8192, 1), (8000, 8000, 1),
                 (16384, 16384, 1), (16000, 16000, 1), (1856, 2208, 8), (7424, 8832, 1))


def _tiled_reference(a: np.ndarray, tw: int, th: int, tx: int, ty: int) -> np.ndarray:
    """Tile (tx, ty) of raster a as the tiled layout defines it."""
    H, W = a.shape
    t = np.zeros((th, tw), np.uint8)
    blk = a[ty * th:(ty + 1) * th, tx * tw:(tx + 1) * tw]
    t[:blk.shape[0], :blk.shape[1]] = blk
    return t.reshape(-1)


def repack_rate(shapes=REPACK_SHAPES, reps: int = 50, tile=(64, 64), seed: int = 5) -> dict:
    import torch

    from .composite import composite_repack_tiled, composite_tiled_bytes
    tw, th = tile
    rng = np.random.default_rng(seed)
    s = torch.cuda.Stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    rows = []
    for W, H, n in shapes:
        tb = composite_tiled_bytes(W, H, tw, th)
        src = torch.randint(0, 256, (n, H * W), dtype=torch.uint8, device="cuda:0")
        dst = torch.empty((n, tb), dtype=torch.uint8, device="cuda:0")
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            dst.fill_(0xA5)
            composite_repack_tiled(src, W * H, dst, tb, n, W, H, tw, th, s)  # warm-up
            ev[0].record(s)
            for _ in range(reps):
                composite_repack_tiled(src, W * H, dst, tb, n, W, H, tw, th, s)
            ev[1].record(s)
        ev[1].synchronize()
        us = ev[0].elapsed_time(ev[1]) * 1e3 / reps
        # sampled tiles of the first and last raster, edge tiles always included
        ntx, nty = -(-W // tw), -(-H // th)
        picks = {(ntx - 1, nty - 1), (0, 0), (ntx - 1, 0), (0, nty - 1)}
        picks |= {(int(rng.integers(ntx)), int(rng.integers(nty))) for _ in range(12)}
        exact = True
        for i in sorted({0, n - 1}):
            a = src[i].view(H, W).cpu().numpy()
            d = dst[i].cpu().numpy()
            for tx, ty in picks:
                o = (ty * ntx + tx) * tw * th
                exact &= bool(np.array_equal(d[o:o + tw * th], _tiled_reference(a, tw, th, tx, ty)))
        moved = n * (W * H + tb)
        rows.append({"W": W, "H": H, "rasters": n, "W_mod_1024": W % 1024, "launch_us": round(us, 2),
                     "bytes_moved": moved, "GBps": round(moved / (us * 1e-6) / 1e9, 1),
                     "frac_of_8TBps": round(moved / (us * 1e-6) / 8e12, 4), "exact": exact})
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
        del src, dst
    return {"tile": [tw, th], "reps": reps, "rows": rows}


def summarize_sweep(res: dict) -> dict:
    r = np.array(res["rate_GBps"])
    sides = np.array(res["sides"])
    out = {"points": int(r.size), "mean": float(r.mean()), "min": float(r.min()),
           "max": float(r.max()), "p10": float(np.percentile(r, 10)),
           "p90": float(np.percentile(r, 90))}
    big = r[np.ix_(sides >= res["hi"] // 4, sides >= res["hi"] // 4)]
    out["large_mean"] = float(big.mean())
    out["large_cv"] = float(big.std() / big.mean())
    # rate against the width's residue modulo powers of two, large rasters only
    cols = sides >= res["hi"] // 4
    for m in (256, 512, 1024, 2048):
        classes = {}
        for W, c in zip(sides[cols], big.T):
            classes.setdefault(int(W % m), []).append(float(c.mean()))
        out[f"by_W_mod_{m}"] = {k: round(float(np.mean(v)), 1) for k, v in sorted(classes.items())}
        out[f"std_by_W_mod_{m}"] = {k: round(float(np.std(v)), 1) for k, v in sorted(classes.items())}
    return out


def _copy_time(torch, ring, n: int) -> float:
    """Plain pinned host-to-device copy of n rasters taken round-robin from the
    ring, one raster per copy, into two alternating device buffers."""
    plane = ring[0].numel()
    bufs = [torch.empty(plane, dtype=torch.uint8, device="cuda:0") for _ in range(2)]
    s = torch.cuda.Stream()
    best = None
    for _ in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with torch.cuda.stream(s):
            for i in range(n):
                bufs[i & 1].copy_(ring[i % len(ring)].view(-1), non_blocking=True)
        s.synchronize()
        dt = time.perf_counter() - t0
        best = dt if best is None else min(best, dt)
    return best


class ClockSampler:
    """Samples the current graphics and memory clock levels (the DPM tables
    the kernel driver exposes in sysfs, where they are readable) every few
    milliseconds on a thread, so that each timed pass can report the levels it
    ran at."""

    FILES = ("pp_dpm_sclk", "pp_dpm_mclk", "pp_dpm_fclk", "pp_dpm_socclk")

    def __init__(self, period_s: float = 0.005):
        import glob
        import os
        import threading
        self.paths = {}
        for dev in sorted(glob.glob("/sys/class/drm/card*/device")):
            for f in self.FILES:
                path = os.path.join(dev, f)
                try:
                    open(path).read()
                except OSError:
                    continue
                self.paths.setdefault(f, path)
        self.samples = []
        self.period = period_s
        self._stop = threading.Event()
        self._t = threading.Thread(target=self._run, daemon=True)
        if self.paths:
            self._t.start()

    def _run(self):
        while not self._stop.is_set():
            row = {"t": time.perf_counter()}
            for f, path in self.paths.items():
                try:
                    cur = [ln for ln in open(path).read().splitlines() if ln.rstrip().endswith("*")]
                except OSError:
                    continue
                if cur:  # "1: 2397Mhz *" -> 2397
                    row[f] = int("".join(ch for ch in cur[0].split(":")[-1] if ch.isdigit()))
            self.samples.append(row)
            time.sleep(self.period)

    def window(self, t0: float, t1: float) -> dict:
        """min / median / max MHz of each clock over [t0, t1]."""
        out = {}
        for f in self.paths:
            v = [r[f] for r in self.samples if t0 <= r["t"] <= t1 and f in r]
            if v:
                out[f] = {"samples": len(v), "min": min(v), "median": float(np.median(v)), "max": max(v)}
        return out

    def stop(self):
        self._stop.set()
        if self._t.is_alive():
            self._t.join()


def paper_table(Ns=(10, 100, 1000), ring_size: int = 16, sizes=("2k", "4k", "8k"), only=None,
                reps: int = 5, sample_clocks: bool = False) -> dict:
    import torch

    from . import synth
    from .composite import CMP_LINEAR, CMP_TILED, Composite
    rows = []
    clocks = ClockSampler() if sample_clocks else None
    for name in sizes:
        W, H = PAPER_SIZES[name]
        e = synth.elevation(10 + len(name), H, W, 32.0)
        lv = synth.levels(10, ring_size, 64, 192)
        pinned = [torch.from_numpy(synth.mask(e, int(L))).pin_memory() for L in lv]
        pageable = [synth.mask(e, int(L)) for L in lv]
        variants = {
            "1b final": dict(nbuf=1, chunk_depth=1, layout=CMP_TILED, src=pinned),
            "2b final": dict(nbuf=2, chunk_depth=1, layout=CMP_TILED, src=pinned),
            "1b initial": dict(nbuf=1, chunk_depth=1, layout=CMP_TILED, src=pageable, pageable_host=1),
            "2b initial": dict(nbuf=2, chunk_depth=1, layout=CMP_TILED, src=pageable, pageable_host=1),
            "2b linear chunk 8": dict(nbuf=2, chunk_depth=8, layout=CMP_LINEAR, src=pinned),
        }
        if only:
            variants = {k: v for k, v in variants.items() if k in only}
        for N in Ns:
            copy_s = _copy_time(torch, pinned, N)
            copy_rate = N * W * H / copy_s / 1e9
            for vname, kw in variants.items():
                kw = dict(kw)
                src = kw.pop("src")
                maps = [src[i % ring_size] for i in range(N)]
                times, spans = [], []
                with Composite(W, H, ("count",), 32, **kw) as c:
                    for r in range(reps + 1):      # the first pass warms up
                        c.clear()
                        c.sync()
                        t0 = time.perf_counter()
                        c.add(maps)
                        c.sync()
                        if r:
                            times.append(time.perf_counter() - t0)
                            spans.append((t0, t0 + times[-1]))
                t, tmed, tmax = min(times), float(np.median(times)), max(times)
                rate = N * W * H / t / 1e9
                rows.append({"set": name, "N": N, "alg": vname, "reps": reps, "time_us": round(t * 1e6, 1),
                             "median_us": round(tmed * 1e6, 1), "max_us": round(tmax * 1e6, 1),
                             "rate_GBps": round(rate, 3), "copy_GBps": round(copy_rate, 3),
                             "efficiency_pct": round(100 * rate / copy_rate, 2),
                             "median_efficiency_pct": round(100 * N * W * H / tmed / 1e9 / copy_rate, 2)})
                if clocks is not None:
                    rows[-1]["passes"] = [{"ms": round(1e3 * (b - a), 2),
                                           "efficiency_pct": round(100 * N * W * H / (b - a) / 1e9 / copy_rate, 2),
                                           "clocks_MHz": clocks.window(a, b)} for a, b in spans]
                print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    if clocks is not None:
        clocks.stop()
    return {"ring": ring_size, "rows": rows,
            "clock_files": sorted(clocks.paths) if clocks is not None else None}


def kernel_table(size: str = "4k", launches: int = 10000, seed: int = 12) -> dict:
    """Mean kernel time per launch of one raster, for the four kernels."""
    import torch

    from . import synth
    from .composite import (CMP_TILED, Composite, composite_repack_tiled,
                            composite_tiled_bytes)
    W, H = PAPER_SIZES[size]
    tw, th = 64, 64
    e = synth.elevation(seed, H, W, 32.0)
    m = torch.from_numpy(synth.mask(e, 128)).to("cuda:0")
    tb = composite_tiled_bytes(W, H, tw, th)
    tiled = torch.zeros(tb, dtype=torch.uint8, device="cuda:0")
    torch.cuda.synchronize()
    composite_repack_tiled(m, W * H, tiled, tb, 1, W, H, tw, th)
    torch.cuda.synchronize()
    rows = []
    for name, layout, pp in (("image-kernel 1 and 2: tiled input, two accumulators in turn", "tiled", 1),
                             ("buffer-kernel 1: linear input, one accumulator in place", "linear", 0),
                             ("buffer-kernel 2: linear input, two accumulators in turn", "linear", 1),
                             ("tiled input, one accumulator in place (no counterpart)", "tiled", 0)):
        kw = dict(profile=1, pingpong=pp)
        if layout == "tiled":
            kw.update(layout=CMP_TILED, tile_w=tw, tile_h=th)
        src = tiled if layout == "tiled" else m
        with Composite(W, H, ("count",), 32, **kw) as c:
            for _ in range(20):
                c.add_device([src])
            c.sync()
            c.kernel_stats(reset=True)
            t0 = time.perf_counter()
            for _ in range(launches):
                c.add_device([src])
            c.sync()
            wall = time.perf_counter() - t0
            n, ms = c.kernel_stats(reset=True)
            got = c.read("count")
        exact = bool(np.array_equal(got, (launches + 20) * (e < 128).astype(np.uint32)))
        rows.append({"kernel": name, "launches": n, "avg_us": round(ms * 1e3 / n, 2),
                     "total_us": round(ms * 1e3, 0), "wall_per_launch_us": round(wall * 1e6 / launches, 2),
                     "exact": exact})
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    return {"size": size, "W": W, "H": H, "tile": [tw, th], "output": "count u32", "rows": rows}


def h2d_sweep(lo: int = 64 << 10, hi: int = 64 << 20, step: int = 64 << 10, reps: int = 10) -> dict:
    """Plain pinned host-to-device copy rate (GB/s) by buffer size."""
    import torch
    host = torch.empty(hi, dtype=torch.uint8, pin_memory=True)
    host.fill_(1)
    dev = torch.empty(hi, dtype=torch.uint8, device="cuda:0")
    s = torch.cuda.Stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    sizes = list(range(lo, hi + 1, step))
    rate = []
    t0 = time.perf_counter()
    with torch.cuda.stream(s):
        dev[:lo].copy_(host[:lo], non_blocking=True)          # warm-up
        for n in sizes:
            ev[0].record(s)
            for _ in range(reps):
                dev[:n].copy_(host[:n], non_blocking=True)
            ev[1].record(s)
            ev[1].synchronize()
            rate.append(n * reps / (ev[0].elapsed_time(ev[1]) * 1e-3) / 1e9)
    r = np.array(rate)
    big = r[np.array(sizes) >= (8 << 20)]
    return {"sizes": sizes, "GBps": [round(x, 3) for x in rate], "reps": reps,
            "seconds": round(time.perf_counter() - t0, 1),
            "summary": {"at_64KiB": round(float(r[0]), 2), "at_1MiB": round(float(r[15]), 2),
                        "mean_8MiB_up": round(float(big.mean()), 2),
                        "max": round(float(r.max()), 2)}}


def subdivide_table(N: int = 32, ring_size: int = 8, bands=(17664, 8192, 4096, 1024),
                    W: int = 14848, H: int = 17664, reps: int = 3) -> dict:
    """Rate of banded compositing (member bytes per second of the whole job)
    by band height, next to a plain pinned copy of the same rasters."""
    import torch

    from . import synth
    from .subdivide import composite_banded
    t0 = time.perf_counter()
    e = synth.elevation(16, H, W, 64.0)
    lv = synth.levels(16, ring_size, 64, 192)
    ring = [torch.from_numpy(synth.mask(e, int(L))).pin_memory() for L in lv]
    print(json.dumps({"generated_s": round(time.perf_counter() - t0, 1)}), file=sys.stderr, flush=True)
    maps = [ring[i % ring_size] for i in range(N)]
    # closed form of the count: members whose level exceeds the elevation
    used = np.sort(np.array([int(lv[i % ring_size]) for i in range(N)], dtype=np.int64))
    below = np.searchsorted(used, np.arange(256), side="right")       # levels <= v
    expect = (N - below).astype(np.uint32)[e]
    del e
    copy_rate = N * W * H / _copy_time(torch, ring, N) / 1e9
    pinned_out = torch.empty((H, W), dtype=torch.int32, pin_memory=True).numpy().view(np.uint32)
    rows = []
    for dst in ("pageable", "pinned"):
        for band in bands:
            times = []
            for r in range(reps):
                if dst == "pinned":
                    pinned_out.fill(0xFFFFFFFF)
                torch.cuda.synchronize()
                t = time.perf_counter()
                out = composite_banded(maps, W, H, band, out={"count": pinned_out} if dst == "pinned"
                                       else None, pinned=dst == "pinned")
                times.append(time.perf_counter() - t)
                if not np.array_equal(out["count"], expect):
                    raise RuntimeError(f"banded count differs from its closed form (band {band})")
                del out
            t = min(times[1:]) if reps > 1 else times[0]
            rows.append({"output_memory": dst, "band_rows": band, "bands": -(-H // band),
                         "time_ms": round(t * 1e3, 2), "rate_GBps": round(N * W * H / t / 1e9, 3),
                         "copy_GBps": round(copy_rate, 3),
                         "efficiency_pct": round(100 * N * W * H / t / 1e9 / copy_rate, 2),
                         "exact": True})
            print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    return {"W": W, "H": H, "N": N, "ring": ring_size, "output": "count u32", "rows": rows}


def _depth_inputs(n, side, seed=2):
    """Elevation and levels of the depth workload's recipe (sigma 64, levels
    96..224)."""
    from . import synth
    return synth.elevation(seed, side, side, 64.0), synth.levels(seed, n, 96, 224)


def _depth_members(torch, buf, e, lv, stride):
    """The depth members of (e, lv) written at buf + i * stride."""
    from . import synth
    side = e.shape[0]
    et = torch.from_numpy(e).to("cuda:0")
    for i, L in enumerate(lv):
        synth.member_torch(et, int(L), "depth", out=buf[i * stride:i * stride + side * side].view(side, side))
    torch.cuda.synchronize()


def _depth_closed_form(e, lv, times):
    """count, sum and max of `times` passes over members clamp(L - e, 0, 255)."""
    lv = np.asarray(lv, np.int64)
    d = np.clip(lv[None, :] - np.arange(256)[:, None], 0, 255)
    lut = {"count": (d > 0).sum(1) * times, "sum": d.sum(1) * times, "max": d.max(1)}
    return {k: v[e] for k, v in lut.items()}


def member_layout(pads=(0, 4096, 65536, 2 << 20, (2 << 20) + 4096, 64 << 20), n=128, side=8192,
                  reps=10) -> dict:
    import torch

    from .ceiling import same_traffic_ceiling
    from .composite import Composite
    plane = side * side
    buf = torch.empty(n * (plane + max(pads)) + 64, dtype=torch.uint8, device="cuda:0")
    algo = n * plane + 2 * plane * 9
    e, lv = _depth_inputs(n, side)
    rows = []
    for pad in pads:
        stride = plane + pad
        _depth_members(torch, buf, e, lv, stride)
        ptrs = [buf.data_ptr() + i * stride for i in range(n)]
        with Composite(side, side, ("count", "sum", "max"), 32, profile=1) as c:
            for _ in range(2):
                c.add_device(ptrs)
            c.sync()
            c.kernel_stats(reset=True)
            for _ in range(reps):
                c.add_device(ptrs)
            c.sync()
            launches, ms = c.kernel_stats(reset=True)
            exp = _depth_closed_form(e, lv, reps + 2)
            exact = all(np.array_equal(c.read(k).astype(np.int64), exp[k]) for k in exp)
        ceil = same_traffic_ceiling(torch, buf.data_ptr(), stride, n, plane)
        avg = ms / launches
        rows.append({"pad_bytes": pad, "stride_bytes": stride, "kernel_avg_ms": round(avg, 4),
                     "kernel_GBps": round(algo / (avg * 1e-3) / 1e9, 1),
                     "kernel_frac_of_8TBps": round(algo / (avg * 1e-3) / 8e12, 4),
                     "reference_rmw_ms": round(ceil["rmw_ms"], 4),
                     "reference_read_only_ms": round(ceil["read_only_ms"], 4),
                     "reference_read_only_GBps": round(n * plane / (ceil["read_only_ms"] * 1e-3) / 1e9, 1),
                     "exact": exact})
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    return {"n": n, "side": side, "reps": reps, "algorithmic_bytes_per_launch": algo, "rows": rows}


def pool_layout(pads=(0, 4096, 65536, 1 << 20, (1 << 20) + 4096, 4 << 20), reps=10,
                out_layouts=("packed",)) -> dict:
    """The batched workload's default tune (graph replay) with the pool's
    rasters at a stride of 2048^2 + pad bytes, for each pad, and each request's
    u32 output laid out "packed" (rows of w counts back to back) or "lines"
    (rows padded to a multiple of 32 counts and the buffer placed so that
    raster columns that are multiples of 32 start 128-byte lines: the row
    pieces of the kernel's 512-pixel tiles then cover whole lines): median,
    min and max device time per batch; every output checked against its
    closed form."""
    import torch

    from . import synth
    from .composite import CMP_BATCH_MATRIX, Pool
    wl = synth.BATCHED
    e = wl.elevation()
    lv = wl.levels()
    et = torch.from_numpy(e).to("cuda:0")
    plane = wl.H * wl.W
    buf = torch.empty(wl.pool * (plane + max(pads)) + 64, dtype=torch.uint8, device="cuda:0")
    reqs = wl.requests()
    exp = []
    for r in reqs:
        lvs = np.sort(lv[r["ids"]])
        ec = e[r["y0"]:r["y0"] + r["h"], r["x0"]:r["x0"] + r["w"]]
        exp.append(len(lvs) - np.searchsorted(lvs, ec, side="right"))

    def place(layout):
        # each request's output buffer, and the (h, w) view of its counts
        views = []
        for r in reqs:
            h, w = r["h"], r["w"]
            if layout == "packed":
                t = torch.empty((h, w), dtype=torch.int32, device="cuda:0")
                r["out"], r["pitch"], r["buf"] = t, w, t
                views.append(t)
            else:
                pitch, off = (w + 31) // 32 * 32, r["x0"] % 32
                t = torch.empty(h * pitch + 32, dtype=torch.int32, device="cuda:0")  # 256-byte aligned
                r["out"], r["pitch"], r["buf"] = t.data_ptr() + 4 * off, pitch, t
                views.append(t[off:off + h * pitch].view(h, pitch)[:, :w])
        return views

    rows = []
    for pad in pads:
        stride = plane + pad
        for i, L in enumerate(lv):
            synth.member_torch(et, int(L), "mask", out=buf[i * stride:i * stride + plane].view(wl.H, wl.W))
        torch.cuda.synchronize()
        for layout in out_layouts:
            views = place(layout)
            with Pool(buf, wl.pool, wl.W, wl.H, stride, buf.numel()) as pool:
                ms = []
                for _ in range(reps + 1):
                    for r in reqs:
                        r["buf"].fill_(-1)
                    pool.run(reqs)
                    ms.append(pool.last()[0])
                mode = pool.last()[2]
                exact = all(np.array_equal(v.cpu().numpy().view(np.uint32), x) for v, x in zip(views, exp))
            d = np.array(ms[1:])
            rows.append({"pad_bytes": pad, "stride_bytes": stride, "out_layout": layout,
                         "matrix_mode": mode == CMP_BATCH_MATRIX,
                         "device_ms_median": round(float(np.median(d)), 4),
                         "device_ms_min": round(float(d.min()), 4), "device_ms_max": round(float(d.max()), 4),
                         "exact": exact})
            print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    return {"pool": wl.pool, "W": wl.W, "H": wl.H, "requests": len(reqs), "reps": reps, "rows": rows}


def serve_layout(pads=(0, 4096, 65536, 1 << 20), seconds: float = 3.0, check: int = 8,
                 view_groups=(0,)) -> dict:
    """The served workload's continuous-batching run (uint16 composites, an
    8 GiB budget, Poisson 2000 req/s) for `seconds` of its schedule, with the
    pool's depth maps at a stride of 4096^2 + pad bytes and the server's
    view_group (row blocks per workgroup of the viewport launch; 0: the
    library's choice) taking each of `view_groups`: device time per request,
    the viewport launch's time per step, p50 and p99.  `check` sessions' final
    viewports are compared with the closed form of their final members."""
    import torch

    from . import synth
    from .composite import CMP_OP_ADD, Pool, Server
    wl = synth.SERVED
    e = wl.elevation()
    lv = wl.levels()
    et = torch.from_numpy(e).to("cuda:0")
    plane = wl.H * wl.W
    buf = torch.empty(wl.pool * (plane + max(pads)) + 64, dtype=torch.uint8, device="cuda:0")
    sched = wl.schedule(int(wl.rate * seconds))
    budget = wl.sessions // 2 * plane * 4
    ring = [torch.empty((wl.view, wl.view), dtype=torch.int16, pin_memory=True) for _ in range(64)]
    dst = torch.empty((wl.view, wl.view), dtype=torch.int16, pin_memory=True)
    rows = []
    for pad in pads:
        stride = plane + pad
        for i, L in enumerate(lv):
            synth.member_torch(et, int(L), "depth", out=buf[i * stride:i * stride + plane].view(wl.H, wl.W))
        torch.cuda.synchronize()
        for vg in view_groups:
            with Pool(buf, wl.pool, wl.W, wl.H, stride, buf.numel()) as pool:
                with Server(pool, count_bits=16, max_batch=64, overlap=1, hbm_budget_bytes=budget,
                            view_group=vg) as srv:
                    sids = [srv.open() for _ in range(wl.sessions)]
                    st0 = srv.stats()
                    lat, status = srv.replay(sched, sids, ring, wl.view, with_status=True)
                    st = srv.stats()
                    # final members of a few sessions against their closed form
                    cur = [dict() for _ in range(wl.sessions)]
                    for r, g in zip(sched, status):
                        if g != 0:
                            continue
                        c = cur[r["sid"]]
                        for i in (int(x) for x in r["ids"]):
                            c[i] = c.get(i, 0) + (1 if r["op"] == "add" else -1)
                            if c[i] == 0:
                                del c[i]
                    exact = True
                    for k in range(0, wl.sessions, wl.sessions // check):
                        srv.wait(srv.submit(sids[k], CMP_OP_ADD, [], (0, 0, wl.view, wl.view), dst))
                        c = cur[k]
                        lvs = np.sort(np.repeat(lv[list(c)], list(c.values()))) if c else np.zeros(0, lv.dtype)
                        exp = len(lvs) - np.searchsorted(lvs, e[:wl.view, :wl.view], side="right")
                        exact &= bool(np.array_equal(dst.numpy().view(np.uint16), exp))
            ok = status == 0
            lat_ms = lat[ok] / 1e6
            nreq = st["requests"] - st0["requests"]
            nstep = st["steps"] - st0["steps"]
            rows.append({"pad_bytes": pad, "stride_bytes": stride, "view_group": vg,
                         "requests": int(ok.sum()),
                         "device_ms_per_request": round((st["device_ms"] - st0["device_ms"]) / max(1, nreq), 4),
                         "view_launch_ms_per_step": round((st["view_ms"] - st0["view_ms"]) / max(1, nstep), 4),
                         "p50_ms": round(float(np.percentile(lat_ms, 50)), 3),
                         "p99_ms": round(float(np.percentile(lat_ms, 99)), 3), "exact": exact})
            print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    return {"seconds": seconds, "sessions": wl.sessions, "rows": rows}


def tile_reads(blocks_per_cu=(1, 2, 4), pads=(0, 4096), write_segments=(0,)) -> dict:
    """The batched matrix kernel's read pattern (every pool raster's 512-pixel
    piece of every tile, 4 waves per tile) with trivial arithmetic, over the
    batched workload's pool shape (2048 rasters of 2048x2048): rasters stored
    one after another at 4 MiB + pad, or row-interleaved (row y of every
    raster side by side: raster k's row y at (y * 2048 + k) * 2048); with
    each tile also writing each of `write_segments` pieces of 2 KiB (23 is
    the 64-request batch's output volume, 0.386 GB)."""
    import torch

    from . import synth
    from .ceiling import tile_read_ceiling
    wl = synth.BATCHED
    P, W, H = wl.pool, wl.W, wl.H
    plane = W * H
    buf = torch.randint(0, 256, (P * (plane + max(pads)) + 64,), dtype=torch.uint8, device="cuda:0")
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    layouts = [(f"raster-major, stride 4 MiB + {pad}", plane + pad, W) for pad in pads]
    layouts.append(("row-interleaved", W, P * W))
    ntiles = H * ((W + 511) // 512)
    rows = []
    for ws in write_segments:
        for name, stride, pitch in layouts:
            for b in blocks_per_cu:
                ms = tile_read_ceiling(torch, buf.data_ptr(), stride, pitch, P, W, H, cus * b,
                                       write_segments=ws)
                moved = P * plane + ntiles * ws * 2048
                rows.append({"layout": name, "stride_bytes": stride, "row_pitch_bytes": pitch,
                             "workgroups_per_cu": b, "write_segments": ws,
                             "written_bytes": ntiles * ws * 2048, "ms": round(ms, 4),
                             "GBps": round(moved / (ms * 1e-3) / 1e9, 1)})
                print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    return {"pool": P, "W": W, "H": H, "bytes": P * plane, "rows": rows}


def two_phase(n=128, side=8192, configs=((2, 1), (2, 2), (4, 1), (4, 2), (8, 1), (8, 2))) -> dict:
    """The set pass's traffic (n member streams read, the 9 B/px composite
    written) with the grid's reads and writes kept apart by grid-wide
    barriers, band by band, against the same traffic interleaved (mode 4 of
    the reference)."""
    import torch

    from .ceiling import same_traffic_ceiling, two_phase_ceiling
    plane = side * side
    buf = torch.randint(0, 256, (n * plane + 64,), dtype=torch.uint8, device="cuda:0")
    base = same_traffic_ceiling(torch, buf.data_ptr(), plane, n, plane, ((4, "set"), (0, "reads")))
    rows = [{"variant": "interleaved (mode 4)", "ms": round(base["set"], 4)},
            {"variant": "member reads only (mode 0)", "ms": round(base["reads"], 4)}]
    for r in rows:
        print(json.dumps(r), file=sys.stderr, flush=True)
    for V, bpc in configs:
        ms = two_phase_ceiling(torch, buf.data_ptr(), plane, n, plane, V, bpc)
        rows.append({"variant": f"two-phase V={V}, {bpc} workgroups per CU", "V": V, "workgroups_per_cu": bpc,
                     "bands": -(-plane // 16 // (torch.cuda.get_device_properties(0).multi_processor_count
                                                  * bpc * 256 * V)), "ms": round(ms, 4)})
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    algo = n * plane + 9 * plane
    for r in rows:
        r["GBps_of_set_pass_bytes"] = round(algo / (r["ms"] * 1e-3) / 1e9, 1)
    return {"members": n, "side": side, "rows": rows}


def write_mix(ns=(16, 64, 128), side=8192, pad=0) -> dict:
    import torch

    from .ceiling import same_traffic_ceiling
    plane = side * side
    stride = plane + pad
    buf = torch.empty(max(ns) * stride + 64, dtype=torch.uint8, device="cuda:0")
    e, lv = _depth_inputs(max(ns), side)
    _depth_members(torch, buf, e, lv, stride)
    comp = 9 * plane
    rows = []
    for n in ns:
        t = same_traffic_ceiling(torch, buf.data_ptr(), stride, n, plane,
                                 ((0, "reads"), (5, "reads+composite_read"),
                                  (4, "reads+composite_write"), (1, "reads+rmw"),
                                  (6, "rotated_reads+composite_write"),
                                  (7, "phased_V2_2wg+composite_write"), (8, "phased_V4_2wg+composite_write"),
                                  (9, "phased_V8_2wg+composite_write"), (10, "phased_V2_4wg+composite_write"),
                                  (11, "phased_V4_4wg+composite_write"), (12, "phased_V8_4wg+composite_write"),
                                  (13, "interleaved_reads+composite_write")))
        row = {"members": n, "member_GB": round(n * plane / 1e9, 3), "composite_GB": round(comp / 1e9, 3)}
        row.update({k + "_ms": round(v, 4) for k, v in t.items()})
        row["read_cost_ms_per_GB"] = round((t["reads+composite_read"] - t["reads"]) / (comp / 1e9), 3)
        row["write_cost_ms_per_GB"] = round((t["reads+composite_write"] - t["reads"]) / (comp / 1e9), 3)
        row["rmw_cost_ms_per_GB_moved"] = round((t["reads+rmw"] - t["reads"]) / (2 * comp / 1e9), 3)
        row["member_read_GBps"] = round(n * plane / (t["reads"] * 1e-3) / 1e9, 1)
        rows.append(row)
        print(json.dumps(row), file=sys.stderr, flush=True)
    # plain fill and copy of the composite's bytes, for scale
    a = torch.empty(comp, dtype=torch.uint8, device="cuda:0")
    b = torch.empty(comp, dtype=torch.uint8, device="cuda:0")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    plain = {}
    for name, fn in (("fill", lambda: a.fill_(3)), ("copy", lambda: b.copy_(a))):
        best = None
        for _ in range(6):
            ev[0].record()
            fn()
            ev[1].record()
            ev[1].synchronize()
            ms = ev[0].elapsed_time(ev[1])
            best = ms if best is None else min(best, ms)
        plain[name + "_ms"] = round(best, 4)
    plain["fill_GBps"] = round(comp / (plain["fill_ms"] * 1e-3) / 1e9, 1)
    plain["copy_GBps"] = round(2 * comp / (plain["copy_ms"] * 1e-3) / 1e9, 1)
    return {"side": side, "stride_bytes": stride, "rows": rows, "plain": plain}


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("repack-sweep")
    a.add_argument("--lo", type=int, default=128)
    a.add_argument("--hi", type=int, default=16384)
    a.add_argument("--step", type=int, default=128)
    a.add_argument("--reps", type=int, default=3)
    a.add_argument("--out", default=None)
    b = sub.add_parser("paper-table")
    b.add_argument("--ns", default="10,100,1000")
    b.add_argument("--sizes", default="2k,4k,8k")
    b.add_argument("--variants", default=None, help="comma-separated variant names (default: all)")
    b.add_argument("--reps", type=int, default=5)
    b.add_argument("--sample-clocks", action="store_true",
                   help="report the clock levels (sysfs DPM tables) seen during each timed pass")
    b.add_argument("--out", default=None)
    rr = sub.add_parser("repack-rate")
    rr.add_argument("--reps", type=int, default=50)
    rr.add_argument("--out", default=None)
    c = sub.add_parser("kernel-table")
    c.add_argument("--size", default="4k", choices=sorted(PAPER_SIZES))
    c.add_argument("--launches", type=int, default=10000)
    c.add_argument("--out", default=None)
    d = sub.add_parser("h2d-sweep")
    d.add_argument("--reps", type=int, default=10)
    d.add_argument("--out", default=None)
    f = sub.add_parser("subdivide")
    f.add_argument("--n", type=int, default=32)
    f.add_argument("--bands", default="17664,8192,4096,1024")
    f.add_argument("--out", default=None)
    g = sub.add_parser("member-layout")
    g.add_argument("--pads", default=None, help="comma-separated pads in bytes")
    g.add_argument("--reps", type=int, default=10)
    g.add_argument("--out", default=None)
    pl = sub.add_parser("pool-layout")
    pl.add_argument("--pads", default=None, help="comma-separated pads in bytes")
    pl.add_argument("--reps", type=int, default=10)
    pl.add_argument("--out-layouts", default=None, help="comma-separated: packed, lines")
    pl.add_argument("--out", default=None)
    sl = sub.add_parser("serve-layout")
    sl.add_argument("--pads", default=None, help="comma-separated pads in bytes")
    sl.add_argument("--seconds", type=float, default=3.0)
    sl.add_argument("--view-groups", default=None,
                    help="comma-separated view_group values (0: the library's choice)")
    sl.add_argument("--out", default=None)
    tr = sub.add_parser("tile-reads")
    tr.add_argument("--write-segments", default=None,
                    help="comma-separated 2 KiB pieces written per tile (23: the batch's outputs)")
    tr.add_argument("--out", default=None)
    tp = sub.add_parser("two-phase")
    tp.add_argument("--out", default=None)
    w = sub.add_parser("write-mix")
    w.add_argument("--ns", default="16,64,128")
    w.add_argument("--pad", type=int, default=0)
    w.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    if args.cmd == "repack-sweep":
        res = repack_sweep(args.lo, args.hi, args.step, args.reps)
        res["summary"] = summarize_sweep(res)
        print(json.dumps(res["summary"]))
    elif args.cmd == "repack-rate":
        res = repack_rate(reps=args.reps)
        print(json.dumps(res))
    elif args.cmd == "kernel-table":
        res = kernel_table(args.size, args.launches)
        print(json.dumps(res))
    elif args.cmd == "h2d-sweep":
        res = h2d_sweep(reps=args.reps)
        print(json.dumps(res["summary"]))
    elif args.cmd == "subdivide":
        res = subdivide_table(args.n, bands=tuple(int(x) for x in args.bands.split(",")))
        print(json.dumps(res))
    elif args.cmd == "member-layout":
        kw = {"reps": args.reps}
        if args.pads:
            kw["pads"] = tuple(int(x) for x in args.pads.split(","))
        res = member_layout(**kw)
        print(json.dumps(res))
    elif args.cmd == "pool-layout":
        kw = {"reps": args.reps}
        if args.pads:
            kw["pads"] = tuple(int(x) for x in args.pads.split(","))
        if args.out_layouts:
            kw["out_layouts"] = tuple(args.out_layouts.split(","))
        res = pool_layout(**kw)
        print(json.dumps(res))
    elif args.cmd == "serve-layout":
        kw = {"seconds": args.seconds}
        if args.pads:
            kw["pads"] = tuple(int(x) for x in args.pads.split(","))
        if args.view_groups:
            kw["view_groups"] = tuple(int(x) for x in args.view_groups.split(","))
        res = serve_layout(**kw)
        print(json.dumps(res))
    elif args.cmd == "tile-reads":
        kw = {}
        if args.write_segments:
            kw["write_segments"] = tuple(int(x) for x in args.write_segments.split(","))
        res = tile_reads(**kw)
        print(json.dumps(res))
    elif args.cmd == "two-phase":
        res = two_phase()
        print(json.dumps(res))
    elif args.cmd == "write-mix":
        res = write_mix(tuple(int(x) for x in args.ns.split(",")), pad=args.pad)
        print(json.dumps(res))
    else:
        res = paper_table(tuple(int(x) for x in args.ns.split(",")),
                          sizes=tuple(args.sizes.split(",")),
                          only=tuple(args.variants.split(",")) if args.variants else None,
                          reps=args.reps, sample_clocks=args.sample_clocks)
        print(json.dumps(res))
    if args.out:
        json.dump(res, open(args.out, "w"))


if __name__ == "__main__":
    main()
