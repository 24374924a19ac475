"""Autotuner of the batched launch.

Persistent mode: sweeps the work-item size (16-pixel vectors per item), the
occupancy (workgroups per compute unit), the queue order (largest items first,
or top to bottom through the raster so that requests sharing members hit in
the caches) and the load hint (non-temporal or cached).  Shared mode: sweeps
the requests per pass over a tile (fewer use less LDS, so more workgroups fit,
but re-read members where many requests overlap), the occupancy and the load
hint; it is skipped when the batch does not qualify (a request repeating an
id).  Matrix mode: sweeps the occupancy (one or two workgroups per compute
unit) and the load hint, and is skipped when the batch or pool does not
qualify.  Each candidate runs on the actual batch, timed with the library's own
event timing, and the fastest is kept.  Results
are cached per shape class (arch, raster size, request count, typical window
side and set size, each bucketed to a power of two) in memory and, when a path
is given, in a JSON file."""

from __future__ import annotations

import json
import math
import os
import time
from typing import Dict, Optional, Sequence

from .composite import (CMP_BATCH_MATRIX, CMP_BATCH_PERSISTENT, CMP_BATCH_SHARED, CMP_ORDER_COST,
                        CMP_ORDER_ROWS, Pool, make_tune)

TILE_VECS = (64, 128, 256, 512, 1024, 2048, 4096)
BLOCKS_PER_CU = (1, 2, 4, 8, 16)
ORDERS = (CMP_ORDER_COST, CMP_ORDER_ROWS)
STREAM_LOADS = (0, 1)
SHARED_SLOTS = (0, 24, 20, 16)
SHARED_BLOCKS_PER_CU = (2, 3, 4, 6)
MATRIX_BLOCKS_PER_CU = (1, 2)

_cache: Dict[str, dict] = {}


def _bucket(x: float) -> int:
    return 1 << max(0, int(round(math.log2(max(1.0, x)))))


def shape_key(pool: Pool, requests: Sequence[dict], arch: str = "gfx950") -> str:
    nreq = len(requests)
    side = sum((r["w"] * r["h"]) ** 0.5 for r in requests) / max(1, nreq)
    n = sum(len(r["ids"]) for r in requests) / max(1, nreq)
    return f"{arch}/W{pool.W}xH{pool.H}/req{_bucket(nreq)}/side{_bucket(side)}/n{_bucket(n)}"


def autotune(pool: Pool, requests: Sequence[dict], reps: int = 3,
             cache_path: Optional[str] = None, use_graph: int = 1) -> dict:
    """Returns {'mode', 'tile_vecs', 'blocks_per_cu', 'order', 'stream_loads',
    'slots', 'ms', 'by_mode', 'key', 'seconds', 'cached'}: the fastest candidate,
    and in 'by_mode' the fastest of each mode that ran (keyed by mode number)."""
    key = shape_key(pool, requests)
    if cache_path and os.path.exists(cache_path) and not _cache:
        try:
            _cache.update(json.load(open(cache_path)))
        except (OSError, ValueError):
            pass
    if key in _cache:
        return dict(_cache[key], key=key, cached=True, seconds=0.0)
    t0 = time.perf_counter()
    best = None
    by_mode: Dict[str, dict] = {}

    def trial(mode, tv, bpc, order, sl, slots):
        nonlocal best
        tune = make_tune(mode, tv, bpc, use_graph, order, sl, slots)
        ms = []
        for _ in range(reps):
            pool.run(requests, tune)
            ms.append(pool.last()[0])
        if pool.last()[2] != mode:
            return False                      # the batch does not qualify
        m = min(ms)
        cand = {"mode": mode, "tile_vecs": tv, "blocks_per_cu": bpc, "order": order,
                "stream_loads": sl, "slots": slots, "ms": m}
        if best is None or m < best["ms"]:
            best = cand
        if str(mode) not in by_mode or m < by_mode[str(mode)]["ms"]:
            by_mode[str(mode)] = cand
        return True

    for order in ORDERS:
        for sl in STREAM_LOADS:
            for tv in TILE_VECS:
                for bpc in BLOCKS_PER_CU:
                    trial(CMP_BATCH_PERSISTENT, tv, bpc, order, sl, 0)
    # the shared mode's fallback uses the best persistent parameters
    fb = dict(by_mode[str(CMP_BATCH_PERSISTENT)])
    shared_ok = True
    for slots in SHARED_SLOTS:
        for bpc in SHARED_BLOCKS_PER_CU:
            for sl in STREAM_LOADS:
                if shared_ok:
                    shared_ok = trial(CMP_BATCH_SHARED, fb["tile_vecs"], bpc, fb["order"], sl, slots)
    # the matrix mode (its fallback: the shared mode with these parameters)
    matrix_ok = True
    for bpc in MATRIX_BLOCKS_PER_CU:
        for sl in STREAM_LOADS:
            if matrix_ok:
                matrix_ok = trial(CMP_BATCH_MATRIX, fb["tile_vecs"], bpc, fb["order"], sl, 0)
    best = dict(best, by_mode=by_mode)
    _cache[key] = best
    if cache_path:
        try:
            json.dump(_cache, open(cache_path, "w"), indent=1, sort_keys=True)
        except OSError:
            pass
    return dict(best, key=key, cached=False, seconds=time.perf_counter() - t0)
