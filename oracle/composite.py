"""CPU oracle for ensemble compositing.  TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this module.  It shares no code with the HIP library: no kernels, no
helpers, no constants, no pre- or post-processing.  Inputs reach it as plain
numpy arrays.

What it computes (Johnson & Jankun-Kelly, arXiv 2104.14667):

* Section 2 and the caption of Figure 1: N input surfaces (flood extents) are
  combined into one composite image whose value grows with the overlap of the
  surfaces; the user adds and removes surfaces from the working set at will.
* Section 1: the composite is built iteratively, a working composite being
  updated as each layer of data is processed.
* Section 4, the single-buffer and dual-buffer listings (Figures 2 and 3): the
  accumulators are cleared, then each input in turn is folded into them by the
  accumulation kernel.

The paper never writes out the accumulation operator.  This oracle takes the
reading used throughout this repository: per pixel p, over the current
multiset M of members m (uint8 rasters),

    count[p] = #{m in M : m[p] != 0}
    sum[p]   = sum over m in M of m[p]
    max[p]   = max({0} U {m[p] : m in M})

with unbounded (int64) accumulators.  Narrowing to the stored widths is a
separate, checked step (``narrow``).  A remove is never computed by
subtraction here: the composite is recomputed over the multiset that remains.

Every function works member by member, in list order, exactly as the listings
fold inputs one at a time; nothing is blocked, fused or reordered.
"""

from __future__ import annotations

from collections import OrderedDict
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

import numpy as np

OUTPUTS = ("count", "sum", "max")


class OracleRangeError(ValueError):
    """A composite value does not fit the requested stored width."""


def accumulate(members: Iterable[np.ndarray], shape: Optional[Tuple[int, ...]] = None,
               outputs: Sequence[str] = OUTPUTS) -> Dict[str, np.ndarray]:
    """Fold members into cleared accumulators, one member at a time.

    Follows the accumulation loop of Section 4 (Figures 2 and 3): clear, then
    for each input update the composite.  ``members`` is any iterable of uint8
    arrays of one shape (2-D rasters, or 1-D samples of pixels); ``shape`` is
    needed only when the iterable may be empty.  Returns int64 ``count`` and
    ``sum`` and uint8 ``max`` for the requested outputs."""
    for o in outputs:
        if o not in OUTPUTS:
            raise ValueError(f"unknown output {o!r}")
    acc: Dict[str, np.ndarray] = {}
    started = False
    for m in members:
        m = np.asarray(m)
        if m.dtype != np.uint8:
            raise TypeError("members must be uint8")
        if not started:
            if shape is not None and tuple(m.shape) != tuple(shape):
                raise ValueError("member shape differs from the given shape")
            shape = m.shape
            acc = _cleared(shape, outputs)
            started = True
        elif m.shape != shape:
            raise ValueError("members differ in shape")
        if "count" in acc:
            acc["count"] += (m != 0)
        if "sum" in acc:
            acc["sum"] += m
        if "max" in acc:
            acc["max"] = np.maximum(acc["max"], m)
    if not started:
        if shape is None:
            raise ValueError("empty member list needs an explicit shape")
        acc = _cleared(shape, outputs)
    return acc


def _cleared(shape, outputs) -> Dict[str, np.ndarray]:
    """Step 1 of both listings: clear the accumulation buffers."""
    acc = {}
    if "count" in outputs:
        acc["count"] = np.zeros(shape, dtype=np.int64)
    if "sum" in outputs:
        acc["sum"] = np.zeros(shape, dtype=np.int64)
    if "max" in outputs:
        acc["max"] = np.zeros(shape, dtype=np.uint8)
    return acc


def narrow(result: Dict[str, np.ndarray], count_bits: int) -> Dict[str, np.ndarray]:
    """Cast the wide composite to its stored widths, refusing any value that
    does not fit (no saturation, no wrap-around): count to uint16 or uint32,
    sum to uint32, max stays uint8."""
    if count_bits not in (16, 32):
        raise ValueError("count_bits must be 16 or 32")
    out = {}
    for k, v in result.items():
        if k == "count":
            lim = (1 << count_bits) - 1
            dt = np.uint16 if count_bits == 16 else np.uint32
        elif k == "sum":
            lim = (1 << 32) - 1
            dt = np.uint32
        else:
            out[k] = v.astype(np.uint8)
            continue
        if v.size and (int(v.max()) > lim or int(v.min()) < 0):
            raise OracleRangeError(f"{k} out of range for its stored width")
        out[k] = v.astype(dt)
    return out


def window(a: np.ndarray, x0: int, y0: int, w: int, h: int) -> np.ndarray:
    """The part of a row-major raster (rows = y, columns = x) inside a window."""
    H, W = a.shape[-2], a.shape[-1]
    if not (0 <= x0 and 0 <= y0 and w >= 0 and h >= 0 and x0 + w <= W and y0 + h <= H):
        raise ValueError("window outside the raster")
    return a[..., y0:y0 + h, x0:x0 + w]


class Multiset:
    """The working set of the application in Figure 1: surfaces added and
    removed by the user.  Members are keyed by an id; an id may be present
    more than once.  The composite is always recomputed from what is held."""

    def __init__(self, shape: Tuple[int, int]):
        self.shape = tuple(shape)
        self._held: "OrderedDict[int, List[np.ndarray]]" = OrderedDict()

    def add(self, ids: Sequence[int], rasters: Sequence[np.ndarray]) -> None:
        if len(ids) != len(rasters):
            raise ValueError("ids and rasters differ in length")
        for i, r in zip(ids, rasters):
            r = np.asarray(r)
            if r.shape != self.shape or r.dtype != np.uint8:
                raise ValueError("raster shape or dtype mismatch")
            self._held.setdefault(int(i), []).append(r)

    def remove(self, ids: Sequence[int]) -> None:
        need: Dict[int, int] = {}
        for i in ids:
            need[int(i)] = need.get(int(i), 0) + 1
        for i, k in need.items():
            if len(self._held.get(i, [])) < k:
                raise KeyError(f"id {i} is not held {k} time(s)")
        for i, k in need.items():
            del self._held[i][:k]
            if not self._held[i]:
                del self._held[i]

    def __len__(self) -> int:
        return sum(len(v) for v in self._held.values())

    def members(self) -> List[np.ndarray]:
        return [r for rs in self._held.values() for r in rs]

    def composite(self, outputs: Sequence[str] = OUTPUTS) -> Dict[str, np.ndarray]:
        return accumulate(self.members(), shape=self.shape, outputs=outputs)


def batch(pool: np.ndarray, requests: Sequence[dict]) -> List[np.ndarray]:
    """Each request asks for the member count composite of ``pool[ids]``
    restricted to its window; the window applies per pixel, so only the pixels
    inside it are evaluated.  ``pool`` is (P, H, W) uint8 (a numpy memmap or
    array); each request is a dict with ids, x0, y0, w, h.  Returns one int64
    count array (h, w) per request."""
    out = []
    for r in requests:
        x0, y0, w, h = int(r["x0"]), int(r["y0"]), int(r["w"]), int(r["h"])
        crops = (window(pool[int(i)], x0, y0, w, h) for i in r["ids"])
        out.append(accumulate(crops, shape=(h, w), outputs=("count",))["count"])
    return out


def replay_session(pool: np.ndarray, ops: Sequence[dict],
                   outputs: Sequence[str] = ("count",)) -> List[Dict[str, np.ndarray]]:
    """Replays one session's requests in order.  Each op is a dict with op
    ('add' | 'remove'), ids, and a viewport vx0, vy0, vw, vh; after applying
    the op the viewport of the recomputed composite is recorded."""
    H, W = pool.shape[-2], pool.shape[-1]
    ms = Multiset((H, W))
    views = []
    for op in ops:
        ids = [int(i) for i in op["ids"]]
        if op["op"] == "add":
            ms.add(ids, [pool[i] for i in ids])
        elif op["op"] == "remove":
            ms.remove(ids)
        else:
            raise ValueError("op must be add or remove")
        x0, y0, w, h = op["vx0"], op["vy0"], op["vw"], op["vh"]
        crops = (window(m, x0, y0, w, h) for m in ms.members())
        views.append(accumulate(crops, shape=(h, w), outputs=outputs))
    return views


def overlap_histogram(count: np.ndarray, nbins: int) -> np.ndarray:
    """Frequency of each overlap class of a count composite (Figure 1, lower
    left panel): bin k holds the number of pixels covered by exactly k
    members, for k = 0 .. nbins - 1.  A pixel with count >= nbins is an error."""
    c = np.asarray(count).ravel()
    hist = np.zeros(nbins, dtype=np.int64)
    for k in range(nbins):
        hist[k] = int(np.sum(c == k))
    if int(hist.sum()) != c.size:
        raise OracleRangeError("a count falls outside the histogram")
    return hist
