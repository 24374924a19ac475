"""Spatial subdivision on top of the streamed path (Section 1: data too large
for device memory is split spatially and/or processed iteratively as layers).

The raster is cut into bands of whole rows.  Rows [y0, y1) of a row-major
raster are contiguous in host memory, so each band is composited by a
context of W x (y1 - y0) that streams exactly that slice of every member
(iterative subdivision over members inside the context), and the band's
composite is read back into its rows of the host result.  Bands are
independent: a per-pixel composite needs no halo.  Two contexts per band
height are used in turn (cleared before reuse), so the read-back of one band
runs on a worker thread while the next band uploads: the two directions of
the PCIe link overlap.  There are at most four contexts: two of the full
band's height and two of the ragged last one's.  Only argument marshalling
happens here; every step runs in the library."""

from __future__ import annotations

from concurrent.futures import Future, ThreadPoolExecutor
from typing import Dict, Optional, Sequence, Tuple

import numpy as np

from .composite import Composite


def _page_locked(m) -> bool:
    """True for a torch tensor in page-locked host memory; False for anything
    else (a numpy array may be pageable, so it is treated as such)."""
    f = getattr(m, "is_pinned", None)
    if f is None:
        return False
    try:
        return bool(f())
    except (RuntimeError, TypeError):
        return False


def composite_banded(host_maps: Sequence, W: int, H: int, band_rows: int,
                     outputs=("count",), count_bits: int = 32, out: Optional[Dict] = None,
                     pinned: bool = False, **opts) -> Dict[str, np.ndarray]:
    """Composite of uint8 W x H host rasters (numpy arrays or pinned torch
    tensors, row-major), computed band by band.  Returns host arrays: those of
    `out` (name -> C-contiguous H x W array of the output's dtype) when given,
    which the copy engine fills directly when `pinned` says they are
    page-locked, else new pageable ones.  Members that are not page-locked
    torch tensors are uploaded through the library's pinned bounce buffers
    (opts pageable_host = 1, set here); asking for pageable_host = 0 with such
    members is an error."""
    if band_rows < 1:
        raise ValueError("band_rows must be >= 1")
    if not all(_page_locked(m) for m in host_maps):
        if opts.get("pageable_host", 1) == 0:
            raise ValueError("pageable_host=0 needs page-locked members (pinned torch tensors)")
        opts = dict(opts, pageable_host=1)
    for m in host_maps:
        if int(np.prod(m.shape)) != W * H:
            raise ValueError("every member must hold W * H bytes")
    dts = {"count": np.uint16 if count_bits == 16 else np.uint32, "sum": np.uint32, "max": np.uint8}
    if out is None:
        out = {k: np.empty((H, W), dtype=dts[k]) for k in outputs}
    for k in outputs:
        a = out[k]
        if a.dtype != dts[k] or a.shape != (H, W) or not a.flags.c_contiguous:
            raise ValueError(f"out[{k!r}] must be a C-contiguous (H, W) array of {np.dtype(dts[k])}")
    flat = [m.reshape(-1) if hasattr(m, "reshape") else m for m in host_maps]
    ctxs: Dict[Tuple[int, int], Composite] = {}
    reads: Dict[Tuple[int, int], Future] = {}

    def read_band(c: Composite, y0: int, h: int) -> None:
        for k in outputs:
            c.read(k, out=out[k][y0:y0 + h], pinned=pinned)

    with ThreadPoolExecutor(max_workers=1) as reader:
        try:
            for b, y0 in enumerate(range(0, H, band_rows)):
                h = min(band_rows, H - y0)
                key = (h, b & 1)
                c = ctxs.get(key)
                if c is None:
                    c = ctxs[key] = Composite(W, h, outputs, count_bits, **opts)
                else:
                    reads.pop(key).result()       # its last band is in host memory
                    c.clear()
                c.add([f[y0 * W:(y0 + h) * W] for f in flat])
                reads[key] = reader.submit(read_band, c, y0, h)
            for f in reads.values():
                f.result()
        finally:
            for f in reads.values():
                f.exception()                     # waits; errors already raised above
            for c in ctxs.values():
                c.close()
    return {k: out[k] for k in outputs}
