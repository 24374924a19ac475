"""Spatial subdivision on top of the streamed path (Section 1: data too large
for device memory is split spatially and/or processed iteratively as layers).

The raster is cut into bands of whole rows.  Rows [y0, y1) of a row-major
raster are contiguous in host memory, so each band is composited by one
context of W x (y1 - y0) that streams exactly that slice of every member
(iterative subdivision over members inside the context), and the band's
composite is read back into its rows of the host result.  Bands are
independent: a per-pixel composite needs no halo.  Only argument marshalling
happens here; every step runs in the library."""

from __future__ import annotations

from typing import Dict, Sequence

import numpy as np

from .composite import Composite


def composite_banded(host_maps: Sequence, W: int, H: int, band_rows: int,
                     outputs=("count",), count_bits: int = 32, **opts) -> Dict[str, np.ndarray]:
    """Composite of uint8 W x H host rasters (numpy arrays or pinned torch
    tensors, row-major), computed band by band.  Returns host arrays."""
    if band_rows < 1:
        raise ValueError("band_rows must be >= 1")
    for m in host_maps:
        if int(np.prod(m.shape)) != W * H:
            raise ValueError("every member must hold W * H bytes")
    dts = {"count": np.uint16 if count_bits == 16 else np.uint32, "sum": np.uint32, "max": np.uint8}
    out = {k: np.empty((H, W), dtype=dts[k]) for k in outputs}
    flat = [m.reshape(-1) if hasattr(m, "reshape") else m for m in host_maps]
    for y0 in range(0, H, band_rows):
        h = min(band_rows, H - y0)
        with Composite(W, h, outputs, count_bits, **opts) as c:
            c.add([f[y0 * W:(y0 + h) * W] for f in flat])
            for k in outputs:
                c.read(k, out=out[k][y0:y0 + h])
    return out
