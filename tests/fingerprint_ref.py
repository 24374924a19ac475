"""The member fingerprint of the C ABI (cmp_opts.verify_members), written from
its definition in include/composite.h: the sum over a raster's little-endian
32-bit words d_j (the last zero-padded) of d_j * w_j mod 2^64, where w_j is
Wellons' lowbias32 hash of j with the low bit set.  Test infrastructure only."""

from __future__ import annotations

import numpy as np

M32 = 0xFFFFFFFF


def weight(j: int) -> int:
    x = j & M32
    x ^= x >> 16
    x = (x * 0x7FEB352D) & M32
    x ^= x >> 15
    x = (x * 0x846CA68B) & M32
    x ^= x >> 16
    return x | 1


def fingerprint(raster: np.ndarray) -> int:
    b = np.ascontiguousarray(raster, dtype=np.uint8).ravel()
    pad = (-b.size) % 4
    words = np.concatenate([b, np.zeros(pad, np.uint8)]).view("<u4")
    total = 0
    for j, d in enumerate(words.tolist()):
        if d:
            total += d * weight(j)
    return total % (1 << 64)


def colliding(raster: np.ndarray, j: int, k: int) -> np.ndarray:
    """A different raster with the same fingerprint: word j is raised by w_k
    and word k lowered by w_j (so the sum changes by w_k*w_j - w_j*w_k = 0).
    Word j must be zero and word k all ones."""
    b = np.ascontiguousarray(raster, dtype=np.uint8).ravel()
    pad = (-b.size) % 4
    words = np.concatenate([b, np.zeros(pad, np.uint8)]).view("<u4").copy()
    assert words[j] == 0 and words[k] == M32
    words[j] = weight(k)
    words[k] = M32 - weight(j)
    out = words.view(np.uint8)[: b.size]
    assert np.all(words.view(np.uint8)[b.size:] == 0), "padding must stay zero"
    return out.reshape(raster.shape).copy()


def tile(raster: np.ndarray, tw: int, th: int) -> np.ndarray:
    """The tiled layout of include/composite.h (cmp_layout): tiles of tw bytes
    x th rows, stored tile after tile in row-major tile order, each tile
    row-major, zero padding past the raster's edges; returned flat."""
    H, W = raster.shape
    ntx, nty = -(-W // tw), -(-H // th)
    pad = np.zeros((nty * th, ntx * tw), np.uint8)
    pad[:H, :W] = raster
    return pad.reshape(nty, th, ntx, tw).transpose(0, 2, 1, 3).reshape(-1).copy()


def untile(flat: np.ndarray, W: int, H: int, tw: int, th: int) -> np.ndarray:
    ntx, nty = -(-W // tw), -(-H // th)
    pad = flat.reshape(nty, ntx, th, tw).transpose(0, 2, 1, 3).reshape(nty * th, ntx * tw)
    return pad[:H, :W].copy()
