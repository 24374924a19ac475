"""Seeded synthetic ensembles of flood rasters.

The paper's flood-extent data (simulated and observed extents over LIDAR
terrain, Section 2) is not available, so every input here is generated from a
seed.  The recipe:

* an elevation field ``e``: float64 standard-normal white noise drawn from
  ``numpy.random.Generator(PCG64)``, smoothed with a periodic Gaussian of
  standard deviation ``sigma`` pixels (applied in the Fourier domain, i.e. a
  wrap-around convolution with the untruncated kernel), min-max scaled to
  [0, 255] and rounded half-to-even to uint8;
* per-member water levels ``L_i``: integers drawn uniformly, bounds inclusive;
* a flood-extent member is the binary mask ``e < L_i`` (uint8 0/1);
* a flood-depth member is ``clamp(L_i - e, 0, 255)`` (uint8).

All members of one ensemble share the one elevation field, as real ensembles
over one terrain do.

This module is the only code that both the oracle side and the HIP side use:
it produces inputs and holds none of the compositing arithmetic.  Torch
helpers build the same members on the device with integer operations that are
bit-identical to the numpy ones (a CPU test checks this).
"""

from __future__ import annotations

import hashlib
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

# SeedSequence children, one per independent stream of one seed.
_NOISE, _LEVELS, _REQUESTS, _SCHEDULE = range(4)


def _rng(seed: int, stream: int) -> np.random.Generator:
    child = np.random.SeedSequence(int(seed)).spawn(4)[stream]
    return np.random.Generator(np.random.PCG64(child))


def elevation(seed: int, H: int, W: int, sigma: float) -> np.ndarray:
    """Seeded smoothed elevation field, uint8 of shape (H, W)."""
    rng = _rng(seed, _NOISE)
    noise = rng.standard_normal((H, W))
    spec = np.fft.rfft2(noise)
    del noise
    fy = np.fft.fftfreq(H)[:, None]
    fx = np.fft.rfftfreq(W)[None, :]
    spec *= np.exp(-2.0 * np.pi ** 2 * float(sigma) ** 2 * (fy ** 2 + fx ** 2))
    smooth = np.fft.irfft2(spec, s=(H, W))
    del spec
    lo = float(smooth.min())
    hi = float(smooth.max())
    if hi <= lo:
        return np.zeros((H, W), dtype=np.uint8)
    smooth -= lo
    smooth *= 255.0 / (hi - lo)
    np.rint(smooth, out=smooth)
    np.clip(smooth, 0.0, 255.0, out=smooth)
    return smooth.astype(np.uint8)


def levels(seed: int, n: int, lo: int, hi: int) -> np.ndarray:
    """``n`` water levels drawn uniformly from the integers lo..hi inclusive."""
    rng = _rng(seed, _LEVELS)
    return rng.integers(lo, hi + 1, size=int(n)).astype(np.int64)


def mask(elev: np.ndarray, level: int) -> np.ndarray:
    """Binary flood extent of one member: 1 where elev < level."""
    return (elev.astype(np.int16) < int(level)).astype(np.uint8)


def depth(elev: np.ndarray, level: int) -> np.ndarray:
    """Quantized flood depth of one member: clamp(level - elev, 0, 255)."""
    d = np.int16(level) - elev.astype(np.int16)
    return np.clip(d, 0, 255).astype(np.uint8)


def members(elev: np.ndarray, lv: Sequence[int], kind: str) -> np.ndarray:
    """Stack of members, shape (n, H, W) uint8; ``kind`` is 'mask' or 'depth'."""
    make = mask if kind == "mask" else depth
    out = np.empty((len(lv),) + elev.shape, dtype=np.uint8)
    for i, L in enumerate(lv):
        out[i] = make(elev, int(L))
    return out


def member_torch(elev_t, level: int, kind: str, out=None):
    """Device version of :func:`mask` / :func:`depth` for one member.

    ``elev_t`` is a uint8 torch tensor; the result is uint8 on its device."""
    import torch

    if kind == "mask":
        r = (elev_t.to(torch.int16) < int(level)).to(torch.uint8)
    else:
        r = (int(level) - elev_t.to(torch.int16)).clamp_(0, 255).to(torch.uint8)
    if out is not None:
        out.copy_(r)
        return out
    return r


def random_members(seed: int, n: int, H: int, W: int,
                   p_zero: float = 0.3) -> np.ndarray:
    """Unstructured uint8 members with exact zeros and the extreme value 255.

    Used for edge cases the smooth generator does not reach."""
    rng = _rng(seed, _NOISE)
    x = rng.integers(0, 256, size=(n, H, W), dtype=np.uint8)
    z = rng.random((n, H, W)) < p_zero
    x[z] = 0
    hot = rng.random((n, H, W)) < 0.05
    x[hot] = 255
    return x


def sha256(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


# ---------------------------------------------------------------------------
# The five workloads.  Each dataclass holds the recipe of one workload with the
# sizes it is specified at; ``scaled`` returns the same recipe at other sizes
# for tests that must finish on the CPU.

@dataclass(frozen=True)
class Ensemble:
    """N members of W x H from one shared elevation field."""
    name: str
    N: int
    H: int
    W: int
    sigma: float
    level_lo: int
    level_hi: int
    kind: str              # 'mask' or 'depth'
    outputs: tuple         # subset of ('count', 'sum', 'max')
    count_bits: int
    seed: int

    def elevation(self) -> np.ndarray:
        return elevation(self.seed, self.H, self.W, self.sigma)

    def levels(self) -> np.ndarray:
        return levels(self.seed, self.N, self.level_lo, self.level_hi)

    def scaled(self, N: Optional[int] = None, H: Optional[int] = None,
               W: Optional[int] = None, sigma: Optional[float] = None) -> "Ensemble":
        return Ensemble(self.name, N or self.N, H or self.H, W or self.W,
                        sigma or self.sigma, self.level_lo, self.level_hi,
                        self.kind, self.outputs, self.count_bits, self.seed)


PLAIN_SMALL = Ensemble("plain-small N=16 512x512 mask", 16, 512, 512, 16.0,
                       64, 192, "mask", ("count",), 16, seed=0)
STREAMED = Ensemble("streamed N=256 4096x4096 mask", 256, 4096, 4096, 64.0,
                    64, 192, "mask", ("count",), 32, seed=1)
DEPTH = Ensemble("depth N=128 8192x8192", 128, 8192, 8192, 64.0,
                 96, 224, "depth", ("count", "sum", "max"), 32, seed=2)


@dataclass
class BatchWorkload:
    """Many crop requests against one device-resident pool of binary maps."""
    name: str = "batched 64 req, pool 2048 x 2048x2048 mask"
    pool: int = 2048
    H: int = 2048
    W: int = 2048
    sigma: float = 16.0
    level_lo: int = 64
    level_hi: int = 192
    nreq: int = 64
    n_lo: int = 4
    n_hi: int = 512
    side_lo: int = 512
    side_hi: int = 2048
    seed: int = 3

    def elevation(self) -> np.ndarray:
        return elevation(self.seed, self.H, self.W, self.sigma)

    def levels(self) -> np.ndarray:
        return levels(self.seed, self.pool, self.level_lo, self.level_hi)

    def requests(self) -> List[dict]:
        """Each request: ids (int32, without replacement), x0, y0, side."""
        rng = _rng(self.seed, _REQUESTS)
        out = []
        for _ in range(self.nreq):
            n = int(rng.integers(self.n_lo, min(self.n_hi, self.pool) + 1))
            ids = rng.choice(self.pool, size=n, replace=False).astype(np.int32)
            side = int(rng.integers(self.side_lo, self.side_hi + 1))
            side = min(side, self.W, self.H)
            x0 = int(rng.integers(0, self.W - side + 1))
            y0 = int(rng.integers(0, self.H - side + 1))
            out.append(dict(ids=ids, x0=x0, y0=y0, w=side, h=side))
        return out

    def scaled(self, **kw) -> "BatchWorkload":
        d = dict(self.__dict__)
        d.update(kw)
        return BatchWorkload(**d)


@dataclass
class ServeWorkload:
    """Open-loop Poisson add/remove/read requests over per-session composites."""
    name: str = "served 256 sessions 4096x4096 count, pool 1024 depth maps"
    sessions: int = 256
    pool: int = 1024
    H: int = 4096
    W: int = 4096
    sigma: float = 64.0
    level_lo: int = 96
    level_hi: int = 224
    rate: float = 2000.0
    duration_s: float = 20.0
    k_lo: int = 1
    k_hi: int = 32
    p_add: float = 0.6
    view: int = 1024
    seed: int = 4

    def elevation(self) -> np.ndarray:
        return elevation(self.seed, self.H, self.W, self.sigma)

    def levels(self) -> np.ndarray:
        return levels(self.seed, self.pool, self.level_lo, self.level_hi)

    def schedule(self, n_requests: Optional[int] = None) -> List[dict]:
        """Requests in arrival order.

        Each: t (seconds from start), sid, op ('add' | 'remove'), ids, vx0,
        vy0, vw, vh.  An add draws ids absent from the session; a remove of
        more members than the session holds removes all of them; a remove on
        an empty session becomes an add, and an add on a session that holds
        the whole pool becomes a remove.  Session membership is tracked here
        only to draw valid requests."""
        rng = _rng(self.seed, _SCHEDULE)
        n = n_requests if n_requests is not None else int(self.rate * self.duration_s)
        held = [set() for _ in range(self.sessions)]
        order = [[] for _ in range(self.sessions)]   # insertion order per session
        t = 0.0
        out = []
        view = min(self.view, self.W, self.H)
        for _ in range(n):
            t += float(rng.exponential(1.0 / self.rate))
            sid = int(rng.integers(0, self.sessions))
            k = int(rng.integers(self.k_lo, self.k_hi + 1))
            op = "add" if rng.random() < self.p_add else "remove"
            if op == "remove" and not held[sid]:
                op = "add"
            elif op == "add" and len(held[sid]) >= self.pool:
                op = "remove"
            if op == "add":
                free = np.setdiff1d(np.arange(self.pool), np.fromiter(held[sid], dtype=np.int64, count=len(held[sid])))
                k = min(k, len(free))
                ids = rng.choice(free, size=k, replace=False).astype(np.int32)
                held[sid].update(int(i) for i in ids)
                order[sid].extend(int(i) for i in ids)
            else:
                cur = np.array(order[sid], dtype=np.int32)
                if k >= len(cur):
                    ids = cur.copy()
                else:
                    ids = rng.choice(cur, size=k, replace=False).astype(np.int32)
                for i in ids:
                    held[sid].discard(int(i))
                gone = set(int(i) for i in ids)
                order[sid] = [i for i in order[sid] if i not in gone]
            vx0 = int(rng.integers(0, self.W - view + 1))
            vy0 = int(rng.integers(0, self.H - view + 1))
            out.append(dict(t=t, sid=sid, op=op, ids=ids, vx0=vx0, vy0=vy0,
                            vw=view, vh=view))
        return out

    def scaled(self, **kw) -> "ServeWorkload":
        d = dict(self.__dict__)
        d.update(kw)
        return ServeWorkload(**d)


BATCHED = BatchWorkload()
SERVED = ServeWorkload()
