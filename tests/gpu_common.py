"""Shared helpers of the GPU tests: inputs on the device, pinned host copies,
and comparisons against the oracle and the closed form."""

from __future__ import annotations

import functools
import sys

import numpy as np
import torch

import oracle
from paper_2104_14667_amd import synth

from oracle_pins import closed_form_lut


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@functools.lru_cache(maxsize=4)
def elevation_of(ens: synth.Ensemble) -> np.ndarray:
    return ens.elevation()


def device_members(ens: synth.Ensemble, e: np.ndarray, lv) -> torch.Tensor:
    """(N, H, W) uint8 on cuda:0, built member by member on the device."""
    et = torch.from_numpy(e).to("cuda:0")
    out = torch.empty((len(lv), ens.H, ens.W), dtype=torch.uint8, device="cuda:0")
    for i, L in enumerate(lv):
        synth.member_torch(et, int(L), ens.kind, out=out[i])
    torch.cuda.synchronize()   # the library works on its own streams
    return out


def dev_of(a: np.ndarray) -> torch.Tensor:
    t = torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    torch.cuda.synchronize()
    return t


def pinned_copy(t: torch.Tensor) -> torch.Tensor:
    h = torch.empty(t.shape, dtype=t.dtype, pin_memory=True)
    h.copy_(t)
    return h


def expect_oracle(stack: np.ndarray, outputs, count_bits: int) -> dict:
    H, W = stack.shape[1:] if stack.ndim == 3 else (0, 0)
    r = oracle.accumulate(list(stack), shape=stack.shape[1:], outputs=outputs)
    return oracle.narrow(r, count_bits)


def check_full(comp, expected: dict) -> None:
    for name, exp in expected.items():
        got = comp.read(name)
        assert got.dtype == exp.dtype, name
        if not np.array_equal(got, exp):
            bad = np.argwhere(got != exp)
            y, x = bad[0]
            raise AssertionError(f"{name}: {len(bad)} pixels differ, first at (y={y}, x={x}): "
                                 f"got {got[y, x]} expected {exp[y, x]}")


def check_closed_form_and_samples(comp, ens: synth.Ensemble, e: np.ndarray, lv,
                                  n_samples: int = 4096, seed: int = 0) -> None:
    """Every pixel against the closed form, and sampled pixels against the
    oracle evaluated one by one from members rebuilt on the host."""
    c_lut, s_lut, m_lut = closed_form_lut(lv, ens.kind)
    luts = {"count": c_lut, "sum": s_lut, "max": m_lut}
    flat_e = e.ravel()
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, flat_e.size, size=n_samples)
    idx = np.concatenate([idx, [0, ens.W - 1, flat_e.size - ens.W, flat_e.size - 1]])
    es = flat_e[idx]
    make = synth.mask if ens.kind == "mask" else synth.depth
    sample_members = [make(es, int(L)) for L in lv]
    samp = oracle.narrow(oracle.accumulate(sample_members, shape=es.shape,
                                           outputs=ens.outputs), ens.count_bits)
    for name in ens.outputs:
        got = comp.read(name)
        exp = luts[name][e]
        eq = got.astype(np.int64) == exp
        if not eq.all():
            bad = np.argwhere(~eq)
            y, x = bad[0]
            raise AssertionError(f"{name}: {len(bad)} pixels differ from the closed form, first "
                                 f"(y={y}, x={x}) got {got[y, x]} expected {exp[y, x]}")
        g = got.ravel()[idx]
        assert np.array_equal(g, samp[name]), f"{name}: sampled pixels differ from the oracle"
