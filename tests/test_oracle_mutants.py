"""Planted mistakes in copies of the oracle must each be caught by a pin.

The mistakes are made on the CPU, in this file, to oracle functions; the real
oracle is untouched.  A pin that lets a plausible slip through (a dropped
member, a wrong comparison, a transposed window, a wrong multiplicity) would
make parity against the oracle meaningless."""

import types

import numpy as np
import pytest

import oracle
from oracle import composite as oc
from paper_2104_14667_amd import synth

from oracle_pins import (ALL_SMALL, pin_closed_form, pin_exhaustive_binary_2x2)


def _impl(**override):
    ns = types.SimpleNamespace(
        accumulate=oc.accumulate, narrow=oc.narrow, window=oc.window,
        Multiset=oc.Multiset, batch=oc.batch, replay_session=oc.replay_session,
        overlap_histogram=oc.overlap_histogram,
        OracleRangeError=oc.OracleRangeError)
    for k, v in override.items():
        setattr(ns, k, v)
    return ns


def _acc_variant(count_pred=None, skip_first=False, max_fn=np.maximum,
                 sum_shift=0):
    def accumulate(members, shape=None, outputs=oc.OUTPUTS):
        members = list(members)
        if not members:
            return oc.accumulate([], shape=shape, outputs=outputs)
        if skip_first:
            members = members[1:]
            if not members:
                return oc.accumulate([], shape=shape, outputs=outputs)
        acc = oc._cleared(members[0].shape, outputs)
        for m in members:
            if "count" in acc:
                acc["count"] += count_pred(m) if count_pred else (m != 0)
            if "sum" in acc:
                acc["sum"] += m.astype(np.int64) + sum_shift
            if "max" in acc:
                acc["max"] = max_fn(acc["max"], m)
        return acc
    return accumulate


def _window_transposed(a, x0, y0, w, h):
    return a[..., x0:x0 + w, y0:y0 + h]


def _window_off_by_one(a, x0, y0, w, h):
    return a[..., y0:y0 + h, x0 + 1:x0 + w + 1] if x0 + w < a.shape[-1] else a[..., y0:y0 + h, x0:x0 + w]


class _MultisetRemoveAll(oc.Multiset):
    def remove(self, ids):
        for i in set(int(i) for i in ids):
            if i not in self._held:
                raise KeyError(i)
            del self._held[i]


class _MultisetNoCheck(oc.Multiset):
    def remove(self, ids):
        for i in ids:
            lst = self._held.get(int(i), [])
            if lst:
                lst.pop(0)


def _narrow_saturating(result, count_bits):
    out = {}
    for k, v in result.items():
        if k == "count":
            lim = (1 << count_bits) - 1
            out[k] = np.minimum(v, lim).astype(np.uint16 if count_bits == 16 else np.uint32)
        elif k == "sum":
            out[k] = np.minimum(v, (1 << 32) - 1).astype(np.uint32)
        else:
            out[k] = v.astype(np.uint8)
    return out


def _hist_shifted(count, nbins):
    c = np.asarray(count).ravel()
    return np.array([int(np.sum(c == k + 1)) for k in range(nbins)], dtype=np.int64)


def _batch_swapped_xy(pool, requests):
    swapped = [dict(r, x0=r["y0"], y0=r["x0"]) for r in requests]
    try:
        return oc.batch(pool, swapped)
    except ValueError:
        return [np.zeros((r["h"], r["w"]), np.int64) - 1 for r in requests]


MUTANTS = {
    "count_gt1": _impl(accumulate=_acc_variant(count_pred=lambda m: m > 1)),
    "count_ge0": _impl(accumulate=_acc_variant(count_pred=lambda m: m >= 0)),
    "drop_first_member": _impl(accumulate=_acc_variant(skip_first=True)),
    "max_is_min": _impl(accumulate=_acc_variant(max_fn=np.minimum)),
    "sum_plus_one": _impl(accumulate=_acc_variant(sum_shift=1)),
    "window_transposed": _impl(window=_window_transposed),
    "window_off_by_one": _impl(window=_window_off_by_one),
    "remove_all_copies": _impl(Multiset=_MultisetRemoveAll),
    "remove_unchecked": _impl(Multiset=_MultisetNoCheck),
    "narrow_saturates": _impl(narrow=_narrow_saturating),
    "histogram_shifted": _impl(overlap_histogram=_hist_shifted),
    "batch_xy_swapped": _impl(batch=_batch_swapped_xy),
}


def _caught(impl):
    pins = list(ALL_SMALL) + [pin_exhaustive_binary_2x2(),
                              lambda i: pin_closed_form(i, synth.PLAIN_SMALL.scaled(N=6, H=40, W=56, sigma=4.0))]
    for pin in pins:
        try:
            pin(impl)
        except (AssertionError, IndexError, ValueError, KeyError, TypeError):
            return True
    return False


def test_real_oracle_passes_every_pin():
    assert not _caught(_impl())


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    assert _caught(MUTANTS[name]), f"planted mistake {name} slipped through every pin"
