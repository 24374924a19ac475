"""composite_accumulate_static (the entry point that allocates nothing)
against composite_add_device of a context on the same members, through the
C ABI (GPU).  Integer outputs: compared bit-exact, and with the oracle."""

import numpy as np
import pytest
import torch

import oracle
from paper_2104_14667_amd import synth
from paper_2104_14667_amd.composite import (CMP_COUNT, CMP_EINVAL, CMP_ERANGE, CMP_MAX, CMP_OK,
                                            CMP_STATIC_MAX_MEMBERS, CMP_SUM, Composite,
                                            composite_accumulate_static)

from gpu_common import dev_of, say

pytestmark = pytest.mark.gpu

ALL = ("count", "sum", "max")
BITS = {"count": CMP_COUNT, "sum": CMP_SUM, "max": CMP_MAX}


def _outputs(W, H, names, count_bits, fill=0xAB):
    """Caller-owned device accumulators, filled with garbage."""
    ct = torch.int16 if count_bits == 16 else torch.int32
    out = {}
    if "count" in names:
        out["count"] = torch.empty((H, W), dtype=ct, device="cuda:0")
    if "sum" in names:
        out["sum"] = torch.empty((H, W), dtype=torch.int32, device="cuda:0")
    if "max" in names:
        out["max"] = torch.empty((H, W), dtype=torch.uint8, device="cuda:0")
    for t in out.values():
        t.view(torch.uint8).fill_(fill)
    torch.cuda.synchronize()
    return out


def _static(maps, W, H, names, count_bits, out, set_):
    bits = sum(BITS[k] for k in names)
    rc = composite_accumulate_static(maps, W, H, bits, count_bits, out.get("count"), out.get("sum"),
                                     out.get("max"), set=set_)
    torch.cuda.synchronize()
    return rc


def _host(out, count_bits):
    res = {}
    for k, t in out.items():
        a = t.cpu().numpy()
        if k == "count":
            a = a.view(np.uint16 if count_bits == 16 else np.uint32)
        elif k == "sum":
            a = a.view(np.uint32)
        res[k] = a
    return res


def _context(batches, W, H, names, count_bits):
    """The same members through composite_add_device, one call per batch."""
    with Composite(W, H, names, count_bits) as c:
        for maps in batches:
            c.add_device(maps)
        return {k: c.read(k) for k in names}


def _same(got, want, what):
    for k in want:
        assert got[k].dtype == want[k].dtype, (what, k)
        assert np.array_equal(got[k], want[k]), f"{what}: {k} differs"


def test_static_entry_matches_add_device_on_two_calls():
    # first call: 300 members (more than one 256-member group), ragged raster
    W1, H1, n1 = 1000, 37, 300
    say("static entry, call 1:", n1, H1, W1)
    s1 = synth.random_members(41, n1, H1, W1)
    d1 = dev_of(s1)
    m1 = [d1[i] for i in range(n1)]
    out1 = _outputs(W1, H1, ALL, 32)
    assert _static(m1, W1, H1, ALL, 32, out1, True) == CMP_OK
    got1 = _host(out1, 32)
    _same(got1, _context([m1], W1, H1, ALL, 32), "call 1 vs add_device")
    _same(got1, oracle.narrow(oracle.accumulate(list(s1), shape=(H1, W1)), 32), "call 1 vs oracle")

    # second call, smaller: 5 members of 100 x 9, uint16 count only
    W2, H2, n2 = 100, 9, 5
    say("static entry, call 2:", n2, H2, W2)
    s2 = synth.random_members(42, n2 + 3, H2, W2)
    d2 = dev_of(s2)
    m2 = [d2[i] for i in range(n2)]
    out2 = _outputs(W2, H2, ("count",), 16)
    assert _static(m2, W2, H2, ("count",), 16, out2, True) == CMP_OK
    got2 = _host(out2, 16)
    _same(got2, _context([m2], W2, H2, ("count",), 16), "call 2 vs add_device")

    # third call adds three more members onto what the second one wrote
    m3 = [d2[i] for i in range(n2, n2 + 3)]
    assert _static(m3, W2, H2, ("count",), 16, out2, False) == CMP_OK
    got3 = _host(out2, 16)
    _same(got3, _context([m2, m3], W2, H2, ("count",), 16), "call 3 vs add_device")
    _same(got3, oracle.narrow(oracle.accumulate(list(s2), shape=(H2, W2), outputs=("count",)), 16),
          "call 3 vs oracle")


def test_static_entry_empty_set_and_refusals():
    W, H = 33, 5
    s = synth.random_members(43, 2, H, W)
    d = dev_of(s)
    out = _outputs(W, H, ALL, 32)
    # the composite of no member is zero everywhere
    assert _static([], W, H, ALL, 32, out, True) == CMP_OK
    for k, a in _host(out, 32).items():
        assert not a.any(), k
    assert _static([d[0], d[1]], W, H, ALL, 32, out, True) == CMP_OK
    before = _host(out, 32)
    # more members than the fixed table holds: refused, nothing written
    many = [d[0]] * (CMP_STATIC_MAX_MEMBERS + 1)
    assert _static(many, W, H, ALL, 32, out, True) == CMP_ERANGE
    # an output that is not 16-byte aligned: refused
    bad = {"count": out["count"].view(-1)[1:], "sum": out["sum"], "max": out["max"]}
    assert _static([d[0]], W, H, ALL, 32, bad, True) == CMP_EINVAL
    _same(_host(out, 32), before, "after refusals")
    _same(before, oracle.narrow(oracle.accumulate(list(s), shape=(H, W)), 32), "two members vs oracle")
