"""Host logic of banded compositing (CPU): the order of context use when
read-backs run on a worker thread, with a stand-in for the context that
records every call.  No device work."""

import threading
import time

import numpy as np
import pytest

import paper_2104_14667_amd.subdivide as sd


class FakeContext:
    """Records calls; a read takes a while and marks the context busy."""
    log = []
    lock = threading.Lock()
    fail_add_at = None       # fail the add of this band index
    count = 0

    def __init__(self, W, h, outputs, bits, **opts):
        FakeContext.count += 1
        self.id, self.h, self.busy, self.closed = FakeContext.count, h, False, False
        self.opts = opts
        self._log("new", h, opts.get("pageable_host"))

    def _log(self, *what):
        with FakeContext.lock:
            FakeContext.log.append((self.id,) + what)

    def clear(self):
        assert not self.busy and not self.closed, "cleared while its read-back runs"
        self._log("clear")

    def add(self, maps):
        assert not self.busy and not self.closed, "added to while its read-back runs"
        band = sum(1 for e in FakeContext.log if e[1] == "add")
        if FakeContext.fail_add_at is not None and band == FakeContext.fail_add_at:
            raise RuntimeError("add failed")
        self._log("add", [len(m) for m in maps])

    def read(self, name, out, pinned):
        self.busy = True
        time.sleep(0.02)
        out[...] = self.id
        self.busy = False
        self._log("read", name)

    def close(self):
        assert not self.busy, "closed while its read-back runs"
        self.closed = True
        self._log("close")


@pytest.fixture
def fake(monkeypatch):
    monkeypatch.setattr(sd, "Composite", FakeContext)
    FakeContext.log, FakeContext.count, FakeContext.fail_add_at = [], 0, None
    return FakeContext


def test_two_contexts_per_height_in_turn(fake):
    W, H = 8, 53                                    # five bands of 10 rows and one of 3
    out = sd.composite_banded([np.zeros(W * H, np.uint8)] * 2, W, H, 10, ("count", "max"))
    news = [e for e in fake.log if e[1] == "new"]
    assert [e[2] for e in news] == [10, 10, 3]      # two full-height contexts, one for the tail
    assert [e[3] for e in news] == [1, 1, 1]        # numpy members: through pinned bounce buffers
    # band b is written by context 1 + (b % 2), the tail by the third
    assert [int(out["count"][y, 0]) for y in range(0, H, 10)] == [1, 2, 1, 2, 1, 3]
    assert np.array_equal(out["max"], out["count"].astype(np.uint8))
    # every add streams exactly its band's bytes of each member
    assert [e[2] for e in fake.log if e[1] == "add"] == [[80, 80]] * 5 + [[24, 24]]
    assert sum(1 for e in fake.log if e[1] == "clear") == 3
    # each context closed once, after every read
    closes = [i for i, e in enumerate(fake.log) if e[1] == "close"]
    reads = [i for i, e in enumerate(fake.log) if e[1] == "read"]
    assert len(closes) == 3 and min(closes) > max(reads)


def test_failed_add_waits_for_reads_and_closes(fake):
    fake.fail_add_at = 3
    with pytest.raises(RuntimeError, match="add failed"):
        sd.composite_banded([np.zeros(8 * 60, np.uint8)], 8, 60, 10)
    closes = [i for i, e in enumerate(fake.log) if e[1] == "close"]
    reads = [i for i, e in enumerate(fake.log) if e[1] == "read"]
    assert len(closes) == 2 and len(reads) == 3 and min(closes) > max(reads)


def test_argument_checks(fake):
    with pytest.raises(ValueError):
        sd.composite_banded([np.zeros(10, np.uint8)], 4, 4, 2)          # wrong member size
    with pytest.raises(ValueError):
        sd.composite_banded([np.zeros(16, np.uint8)], 4, 4, 0)          # no rows per band
    with pytest.raises(ValueError):
        sd.composite_banded([np.zeros(16, np.uint8)], 4, 4, 2,
                            out={"count": np.zeros((4, 4), np.uint16)})  # wrong dtype
    assert fake.log == []


def test_pageable_members_use_bounce_buffers(fake):
    """numpy members are uploaded with pageable_host = 1; asking for direct
    copies (pageable_host = 0) from them is refused before any context."""
    with pytest.raises(ValueError, match="page-locked"):
        sd.composite_banded([np.zeros(16, np.uint8)], 4, 4, 2, pageable_host=0)
    assert fake.log == []
    sd.composite_banded([np.zeros(16, np.uint8)], 4, 4, 4, pageable_host=1)
    assert [e[3] for e in fake.log if e[1] == "new"] == [1]
