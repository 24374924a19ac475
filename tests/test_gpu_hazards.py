"""Pipeline hazards (GPU): the streamed pipeline stays bit-exact when one of
its streams is held up by a bounded spin kernel enqueued before and between
calls, with released staging slots poisoned (0xA5), one or two slots, and
host-paced or event-only ordering.  Every wait in the test ends: the spin
kernels run for a fixed number of cycles."""

import numpy as np
import pytest
import torch

from paper_2104_14667_amd import synth
from paper_2104_14667_amd.composite import CMP_TILED, Composite

from gpu_common import check_full, expect_oracle, pinned_copy, say

pytestmark = pytest.mark.gpu

SPIN_CYCLES = 2_000_000


@pytest.mark.parametrize("delayed", ["copy", "compute"])
@pytest.mark.parametrize("nbuf,host_paced,layout,copy_streams",
                         [(2, 1, "linear", 0), (2, 0, "linear", 0), (1, 1, "linear", 0),
                          (2, 1, "tiled", 0), (2, 0, "linear", 2), (2, 0, "tiled", 2)])
def test_delayed_stream_stays_exact(delayed, nbuf, host_paced, layout, copy_streams):
    say("hazard", delayed, nbuf, host_paced, layout, copy_streams)
    W, H = 256, 48
    A = synth.random_members(61, 21, H, W)
    hA = pinned_copy(torch.from_numpy(A))
    copy_s, comp_s = torch.cuda.Stream(), torch.cuda.Stream()
    spin_on = copy_s if delayed == "copy" else comp_s
    # with two copy streams the delayed copy stream carries slot 0's uploads only
    kw = dict(nbuf=nbuf, chunk_depth=3, host_paced=host_paced, debug_poison=1,
              copy_stream=copy_s, compute_stream=comp_s, copy_streams=copy_streams)
    if layout == "tiled":
        kw.update(layout=CMP_TILED, tile_w=64, tile_h=16)
    outs = ("count", "sum")
    with Composite(W, H, outs, 32, **kw) as c:
        for k0 in (0, 7, 14):
            with torch.cuda.stream(spin_on):
                torch.cuda._sleep(SPIN_CYCLES)
            c.add([hA[i] for i in range(k0, k0 + 7)])
        with torch.cuda.stream(spin_on):
            torch.cuda._sleep(SPIN_CYCLES)
        c.remove(maps=[hA[i] for i in range(0, 21, 2)])
        check_full(c, expect_oracle(A[1::2], outs, 32))
    torch.cuda.synchronize()
