"""The oracle against its pins (CPU only)."""

import numpy as np
import pytest

import oracle
from paper_2104_14667_amd import synth

from oracle_pins import (ALL_SMALL, closed_form_lut, pin_closed_form,
                         pin_exhaustive_binary_2x2)


@pytest.mark.parametrize("pin", ALL_SMALL, ids=lambda f: f.__name__)
def test_pin(pin):
    pin(oracle)


def test_exhaustive_binary_2x2():
    pin_exhaustive_binary_2x2()(oracle)


def test_closed_form_plain_small_full_size():
    pin_closed_form(oracle, synth.PLAIN_SMALL)


def test_closed_form_streamed_scaled():
    pin_closed_form(oracle, synth.STREAMED.scaled(N=24, H=1024, W=768, sigma=16.0))


def test_closed_form_depth_scaled():
    pin_closed_form(oracle, synth.DEPTH.scaled(N=20, H=640, W=1024, sigma=16.0))


def test_closed_form_depth_odd_shape():
    pin_closed_form(oracle, synth.DEPTH.scaled(N=7, H=17, W=4097, sigma=3.0))


def test_oracle_rejects_bad_input():
    with pytest.raises(TypeError):
        oracle.accumulate([np.zeros((2, 2), dtype=np.int32)])
    with pytest.raises(ValueError):
        oracle.accumulate([np.zeros((2, 2), np.uint8), np.zeros((2, 3), np.uint8)])
    with pytest.raises(ValueError):
        oracle.accumulate([])
    with pytest.raises(ValueError):
        oracle.window(np.zeros((4, 4), np.uint8), 2, 0, 3, 1)


def test_closed_form_lut_extremes():
    # one level above every elevation: a full mask, depth = L - e
    c, s, m = closed_form_lut([256], "depth")
    assert c[0] == 1 and s[0] == 255 and m[0] == 255   # clamp at 255
    c, s, m = closed_form_lut([0], "mask")
    assert not c.any() and not s.any() and not m.any()
