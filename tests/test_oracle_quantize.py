"""Pins of the oracle's UNORM8 plane storage (Sec. 5.1) against closed forms."""
import numpy as np

from oracle import quantize


def test_endpoints_and_clamping():
    v = np.array([0.0, 1.0, -0.3, 1.7, np.nan, np.inf, -np.inf, 1e-12, 1.0 - 1e-12])
    assert quantize.unorm8(v).tolist() == [0, 255, 0, 255, 0, 255, 0, 0, 255]


def test_ties_and_nearest():
    # 255 * 0.5 = 127.5 is exact: the tie goes to the even code
    assert int(quantize.unorm8(0.5)) == 128
    assert int(quantize.unorm8(0.25)) == 64                   # 63.75
    # just either side of the 1.5 tie
    assert int(quantize.unorm8((1.5 - 1e-9) / 255.0)) == 1
    assert int(quantize.unorm8((1.5 + 1e-9) / 255.0)) == 2


def test_every_code_round_trips():
    k = np.arange(256)
    assert np.array_equal(quantize.unorm8(quantize.dequant(k)), k.astype(np.uint8))


def test_error_bound_and_monotone():
    v = np.sort(np.random.default_rng(0).uniform(-0.1, 1.1, 200_001))
    c = quantize.unorm8(v)
    assert np.all(np.diff(c.astype(int)) >= 0)
    inside = (v >= 0) & (v <= 1)
    assert np.abs(quantize.dequant(c[inside]) - v[inside]).max() <= 0.5 / 255.0 + 1e-15


def test_near_tie_band():
    assert bool(quantize.near_tie(0.5, 1e-9))                 # 127.5
    assert not bool(quantize.near_tie(0.5 + 0.01 / 255, 0.005))
    assert bool(quantize.near_tie(0.5 + 0.004 / 255, 0.005))
    assert not bool(quantize.near_tie(10.0 / 255, 0.4))        # on a code
