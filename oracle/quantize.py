"""UNORM8 storage of the sweeping planes (test infrastructure: oracle).

Sec. 5.1 stores the planes' C and T in 8 bits by default.  The planes here hold the
premultiplied colour C and the alpha 1 - T; each channel is stored as

    code = round_half_even(255 * clamp(v, 0, 1)),   read back as code / 255,

with NaN stored as 0.  Plain NumPy in float64.
"""
import numpy as np


def unorm8(v) -> np.ndarray:
    """UNORM8 codes (uint8) of values v (any shape)."""
    v = np.nan_to_num(np.asarray(v, dtype=np.float64), nan=0.0, posinf=1.0, neginf=0.0)
    return np.rint(np.clip(v, 0.0, 1.0) * 255.0).astype(np.uint8)


def dequant(code) -> np.ndarray:
    """The float64 value a code stands for."""
    return np.asarray(code, dtype=np.float64) / 255.0


def near_tie(v, band: float) -> np.ndarray:
    """True where 255 * clamp(v, 0, 1) lies within `band` of a rounding tie (k + 1/2): a
    value computed in float32 may round to either neighbouring code there."""
    x = np.clip(np.nan_to_num(np.asarray(v, dtype=np.float64), nan=0.0), 0.0, 1.0) * 255.0
    return np.abs(x - np.floor(x) - 0.5) < band
