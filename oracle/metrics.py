"""Image-quality and size metrics (test infrastructure only).

* PSNR on 8-bit images, 10 log10(255^2 / MSE), the definition that reproduces
  both rows of the paper's Table II (trilinear vs compressed MFA-DVV).
* Compression ratio of a model: input samples over control points, the
  product over axes; reproduces every ratio printed under Fig. 6.
"""
from __future__ import annotations

import numpy as np


def to_u8(img: np.ndarray) -> np.ndarray:
    """Float image in [0,1] -> 8-bit levels (round half to even, clamped)."""
    return np.rint(np.clip(np.asarray(img, dtype=np.float64), 0.0, 1.0) * 255.0)


def mse(a: np.ndarray, b: np.ndarray) -> float:
    d = np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)
    return float(np.mean(d * d))


def rmse(a: np.ndarray, b: np.ndarray) -> float:
    return float(np.sqrt(mse(a, b)))


def psnr_from_mse(m: float) -> float:
    """PSNR in dB of 8-bit images with mean squared error m (in levels^2)."""
    return float(10.0 * np.log10(255.0 ** 2 / m))


def psnr8(a: np.ndarray, b: np.ndarray) -> float:
    """PSNR of two float images after conversion to 8-bit levels."""
    m = mse(to_u8(a), to_u8(b))
    return float("inf") if m == 0.0 else psnr_from_mse(m)


def compression_ratio(n_in, n_ctrl) -> float:
    """Product over axes of input samples / control points."""
    r = 1.0
    for a, b in zip(n_in, n_ctrl):
        r *= float(a) / float(b)
    return r
