"""Bilinear resampling for mixed-media matching (test infrastructure only).

Sec. V-B matches a still image against a video fingerprint after resizing
and cropping the image's PRNU to the video's geometry.  Reading taken (the
paper takes the parameters from its companion work and gives no kernel):
output pixel (y, x) samples the input at ((y + oy + 0.5)/s - 0.5,
(x + ox + 0.5)/s - 0.5) (pixel centres, s = output/input size), the
coordinates clamped to the plane, with bilinear weights.
"""
from __future__ import annotations

import numpy as np


def bilinear(X: np.ndarray, scale: float, oh: int, ow: int, oy: int = 0, ox: int = 0) -> np.ndarray:
    """[oh][ow] float64 resampled plane."""
    X = np.asarray(X, dtype=np.float64)
    H, W = X.shape
    fy = np.clip((np.arange(oh) + oy + 0.5) / scale - 0.5, 0.0, H - 1)
    fx = np.clip((np.arange(ow) + ox + 0.5) / scale - 0.5, 0.0, W - 1)
    y0 = np.floor(fy).astype(np.int64)
    x0 = np.floor(fx).astype(np.int64)
    y1 = np.minimum(y0 + 1, H - 1)
    x1 = np.minimum(x0 + 1, W - 1)
    wy = (fy - y0)[:, None]
    wx = (fx - x0)[None, :]
    a, b = X[np.ix_(y0, x0)], X[np.ix_(y0, x1)]
    c, d = X[np.ix_(y1, x0)], X[np.ix_(y1, x1)]
    return (1 - wy) * ((1 - wx) * a + wx * b) + wy * ((1 - wx) * c + wx * d)
