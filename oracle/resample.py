"""Bilinear resampling for mixed-media matching and stabilised video (test
infrastructure only).

Sec. V-B matches a still image against a video fingerprint after resizing
and cropping the image's PRNU to the video's geometry.  Reading taken (the
paper takes the parameters from its companion work and gives no kernel):
output pixel (y, x) samples the input at ((y + oy + 0.5)/s - 0.5,
(x + ox + 0.5)/s - 0.5) (pixel centres, s = output/input size), the
coordinates clamped to the plane, with bilinear weights.

Stabilised video (Sec. II-B: the stabiliser shifts, rotates, shears or zooms
each frame; Sec. V-E) needs the general case: affine() samples the input at
u = m0 x + m1 y + m2 (column), v = m3 x + m4 y + m5 (row) for output pixel
(row y, column x), in pixel-index coordinates, with the same clamping and
weights.  rotation() builds the matrix of a rotation by an angle and a zoom
about the two planes' centres plus a translation.
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


def affine(X: np.ndarray, M, oh: int, ow: int) -> np.ndarray:
    """[oh][ow] float64: output (y, x) = bilinear sample of X at column
    u = M[0] x + M[1] y + M[2], row v = M[3] x + M[4] y + M[5], both clamped
    to the plane."""
    X = np.asarray(X, dtype=np.float64)
    H, W = X.shape
    m = [float(t) for t in M]
    yy, xx = np.mgrid[0:oh, 0:ow].astype(np.float64)
    u = np.clip(m[0] * xx + m[1] * yy + m[2], 0.0, W - 1)
    v = np.clip(m[3] * xx + m[4] * yy + m[5], 0.0, H - 1)
    x0 = np.floor(u).astype(np.int64)
    y0 = np.floor(v).astype(np.int64)
    x1 = np.minimum(x0 + 1, W - 1)
    y1 = np.minimum(y0 + 1, H - 1)
    wx = u - x0
    wy = v - y0
    top = (1 - wx) * X[y0, x0] + wx * X[y0, x1]
    bot = (1 - wx) * X[y1, x0] + wx * X[y1, x1]
    return (1 - wy) * top + wy * bot


def rotation(theta: float, zoom: float, H: int, W: int, oh: int, ow: int, ty: float = 0.0, tx: float = 0.0):
    """Matrix for affine(): output pixel p maps to the source point
    c_in + R(theta) (p - c_out) / zoom + (tx, ty), c the planes' centres
    ((n - 1) / 2), R the rotation by theta (radians) in (column, row)
    coordinates."""
    c, s = np.cos(theta) / zoom, np.sin(theta) / zoom
    cx_o, cy_o, cx_i, cy_i = (ow - 1) / 2.0, (oh - 1) / 2.0, (W - 1) / 2.0, (H - 1) / 2.0
    return [c, -s, cx_i + tx - c * cx_o + s * cy_o, s, c, cy_i + ty - s * cx_o - c * cy_o]
