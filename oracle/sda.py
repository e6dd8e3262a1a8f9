"""Spatial-domain averaged frames (test infrastructure only).

Sec. III-B: the m frames are split into disjoint groups of d consecutive
frames and every group is replaced by the arithmetic mean of its frames
(the SDA frame).  Group i (0-based) holds frames i*d .. i*d + d - 1.

Reading taken where the paper assumes g = m/d exactly: when d does not divide
m, the last group keeps the n_g < d remaining frames and is averaged over n_g.
"""
from __future__ import annotations

import numpy as np


def groups(n_frames: int, d: int):
    """List of (first, count) per SDA group."""
    if d < 1 or n_frames < 0:
        raise ValueError("bad group size")
    return [(s, min(d, n_frames - s)) for s in range(0, n_frames, d)]


def sda_sums(frames: np.ndarray, d: int):
    """Exact per-group sums.

    ``frames`` is [m][H][W][C] (any integer dtype, or float).  Returns
    (sums [g][C][H][W], counts [g]); integer input gives exact int64 sums,
    float input float64 sums.
    """
    f = np.asarray(frames)
    m = f.shape[0]
    acc_t = np.int64 if np.issubdtype(f.dtype, np.integer) else np.float64
    gl = groups(m, d)
    C = f.shape[3]
    sums = np.zeros((len(gl), C, f.shape[1], f.shape[2]), dtype=acc_t)
    counts = np.zeros(len(gl), dtype=np.int64)
    for i, (s, n) in enumerate(gl):
        for j in range(s, s + n):
            sums[i] += np.moveaxis(f[j].astype(acc_t), -1, 0)
        counts[i] = n
    return sums, counts


def sda_means(frames: np.ndarray, d: int) -> np.ndarray:
    """SDA frames I_i = S_i / n_i in float64, [g][C][H][W]."""
    sums, counts = sda_sums(frames, d)
    return sums.astype(np.float64) / counts[:, None, None, None]


def sda_means_f32(frames: np.ndarray, d: int) -> np.ndarray:
    """float32 rounding of S_i / n_i (division in float64, one rounding)."""
    return sda_means(frames, d).astype(np.float32)
