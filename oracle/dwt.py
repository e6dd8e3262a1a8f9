"""Periodised separable 2-D discrete wavelet transform (test infrastructure only).

Reading taken (the paper names only "wavelet denoising"): orthonormal
periodised (circular) boundary handling, so the transform preserves energy
exactly and its inverse is its transpose.

1-D analysis of a length-n signal x (n even) with low-pass h and high-pass g
(L taps each):

    a[k] = sum_j h[j] * x[(2k + j) mod n]      k = 0 .. n/2 - 1
    d[k] = sum_j g[j] * x[(2k + j) mod n]

1-D synthesis is the adjoint: every a[k], d[k] adds h[j]*a[k] + g[j]*d[k]
back into x[(2k + j) mod n].

2-D: filter along axis 1 (each row), then along axis 0 (each column).  The
four subbands are named by (axis-0 filter, axis-1 filter):

    ll = lo0(lo1(x)), lh = lo0(hi1(x)), hl = hi0(lo1(x)), hh = hi0(hi1(x))

where lo1/hi1 filter along axis 1 and lo0/hi0 along axis 0.  A multi-level
decomposition repeats the 2-D step on 'll'.
"""
from __future__ import annotations

import numpy as np

from .filters import highpass, lowpass


def analysis_1d(x: np.ndarray, h: np.ndarray, g: np.ndarray, axis: int):
    """One periodised analysis step along ``axis``; returns (a, d)."""
    x = np.moveaxis(np.asarray(x, dtype=np.float64), axis, -1)
    n = x.shape[-1]
    if n % 2:
        raise ValueError("length must be even")
    k = np.arange(n // 2)
    a = np.zeros(x.shape[:-1] + (n // 2,))
    d = np.zeros_like(a)
    for j in range(len(h)):
        xs = x[..., (2 * k + j) % n]
        a += h[j] * xs
        d += g[j] * xs
    return np.moveaxis(a, -1, axis), np.moveaxis(d, -1, axis)


def synthesis_1d(a: np.ndarray, d: np.ndarray, h: np.ndarray, g: np.ndarray, axis: int):
    """Adjoint of :func:`analysis_1d` (its exact inverse for orthonormal filters)."""
    a = np.moveaxis(np.asarray(a, dtype=np.float64), axis, -1)
    d = np.moveaxis(np.asarray(d, dtype=np.float64), axis, -1)
    m = a.shape[-1]
    n = 2 * m
    k = np.arange(m)
    x = np.zeros(a.shape[:-1] + (n,))
    for j in range(len(h)):
        idx = (2 * k + j) % n
        contrib = h[j] * a + g[j] * d
        # idx is a permutation-free injection for fixed j (2k+j distinct mod n)
        x[..., idx] += contrib
    return np.moveaxis(x, -1, axis)


def dwt2(x: np.ndarray, taps: int):
    """One 2-D level: returns dict with 'll', 'lh', 'hl', 'hh'."""
    h, g = lowpass(taps), highpass(taps)
    lo1, hi1 = analysis_1d(x, h, g, axis=1)
    ll, hl = analysis_1d(lo1, h, g, axis=0)
    lh, hh = analysis_1d(hi1, h, g, axis=0)
    return {"ll": ll, "lh": lh, "hl": hl, "hh": hh}


def idwt2(bands: dict, taps: int) -> np.ndarray:
    """Inverse of :func:`dwt2` (adjoint: columns first, then rows)."""
    h, g = lowpass(taps), highpass(taps)
    lo1 = synthesis_1d(bands["ll"], bands["hl"], h, g, axis=0)
    hi1 = synthesis_1d(bands["lh"], bands["hh"], h, g, axis=0)
    return synthesis_1d(lo1, hi1, h, g, axis=1)


def wavedec2(x: np.ndarray, taps: int, levels: int):
    """Multi-level decomposition.

    Returns (ll_L, [details_1, ..., details_L]) where details_l is a dict of
    'lh', 'hl', 'hh' at level l (l = 1 finest).
    """
    cur = np.asarray(x, dtype=np.float64)
    details = []
    for _ in range(levels):
        if cur.shape[0] % 2 or cur.shape[1] % 2:
            raise ValueError("size not divisible by 2^levels")
        b = dwt2(cur, taps)
        details.append({k: b[k] for k in ("lh", "hl", "hh")})
        cur = b["ll"]
    return cur, details


def waverec2(ll: np.ndarray, details: list, taps: int) -> np.ndarray:
    """Inverse of :func:`wavedec2`."""
    cur = np.asarray(ll, dtype=np.float64)
    for lvl in range(len(details) - 1, -1, -1):
        b = dict(details[lvl])
        b["ll"] = cur
        cur = idwt2(b, taps)
    return cur
