"""Daubechies orthonormal wavelet filters (test infrastructure only).

The paper names its denoiser only by citation (Sec. IV, the wavelet denoiser of
Mihcak et al.); the filter bank used here is the Daubechies extremal-phase
family with N = L/2 vanishing moments, "db8" being L = 16 taps.

Construction (Daubechies, "Orthonormal bases of compactly supported wavelets",
1988): with y = sin^2(w/2), the squared modulus of the low-pass response is
cos^{2N}(w/2) * P(y) with P(y) = sum_{k<N} C(N-1+k, k) y^k.  Each root y_r of
P gives the pair z, 1/z solving z + 1/z = 2 - 4 y_r; keeping the member
outside the unit circle for every pair gives H(z) = sum_k h_k z^k proportional
to (1+z)^N * prod_r (z - z_r).  Normalising sum h = sqrt(2) fixes scale and
sign.  All arithmetic is done with mpmath at 60 significant digits.
"""
from __future__ import annotations

import functools

import mpmath as mp
import numpy as np


def _poly_mul(a, b):
    out = [mp.mpc(0)] * (len(a) + len(b) - 1)
    for i, ai in enumerate(a):
        for j, bj in enumerate(b):
            out[i + j] += ai * bj
    return out


def lowpass_mp(taps: int) -> list:
    """Low-pass filter h_0..h_{L-1} of the L-tap Daubechies wavelet as mpmath reals."""
    if taps < 2 or taps % 2:
        raise ValueError("taps must be even and >= 2")
    N = taps // 2
    with mp.workdps(60):
        poly = [mp.mpc(1)]  # ascending coefficients of H(z)
        for _ in range(N):
            poly = _poly_mul(poly, [mp.mpc(1), mp.mpc(1)])  # (1 + z)
        if N > 1:
            # P(y), highest degree first for mpmath.polyroots
            pc = [mp.binomial(N - 1 + k, k) for k in range(N)][::-1]
            for y in mp.polyroots(pc, maxsteps=400, extraprec=200):
                b = 2 - 4 * mp.mpc(y)
                disc = mp.sqrt(b * b - 4)
                z1, z2 = (b + disc) / 2, (b - disc) / 2
                z = z1 if abs(z1) > 1 else z2
                poly = _poly_mul(poly, [-z, mp.mpc(1)])  # (z - z_r)
        coeffs = [mp.re(c) for c in poly]
        s = mp.fsum(coeffs)
        return [c * mp.sqrt(2) / s for c in coeffs]


@functools.lru_cache(maxsize=None)
def daubechies_lowpass(taps: int) -> tuple:
    """Low-pass filter h_0..h_{L-1} rounded to float64."""
    return tuple(float(c) for c in lowpass_mp(taps))


def lowpass(taps: int) -> np.ndarray:
    return np.array(daubechies_lowpass(taps), dtype=np.float64)


def highpass(taps: int) -> np.ndarray:
    """Quadrature-mirror high-pass g_k = (-1)^k h_{L-1-k}."""
    h = lowpass(taps)
    L = len(h)
    return np.array([(-1) ** k * h[L - 1 - k] for k in range(L)], dtype=np.float64)
