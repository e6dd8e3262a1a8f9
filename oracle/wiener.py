"""Local-variance Wiener shrinkage (test infrastructure only).

Reading taken for the denoiser named in Sec. IV (Mihcak et al.'s locally
adaptive wavelet denoiser): for every detail coefficient c of a subband,

    m_w      = (1/w^2) * sum of c^2 over the centred w x w window
               (positions outside the subband count as zero, divisor w^2)
    var_hat  = min over w in {3,5,7,9} of max(0, m_w - s2)
    residual = c * s2 / (var_hat + s2)          (0 when the denominator is 0)

where s2 is the noise variance (sigma0^2, times a per-level weight).  The
denoised coefficient is c - residual = c * var_hat / (var_hat + s2); the noise
residual W = I - F(I) keeps the residual part.
"""
from __future__ import annotations

import numpy as np

WINDOWS = (3, 5, 7, 9)


def box_sum(q: np.ndarray, w: int) -> np.ndarray:
    """Sum over the centred w x w window, zero outside the array (plain shifts)."""
    if w % 2 != 1:
        raise ValueError("window must be odd")
    r = w // 2
    H, W = q.shape
    p = np.zeros((H + 2 * r, W + 2 * r))
    p[r:r + H, r:r + W] = q
    out = np.zeros((H, W))
    for dy in range(w):
        for dx in range(w):
            out += p[dy:dy + H, dx:dx + W]
    return out


def local_variance(c: np.ndarray, s2: float, windows=WINDOWS) -> np.ndarray:
    """var_hat = min_w max(0, m_w - s2)."""
    q = np.asarray(c, dtype=np.float64) ** 2
    est = None
    for w in windows:
        v = np.maximum(0.0, box_sum(q, w) / (w * w) - s2)
        est = v if est is None else np.minimum(est, v)
    return est


def residual_factor(c: np.ndarray, s2: float, windows=WINDOWS) -> np.ndarray:
    """rho = s2 / (var_hat + s2), 0 where the denominator vanishes."""
    est = local_variance(c, s2, windows)
    den = est + s2
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(den > 0, s2 / np.where(den > 0, den, 1.0), 0.0)


def wiener_residual(c: np.ndarray, s2: float, windows=WINDOWS) -> np.ndarray:
    """Noise part of the coefficients: c * s2 / (var_hat + s2)."""
    return np.asarray(c, dtype=np.float64) * residual_factor(c, s2, windows)
