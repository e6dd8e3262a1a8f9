"""Denoiser residual, MLE fingerprint, post-processing and queries
(test infrastructure only).

Steps, in the paper's order:

* noise residual W = I - F(I) of one plane (Sec. II-A), F = 4-level wavelet
  denoiser: symmetric pad to a multiple of 16, periodised Daubechies DWT,
  Wiener shrinkage of every detail subband, approximation band kept by F
  (so the residual's approximation band is zero), inverse DWT, crop;
* SDA frames (Sec. III-B) and the MLE fingerprint
  K = sum_i W_i * I_i / sum_i I_i^2 (Sec. III-A and III-B) per channel;
* finalisation: per-channel zero-mean (row means, then column means),
  ITU-R BT.601 luma for colour, DFT-domain Wiener filtering;
* query residual: the same residual and post-processing on one frame.

Readings for what the paper leaves open are stated on each function.
"""
from __future__ import annotations

import numpy as np

from . import dwt, sda, wiener

LUMA = (0.299, 0.587, 0.114)

FIN_ZM = 1
FIN_LUMA = 2
FIN_WIENER = 4


def pad_amounts(n: int, mult: int = 16):
    """Symmetric padding (before, after) bringing n to a multiple of ``mult``."""
    p = (-n) % mult
    return p // 2, p - p // 2


def pad_symmetric(x: np.ndarray, mult: int = 16) -> np.ndarray:
    """Edge-including mirror padding of a 2-D plane (reading: the paper is silent)."""
    (t, b), (l, r) = pad_amounts(x.shape[0], mult), pad_amounts(x.shape[1], mult)
    return np.pad(np.asarray(x, dtype=np.float64), ((t, b), (l, r)), mode="symmetric")


def denoise_residual(img: np.ndarray, sigma0: float = 3.0, levels: int = 4, taps: int = 16,
                     windows=wiener.WINDOWS, level_weight=(1.0, 1.0, 1.0, 1.0)) -> np.ndarray:
    """W = I - F(I) for one 2-D plane, float64.

    Padding is to a multiple of 16 (= 2^4) regardless of ``levels``.
    ``level_weight[l-1]`` scales the noise variance sigma0^2 at level l.
    """
    img = np.asarray(img, dtype=np.float64)
    H, W = img.shape
    x = pad_symmetric(img, 16)
    ll, det = dwt.wavedec2(x, taps, levels)
    rdet = []
    for lvl, d in enumerate(det):
        s2 = float(level_weight[lvl]) * sigma0 * sigma0
        rdet.append({k: wiener.wiener_residual(v, s2, windows) for k, v in d.items()})
    resid = dwt.waverec2(np.zeros_like(ll), rdet, taps)
    (t, _), (l, _) = pad_amounts(H, 16), pad_amounts(W, 16)
    return resid[t:t + H, l:l + W]


def denoised(img: np.ndarray, **kw) -> np.ndarray:
    """F(I) computed from the shrunk pyramid directly (approximation kept,
    details multiplied by var_hat/(var_hat+s2)); used to check F(I) + W = I."""
    sigma0 = kw.get("sigma0", 3.0)
    levels = kw.get("levels", 4)
    taps = kw.get("taps", 16)
    windows = kw.get("windows", wiener.WINDOWS)
    lw = kw.get("level_weight", (1.0, 1.0, 1.0, 1.0))
    img = np.asarray(img, dtype=np.float64)
    H, W = img.shape
    x = pad_symmetric(img, 16)
    ll, det = dwt.wavedec2(x, taps, levels)
    ddet = []
    for lvl, d in enumerate(det):
        s2 = float(lw[lvl]) * sigma0 * sigma0
        band = {}
        for k, v in d.items():
            est = wiener.local_variance(v, s2, windows)
            den = est + s2
            # Wiener estimate of the clean coefficient: c * var_hat / (var_hat + s2)
            band[k] = np.where(den > 0, v * est / np.where(den > 0, den, 1.0), v)
        ddet.append(band)
    out = dwt.waverec2(ll, ddet, taps)
    (t, _), (l, _) = pad_amounts(H, 16), pad_amounts(W, 16)
    return out[t:t + H, l:l + W]


def mle_accumulate(residuals, images):
    """A = sum_i W_i * I_i, B = sum_i I_i^2, summed in the given order (float64)."""
    A = None
    B = None
    for Wi, Ii in zip(residuals, images):
        Wi = np.asarray(Wi, dtype=np.float64)
        Ii = np.asarray(Ii, dtype=np.float64)
        A = Wi * Ii if A is None else A + Wi * Ii
        B = Ii * Ii if B is None else B + Ii * Ii
    return A, B


def mle_ratio(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """K = A / B, 0 where B = 0."""
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(B > 0, A / np.where(B > 0, B, 1.0), 0.0)


def fingerprint_accumulate(frames: np.ndarray, d: int, **dn):
    """SDA grouping of [m][H][W][C] frames, then per-channel MLE accumulators
    over the g SDA frames.  Returns (A, B) each [C][H][W] float64.  d = 1 is
    the conventional estimator (every frame denoised)."""
    means = sda.sda_means(frames, d)  # [g][C][H][W]
    g, C, H, W = means.shape
    A = np.zeros((C, H, W))
    B = np.zeros((C, H, W))
    for i in range(g):
        for c in range(C):
            I = means[i, c]
            Wr = denoise_residual(I, **dn)
            A[c] += Wr * I
            B[c] += I * I
    return A, B


def zero_mean(X: np.ndarray) -> np.ndarray:
    """Subtract every row's mean, then every column's mean, of a 2-D plane."""
    X = np.asarray(X, dtype=np.float64)
    X = X - X.mean(axis=1, keepdims=True)
    return X - X.mean(axis=0, keepdims=True)


def luma(planes: np.ndarray) -> np.ndarray:
    """ITU-R BT.601 luma of [3][H][W] planes."""
    return LUMA[0] * planes[0] + LUMA[1] * planes[1] + LUMA[2] * planes[2]


def wiener_dft(K: np.ndarray, sigma2: float | None = None, windows=wiener.WINDOWS) -> np.ndarray:
    """DFT-domain Wiener filtering of a 2-D field.

    F = fft2(K); M = |F| / sqrt(HW); s2 = population variance of K unless
    given; rho = the Wiener residual factor of M with noise variance s2 (same
    windows, zero extension at the edges of the frequency array); output
    Re ifft2(F * rho).
    """
    K = np.asarray(K, dtype=np.float64)
    H, W = K.shape
    F = np.fft.fft2(K)
    M = np.abs(F) / np.sqrt(H * W)
    s2 = float(np.var(K)) if sigma2 is None or sigma2 < 0 else float(sigma2)
    rho = wiener.residual_factor(M, s2, windows)
    return np.real(np.fft.ifft2(F * rho))


def finalize(A: np.ndarray, B: np.ndarray, flags: int = FIN_ZM | FIN_LUMA | FIN_WIENER,
             sigma_wf: float = -1.0) -> np.ndarray:
    """K = A/B per channel, then zero-mean per channel, luma (C = 3), DFT Wiener.

    Returns [H][W] when luma is applied or C = 1, else [C][H][W].
    """
    K = mle_ratio(A, B)
    return postprocess(K, flags, sigma_wf)


def postprocess(P: np.ndarray, flags: int, sigma_wf: float = -1.0) -> np.ndarray:
    """Zero-mean / luma / Wiener chain shared by fingerprints and query residuals."""
    P = np.asarray(P, dtype=np.float64)
    C = P.shape[0]
    if flags & FIN_ZM:
        P = np.stack([zero_mean(P[c]) for c in range(C)])
    if C == 3 and flags & FIN_LUMA:
        P = luma(P)[None]
    if flags & FIN_WIENER:
        P = np.stack([wiener_dft(P[c], None if sigma_wf < 0 else sigma_wf * sigma_wf)
                      for c in range(P.shape[0])])
    return P[0] if P.shape[0] == 1 else P


def camera_fingerprint(frames: np.ndarray, d: int, flags: int = FIN_ZM | FIN_LUMA | FIN_WIENER,
                       **dn) -> np.ndarray:
    """Full fingerprint of one camera from [m][H][W][C] frames at SDA depth d."""
    A, B = fingerprint_accumulate(frames, d, **dn)
    return finalize(A, B, flags)


def query_residual(frame: np.ndarray, flags: int = FIN_ZM | FIN_LUMA | FIN_WIENER, **dn):
    """Residual of one [H][W][C] query frame, post-processed like a fingerprint,
    and the frame's luma (or the plane for C = 1).  Returns (Wq, Iq)."""
    f = np.asarray(frame, dtype=np.float64)
    C = f.shape[2]
    Wc = np.stack([denoise_residual(f[:, :, c], **dn) for c in range(C)])
    Wq = postprocess(Wc, flags)
    planes = np.moveaxis(f, -1, 0)
    Iq = luma(planes) if C == 3 else planes[0]
    return Wq, Iq
