"""Circular cross-correlation, PCE and NCC (test infrastructure only).

Sec. II-A: a query's noise residual is correlated with the camera fingerprint;
Sec. IV decides "same camera" when the peak-to-correlation energy exceeds 60.

Readings taken (the paper cites Goljan et al. for PCE without its formula):

* both fields are made zero-mean first;
* C(s) = sum_y X(y + s) * Y(y), circular in both axes;
* the peak is C(0,0) (aligned verification) or the first maximum of C in
  row-major order (shift search);
* the energy is the mean of C^2 over all shifts outside the nbhd x nbhd block
  centred on the peak (circular), and PCE = sign(C_p) * C_p^2 / energy;
* NCC = C(0,0) / (|X| |Y|).
"""
from __future__ import annotations

import numpy as np

PEAK_FIXED_00 = 0
PEAK_ARGMAX = 1


def xcorr_fft(X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """C(s) = sum_y X(y+s) Y(y) via the DFT: ifft2(fft2(X) * conj(fft2(Y)))."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    return np.real(np.fft.ifft2(np.fft.fft2(X) * np.conj(np.fft.fft2(Y))))


def xcorr_brute(X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """C(s) = sum_y X(y+s) Y(y) by direct summation (tiny sizes only)."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    h, w = X.shape
    C = np.zeros((h, w))
    for sy in range(h):
        for sx in range(w):
            acc = 0.0
            for yy in range(h):
                for yx in range(w):
                    acc += X[(yy + sy) % h, (yx + sx) % w] * Y[yy, yx]
            C[sy, sx] = acc
    return C


def pce(X: np.ndarray, Y: np.ndarray, peak_mode: int = PEAK_FIXED_00, nbhd: int = 11,
        C: np.ndarray | None = None):
    """PCE, NCC and peak position of the pair (X, Y).

    Returns dict(pce, ncc, peak=(py, px), cpeak, energy).
    """
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    h, w = X.shape
    if h <= nbhd or w <= nbhd or nbhd % 2 != 1:
        raise ValueError("field must be larger than the odd neighbourhood")
    Xc = X - X.mean()
    Yc = Y - Y.mean()
    if C is None:
        C = xcorr_fft(Xc, Yc)
    if peak_mode == PEAK_FIXED_00:
        py, px = 0, 0
    elif peak_mode == PEAK_ARGMAX:
        flat = int(np.argmax(C))  # first maximum in row-major order
        py, px = divmod(flat, w)
    else:
        raise ValueError("peak mode")
    r = nbhd // 2
    mask = np.ones((h, w), dtype=bool)
    rows = [(py + dy) % h for dy in range(-r, r + 1)]
    cols = [(px + dx) % w for dx in range(-r, r + 1)]
    mask[np.ix_(rows, cols)] = False
    energy = float(np.sum(C[mask] ** 2)) / (h * w - nbhd * nbhd)
    cp = float(C[py, px])
    nx, ny = float(np.sqrt(np.sum(Xc * Xc))), float(np.sqrt(np.sum(Yc * Yc)))
    ncc = float(C[0, 0]) / (nx * ny) if nx > 0 and ny > 0 else 0.0
    val = np.sign(cp) * cp * cp / energy if energy > 0 else 0.0
    return {"pce": float(val), "ncc": ncc, "peak": (py, px), "cpeak": cp, "energy": energy}


def blocks(X: np.ndarray, b: int) -> list:
    """The disjoint b x b blocks of a plane in row-major block order (Sec. IV
    divides fingerprints and test residuals into 500 x 500 blocks); rows and
    columns past the last whole block are not used."""
    X = np.asarray(X)
    h, w = X.shape
    return [X[r * b:(r + 1) * b, c * b:(c + 1) * b] for r in range(h // b) for c in range(w // b)]


def pce_blocks(X: np.ndarray, Y: np.ndarray, b: int, nbhd: int = 11) -> np.ndarray:
    """Block-wise fixed-peak PCE of a query residual X against a fingerprint
    term Y (Sec. IV): block k of X correlated with block k of Y, each block a
    field of its own (zero-mean, circular).  Returns one PCE per block."""
    return np.array([pce(x, y, PEAK_FIXED_00, nbhd)["pce"] for x, y in zip(blocks(X, b), blocks(Y, b))])
