"""Pins of the oracle's Daubechies filters against closed forms and the
defining properties (orthonormality, vanishing moments, extremal phase)."""
import os

import mpmath as mp
import numpy as np
import pytest

from oracle import filters

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "daubechies_closed_forms.txt")


def _golden():
    out = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        head, *vals = line.split()
        out[int(head.split("=")[1])] = [float(v) for v in vals]
    return out


@pytest.mark.parametrize("taps", [2, 4])
def test_closed_form(taps):
    ref = _golden()[taps]
    np.testing.assert_allclose(filters.lowpass(taps), ref, rtol=0, atol=2e-16)


@pytest.mark.parametrize("taps", [4, 6, 8, 12, 16])
def test_orthonormal_and_sum(taps):
    h = filters.lowpass_mp(taps)
    with mp.workdps(60):
        assert abs(mp.fsum(h) - mp.sqrt(2)) < mp.mpf(10) ** -45
        for m in range(taps // 2):
            s = mp.fsum(h[k] * h[k + 2 * m] for k in range(taps - 2 * m))
            assert abs(s - (1 if m == 0 else 0)) < mp.mpf(10) ** -40, (taps, m, s)


@pytest.mark.parametrize("taps", [4, 6, 8, 12, 16])
def test_vanishing_moments(taps):
    """sum_k (-1)^k k^p h_k = 0 for p < N: the high-pass kills polynomials of degree < N."""
    h = filters.lowpass_mp(taps)
    N = taps // 2
    with mp.workdps(60):
        for p in range(N):
            s = mp.fsum((-1) ** k * mp.mpf(k) ** p * h[k] for k in range(taps))
            scale = mp.fsum(abs(mp.mpf(k) ** p * h[k]) for k in range(taps))
            assert abs(s) < mp.mpf(10) ** -40 * scale, (taps, p)
        # ... and not beyond: the N-th moment is non-zero (exactly N moments)
        s = mp.fsum((-1) ** k * mp.mpf(k) ** N * h[k] for k in range(taps))
        assert abs(s) > mp.mpf(10) ** -6


@pytest.mark.parametrize("taps", [4, 8, 16])
def test_extremal_phase(taps):
    """Apart from the N-fold zero at z = -1, every zero of sum h_k z^k lies
    outside the unit circle (minimum phase of sum h_k z^-k)."""
    h = filters.lowpass_mp(taps)
    N = taps // 2
    with mp.workdps(60):
        roots = mp.polyroots(list(reversed(h)), maxsteps=500, extraprec=300)
        near_m1 = [r for r in roots if abs(r + 1) < mp.mpf("1e-3")]
        others = [r for r in roots if abs(r + 1) >= mp.mpf("1e-3")]
        assert len(near_m1) == N
        assert all(abs(r) > 1 + mp.mpf("1e-6") for r in others)


def test_db8_energy_front_loaded():
    """Extremal phase puts the filter's energy first: the partial energies of
    the oracle's 16-tap filter dominate those of its time reverse."""
    h = filters.lowpass(16)
    e = np.cumsum(h ** 2)
    er = np.cumsum(h[::-1] ** 2)
    assert np.all(e[:-1] >= er[:-1] - 1e-15)


def test_highpass_qmf():
    for taps in (2, 8, 16):
        h, g = filters.lowpass(taps), filters.highpass(taps)
        # orthogonal to the low-pass at every even shift, and g sums to 0
        for m in range(-(taps // 2) + 1, taps // 2):
            s = sum(h[k] * g[k + 2 * m] for k in range(taps) if 0 <= k + 2 * m < taps)
            assert abs(s) < 1e-14
        assert abs(g.sum()) < 1e-14
