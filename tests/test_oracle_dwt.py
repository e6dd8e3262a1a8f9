"""Pins of the oracle's periodised DWT: perfect reconstruction, Parseval,
adjointness, the textbook Haar step, an FFT-computed circular correlation,
shift equivariance, constant images and subband orientation."""
import numpy as np
import pytest

import synth
from oracle import dwt, filters


def _rand(shape, key):
    return synth.random_field(shape, synth.CFG_TEST, 1000 + key)


SHAPES = [(16, 16), (32, 48), (64, 80), (48, 16), (128, 96)]


@pytest.mark.parametrize("taps", [2, 4, 8, 16])
@pytest.mark.parametrize("shape", SHAPES)
def test_perfect_reconstruction_and_parseval(taps, shape):
    x = _rand(shape, taps * 7 + shape[0])
    ll, det = dwt.wavedec2(x, taps, 4)
    e = np.sum(ll ** 2) + sum(np.sum(v ** 2) for d in det for v in d.values())
    assert abs(e - np.sum(x ** 2)) <= 1e-12 * np.sum(x ** 2)
    xr = dwt.waverec2(ll, det, taps)
    assert np.max(np.abs(xr - x)) <= 1e-12 * np.max(np.abs(x))


@pytest.mark.parametrize("taps", [4, 16])
def test_adjoint_dot_product(taps):
    x = _rand((32, 64), 1)
    y = _rand((32, 64), 2)
    b = dwt.dwt2(x, taps)
    yb = dwt.dwt2(y, taps)  # any coefficient set
    lhs = sum(np.sum(b[k] * yb[k]) for k in b)
    rhs = np.sum(x * dwt.idwt2(yb, taps))
    assert abs(lhs - rhs) <= 1e-12 * np.sqrt(np.sum(x ** 2) * np.sum(y ** 2))


def test_haar_textbook():
    x = _rand((6, 8), 3)
    b = dwt.dwt2(x, 2)
    a, bb, c, d = x[0::2, 0::2], x[0::2, 1::2], x[1::2, 0::2], x[1::2, 1::2]
    np.testing.assert_allclose(b["ll"], (a + bb + c + d) / 2, atol=1e-14)
    np.testing.assert_allclose(b["lh"], ((a - bb) + (c - d)) / 2, atol=1e-14)
    np.testing.assert_allclose(b["hl"], ((a + bb) - (c + d)) / 2, atol=1e-14)
    np.testing.assert_allclose(b["hh"], ((a - bb) - (c - d)) / 2, atol=1e-14)


@pytest.mark.parametrize("taps", [8, 16])
@pytest.mark.parametrize("n", [10, 32, 40])
def test_analysis_is_downsampled_circular_correlation(taps, n):
    """a = even samples of the circular correlation of x with h, computed with
    the FFT (independent of the oracle's index arithmetic); same for g."""
    x = _rand((3, n), 4 + n)
    h, g = filters.lowpass(taps), filters.highpass(taps)
    a, d = dwt.analysis_1d(x, h, g, axis=1)
    for filt, got in ((h, a), (g, d)):
        f = np.zeros(n)
        for j, v in enumerate(filt):
            f[j % n] += v  # periodised filter
        corr = np.real(np.fft.ifft(np.fft.fft(x, axis=1) * np.conj(np.fft.fft(f))[None], axis=1))
        np.testing.assert_allclose(got, corr[:, 0::2], atol=1e-13)


@pytest.mark.parametrize("taps", [4, 16])
def test_shift_equivariance(taps):
    x = _rand((32, 48), 5)
    b = dwt.dwt2(x, taps)
    bs = dwt.dwt2(np.roll(x, (2, 4), axis=(0, 1)), taps)
    for k in b:
        np.testing.assert_allclose(bs[k], np.roll(b[k], (1, 2), axis=(0, 1)), atol=1e-12)


@pytest.mark.parametrize("taps", [2, 8, 16])
def test_constant_image_has_no_details(taps):
    ll, det = dwt.wavedec2(np.full((64, 32), 123.25), taps, 4)
    for d in det:
        for v in d.values():
            assert np.max(np.abs(v)) < 1e-11
    # the approximation of a constant is the constant times 2^levels
    np.testing.assert_allclose(ll, 123.25 * 16, rtol=1e-13)


def test_subband_orientation():
    """A field varying only along axis 1 has energy only in ll and lh."""
    x = np.tile(_rand((1, 64), 6), (32, 1))
    b = dwt.dwt2(x, 8)
    assert np.max(np.abs(b["hl"])) < 1e-12 and np.max(np.abs(b["hh"])) < 1e-12
    assert np.max(np.abs(b["lh"])) > 0.1
