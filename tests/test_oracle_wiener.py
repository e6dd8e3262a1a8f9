"""Pins of the oracle's Wiener shrinkage and residual W = I - F(I)."""
import numpy as np
import pytest

import synth
from oracle import dwt, pipeline, wiener


def _integral_box(q, w):
    """Window sums from a zero-padded summed-area table (independent method)."""
    r = w // 2
    H, W = q.shape
    S = np.zeros((H + 2 * r + 1, W + 2 * r + 1))
    S[1:, 1:] = np.cumsum(np.cumsum(np.pad(q, r), axis=0), axis=1)
    return S[w:w + H, w:w + W] - S[0:H, w:w + W] - S[w:w + H, 0:W] + S[0:H, 0:W]


@pytest.mark.parametrize("w", [3, 5, 7, 9])
def test_box_sum_vs_summed_area_table(w):
    q = synth.random_field((13, 21), synth.CFG_TEST, 2000 + w) ** 2
    np.testing.assert_allclose(wiener.box_sum(q, w), _integral_box(q, w), atol=1e-11)


def test_isolated_coefficient_closed_form():
    """A lone coefficient c: every window holds c^2 only, so the smallest
    estimate is the 9x9 one: var = max(0, c^2/81 - s2)."""
    for c, s2 in ((30.0, 1.0), (5.0, 1.0), (100.0, 9.0)):
        z = np.zeros((21, 21))
        z[10, 10] = c
        r = wiener.wiener_residual(z, s2)
        var = max(0.0, c * c / 81 - s2)
        assert abs(r[10, 10] - c * s2 / (var + s2)) < 1e-12
        # corner: the window is cut by the edge but the divisor stays w^2
        z = np.zeros((21, 21))
        z[0, 0] = c
        assert abs(wiener.wiener_residual(z, s2)[0, 0] - c * s2 / (var + s2)) < 1e-12


def test_two_coefficients_closed_form():
    """c1 at (10,10), c2 two columns away: the 3x3 window sees c1 only, the
    larger ones both.  Hand-computed estimates for c1."""
    z = np.zeros((21, 21))
    z[10, 10], z[10, 12] = 30.0, 90.0
    s2 = 1.0
    m = {3: 900 / 9, 5: 9000 / 25, 7: 9000 / 49, 9: 9000 / 81}
    var = min(max(0.0, v - s2) for v in m.values())  # = 99 (3x3 window)
    assert var == 99.0
    assert abs(wiener.wiener_residual(z, s2)[10, 10] - 30.0 * s2 / (var + s2)) < 1e-12
    z[10, 12] = 30.0  # now the 9x9 window wins: (1800/81 - 1)
    var = 1800 / 81 - 1
    assert abs(wiener.wiener_residual(z, s2)[10, 10] - 30.0 / (var + 1)) < 1e-12


def test_zero_noise_variance_gives_zero_residual():
    x = synth.tiny_camera(0, 1, 64, 48, cfg=synth.CFG_TEST)[0][0, :, :, 0].astype(float)
    W = pipeline.denoise_residual(x, sigma0=1e-9)
    assert np.max(np.abs(W)) < 1e-9


def test_huge_noise_variance_keeps_only_coarse_band():
    """rho -> 1 when s2 >> coefficients: W = I - reconstruction from LL4 alone."""
    x = synth.tiny_camera(0, 1, 64, 64, cfg=synth.CFG_TEST)[0][0, :, :, 0].astype(float)
    W = pipeline.denoise_residual(x, sigma0=1e8)
    ll, det = dwt.wavedec2(x, 16, 4)
    zero = [{k: np.zeros_like(v) for k, v in d.items()} for d in det]
    coarse = dwt.waverec2(ll, zero, 16)
    np.testing.assert_allclose(W, x - coarse, atol=1e-9)


def test_constant_image_zero_residual():
    W = pipeline.denoise_residual(np.full((40, 56), 77.0))
    assert np.max(np.abs(W)) < 1e-10


@pytest.mark.parametrize("shape", [(64, 64), (54, 70), (17, 33)])
def test_residual_plus_denoised_is_image(shape):
    x = synth.random_field(shape, synth.CFG_TEST, 7) * 20 + 128
    W = pipeline.denoise_residual(x)
    F = pipeline.denoised(x)
    np.testing.assert_allclose(F + W, x, atol=1e-10)


def test_padding_symmetric_and_cropped():
    assert pipeline.pad_amounts(1080) == (4, 4)
    assert pipeline.pad_amounts(1920) == (0, 0)
    assert pipeline.pad_amounts(3000) == (4, 4)
    assert pipeline.pad_amounts(17) == (7, 8)
    x = np.arange(17 * 3, dtype=float).reshape(17, 3)
    p = pipeline.pad_symmetric(x)
    assert p.shape == (32, 16)
    np.testing.assert_array_equal(p[7:24, 6:9], x)     # interior
    np.testing.assert_array_equal(p[6, 6:9], x[0])      # edge-including mirror
    np.testing.assert_array_equal(p[0, 6:9], x[6])
    np.testing.assert_array_equal(p[24, 6:9], x[16])


def test_level_weight_scales_noise_variance():
    """A weight w on a level is the same as sigma0^2 * w at that level: with all
    weights equal to 4 the residual equals the sigma0 = 2*3 residual."""
    x = synth.random_field((64, 64), synth.CFG_TEST, 8) * 10 + 100
    a = pipeline.denoise_residual(x, sigma0=3.0, level_weight=(4, 4, 4, 4))
    b = pipeline.denoise_residual(x, sigma0=6.0)
    np.testing.assert_allclose(a, b, atol=1e-12)
