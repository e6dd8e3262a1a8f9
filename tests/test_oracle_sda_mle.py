"""Pins of the oracle's SDA frames (Sec. III-B) and MLE fingerprint
(Sec. III-A/B), including the paper's variance statements and its
flat-vs-textured behaviour."""
import numpy as np
import pytest

import synth
from oracle import correlate, pipeline, sda


def test_groups_and_remainder():
    assert sda.groups(10, 4) == [(0, 4), (4, 4), (8, 2)]
    assert sda.groups(8, 1) == [(i, 1) for i in range(8)]
    assert sda.groups(5, 10) == [(0, 5)]


def test_sums_exact_vs_python_ints():
    g = synth.rng(synth.CFG_TEST, 3000)
    fr = g.integers(0, 256, size=(11, 5, 7, 3), dtype=np.uint8)
    sums, counts = sda.sda_sums(fr, 4)
    assert list(counts) == [4, 4, 3]
    for i, (s, n) in enumerate(sda.groups(11, 4)):
        for c in range(3):
            for y in range(5):
                for x in range(7):
                    assert sums[i, c, y, x] == sum(int(fr[j, y, x, c]) for j in range(s, s + n))


def test_identical_frames_average_to_the_frame():
    g = synth.rng(synth.CFG_TEST, 3001)
    f = g.integers(0, 256, size=(1, 9, 6, 1), dtype=np.uint8)
    fr = np.repeat(f, 7, axis=0)
    m = sda.sda_means(fr, 7)
    np.testing.assert_array_equal(m[0, 0], f[0, :, :, 0].astype(float))


def test_depth_one_is_the_frames():
    g = synth.rng(synth.CFG_TEST, 3002)
    fr = g.integers(0, 256, size=(5, 4, 6, 3), dtype=np.uint8)
    np.testing.assert_array_equal(sda.sda_means(fr, 1), np.moveaxis(fr, -1, 1).astype(float))


def test_f32_mean_is_correctly_rounded_division():
    """float32(S/n) with the division in float64 is the correctly rounded
    float32 quotient (53 >= 2*24 + 2); checked against exact rationals."""
    from fractions import Fraction
    g = synth.rng(synth.CFG_TEST, 3003)
    fr = g.integers(0, 256, size=(7, 3, 5, 1), dtype=np.uint8)
    s, n = sda.sda_sums(fr, 7)
    m32 = sda.sda_means_f32(fr, 7)
    for v, q in zip(s.ravel(), m32.ravel()):
        exact = Fraction(int(v), 7)
        cand = [np.float32(q), np.nextafter(np.float32(q), np.float32(0)), np.nextafter(np.float32(q), np.float32(1e9))]
        errs = [abs(Fraction(float(c)) - exact) for c in cand]
        assert errs[0] == min(errs)


def test_sda_noise_variance_divides_by_d():
    """Sec. III-B: the averaged noise has variance sigma1^2 / d."""
    g = synth.rng(synth.CFG_TEST, 3004)
    sigma1 = 2.0
    for d in (1, 4, 16):
        psi = g.normal(0, sigma1, size=(d * 64, 32, 32, 1))
        m = sda.sda_means(psi, d)
        v = np.var(m)
        assert abs(v / (sigma1 ** 2 / d) - 1) < 0.05


def test_mle_with_ideal_residuals_recovers_K_exactly():
    """With W_i = I_i * K (no noise, no content leakage), K_hat = K."""
    g = synth.rng(synth.CFG_TEST, 3005)
    K = g.normal(0, 0.02, size=(16, 24))
    imgs = [g.uniform(40, 220, size=(16, 24)) for _ in range(5)]
    A, B = pipeline.mle_accumulate([I * K for I in imgs], imgs)
    np.testing.assert_allclose(pipeline.mle_ratio(A, B), K, rtol=1e-13, atol=1e-17)


def test_mle_variance_matches_cramer_rao_form():
    """Sec. III-A, Eq. (conv1): with W_i = I_i K + psi_i and white psi of
    variance s1^2, the MLE's error variance is s1^2 / sum_i I_i^2."""
    g = synth.rng(synth.CFG_TEST, 3006)
    K = g.normal(0, 0.02, size=(64, 64))
    s1 = 3.0
    level = np.array([60.0, 120.0, 200.0, 90.0])
    imgs = [np.full((64, 64), v) for v in level]
    res = [I * K + g.normal(0, s1, size=I.shape) for I in imgs]
    A, B = pipeline.mle_accumulate(res, imgs)
    err = pipeline.mle_ratio(A, B) - K
    expect = s1 ** 2 / np.sum(level ** 2)
    assert abs(np.var(err) / expect - 1) < 0.05


def test_zero_denominator_gives_zero():
    A = np.array([[1.0, 2.0]])
    B = np.array([[0.0, 4.0]])
    np.testing.assert_array_equal(pipeline.mle_ratio(A, B), [[0.0, 0.5]])


@pytest.mark.slow
def test_planted_prnu_recovered():
    """Full pipeline (SDA d = 4, 4-level db8 denoiser, MLE) on 128 flat-scene
    frames of the tiny camera recovers the planted K with correlation > 0.99."""
    fr, K = synth.tiny_camera(0, 128, 128, 128, cfg=synth.CFG_TEST)
    A, B = pipeline.fingerprint_accumulate(fr, 4)
    Kh = pipeline.mle_ratio(A, B)[0]
    assert np.corrcoef(Kh.ravel(), K.ravel())[0, 1] > 0.99


@pytest.mark.slow
def test_flat_vs_textured_depth_trend():
    """Sec. III-B remarks and Table II: on flat scenes SDA matches the
    conventional estimate; on textured scenes the matched PCE falls as the
    SDA depth grows."""
    res = {}
    for textured in (False, True):
        fr, _ = synth.tiny_camera(5, 32, 128, 128, textured=textured, cfg=synth.CFG_TEST)
        qs, _ = synth.tiny_camera(5, 4, 128, 128, textured=textured, cfg=synth.CFG_TEST, first_frame=100)
        for d in (1, 4, 32):
            Kh = pipeline.camera_fingerprint(fr, d)
            p = []
            for q in qs:
                Wq, Iq = pipeline.query_residual(q)
                p.append(correlate.pce(Wq, Iq * Kh)["pce"])
            res[textured, d] = np.mean(p)
    assert abs(res[False, 32] / res[False, 1] - 1) < 0.03
    assert res[True, 1] > res[True, 4] > res[True, 32]
    assert res[True, 32] / res[True, 1] < 0.95


def _sda_mle_error_var(g, K, levels, d, s1, s2):
    """Empirical error variance of the SDA-d MLE when every frame of a group
    has the constant level of that group, the frame noise psi_i (variance s1^2)
    is averaged by the SDA, and each SDA frame's residual carries an error of
    its own (variance s2^2, the denoising error of the model)."""
    frames = np.concatenate([np.full((d,) + K.shape + (1,), v) for v in levels])
    psi = g.normal(0, s1, size=frames.shape)
    I = sda.sda_means(frames, d)[:, 0]  # [g][C][H][W] -> [g][H][W]
    P = sda.sda_means(psi, d)[:, 0]
    res = [I[j] * K + P[j] + g.normal(0, s2, size=K.shape) for j in range(len(levels))]
    A, B = pipeline.mle_accumulate(res, list(I))
    return np.var(pipeline.mle_ratio(A, B) - K), I


@pytest.mark.parametrize("d", [1, 3, 8])
def test_sda_mle_variance_form(d):
    """Sec. III-B: Var(K_hat) = (s1^2 / d + s2^2) / sum_j (I_j^SDA)^2."""
    g = synth.rng(synth.CFG_TEST, 3010 + d)
    K = g.normal(0, 0.02, size=(64, 64))
    s1, s2 = 3.0, 1.5
    levels = np.array([60.0, 140.0, 200.0, 90.0, 170.0])
    v, I = _sda_mle_error_var(g, K, levels, d, s1, s2)
    expect = (s1 ** 2 / d + s2 ** 2) / np.sum(levels ** 2)
    assert abs(v / expect - 1) < 0.08


def test_sda_frame_budget_for_equal_variance():
    """Sec. III-B: n conventional frames and m = n (s1^2 + d s2^2) / (s1^2 +
    s2^2) frames in SDA-d groups give the same error variance.  With s1^2 = 6,
    s2^2 = 2, d = 3 and n = 20 that is m = 30, ten SDA frames; a third as many
    SDA frames as the budget gives a larger variance."""
    g = synth.rng(synth.CFG_TEST, 3020)
    K = g.normal(0, 0.02, size=(96, 96))
    s1, s2, d, n = np.sqrt(6.0), np.sqrt(2.0), 3, 20
    m = n * (s1 ** 2 + d * s2 ** 2) / (s1 ** 2 + s2 ** 2)
    assert m == 30
    v_conv, _ = _sda_mle_error_var(g, K, np.full(n, 120.0), 1, s1, s2)
    v_sda, _ = _sda_mle_error_var(g, K, np.full(int(m) // d, 120.0), d, s1, s2)
    assert abs(v_sda / v_conv - 1) < 0.08
    v_short, _ = _sda_mle_error_var(g, K, np.full(int(m) // d // 3, 120.0), d, s1, s2)
    assert v_short > 2.0 * v_conv
