"""Pins of the oracle's post-processing (zero-mean, luma, DFT Wiener) and of
the correlation, PCE and NCC used for matching (Sec. II-A, Sec. IV)."""
import numpy as np
import pytest

import synth
from oracle import correlate, pipeline


def _f(shape, k):
    return synth.random_field(shape, synth.CFG_TEST, 4000 + k)


# ---------------------------------------------------------------- zero-mean
def test_zero_mean_rows_and_columns():
    Z = pipeline.zero_mean(_f((30, 44), 1) + 5)
    assert np.max(np.abs(Z.mean(axis=0))) < 1e-13
    assert np.max(np.abs(Z.mean(axis=1))) < 1e-13


def test_zero_mean_removes_separable_offsets_and_is_idempotent():
    X = _f((20, 30), 2)
    Z = pipeline.zero_mean(X)
    a, b = _f((20, 1), 3), _f((1, 30), 4)
    np.testing.assert_allclose(pipeline.zero_mean(X + a + b), Z, atol=1e-13)
    np.testing.assert_allclose(pipeline.zero_mean(Z), Z, atol=1e-13)


# ---------------------------------------------------------------- luma
def test_luma_weights():
    assert abs(sum(pipeline.LUMA) - 1.0) < 1e-15
    g = _f((5, 6), 5)
    np.testing.assert_allclose(pipeline.luma(np.stack([g, g, g])), g, atol=1e-15)
    e = np.zeros((3, 1, 1))
    for c, wgt in enumerate((0.299, 0.587, 0.114)):
        e[:] = 0
        e[c] = 1
        assert pipeline.luma(e)[0, 0] == wgt


# ---------------------------------------------------------------- DFT Wiener
def test_wiener_dft_limits():
    K = _f((48, 60), 6) * 0.01
    np.testing.assert_allclose(pipeline.wiener_dft(K, sigma2=1e30), K, atol=1e-15)
    assert np.max(np.abs(pipeline.wiener_dft(K, sigma2=1e-30))) < 1e-12


def test_wiener_dft_keeps_white_noise_and_kills_periodic_pattern():
    """White noise has a flat spectrum at the noise level (|F|/sqrt(N) has
    mean square var(K)), so it passes almost unchanged; a strong periodic
    component sits far above that level and is attenuated."""
    H, W = 96, 128
    K = _f((H, W), 7)
    out = pipeline.wiener_dft(K)
    assert np.corrcoef(out.ravel(), K.ravel())[0, 1] > 0.95
    yy, xx = np.mgrid[0:H, 0:W]
    cosine = 3.0 * np.cos(2 * np.pi * (5 * yy / H + 9 * xx / W))
    out2 = pipeline.wiener_dft(K + cosine)
    proj_in = np.sum((K + cosine) * cosine) / np.sum(cosine * cosine)
    proj_out = np.sum(out2 * cosine) / np.sum(cosine * cosine)
    assert proj_in > 0.95 and abs(proj_out) < 0.1


@pytest.mark.parametrize("sigma2", [None, 0.2])
def test_wiener_dft_single_cosine_closed_form(sigma2):
    """A cosine with whole periods has two isolated DFT bins of magnitude
    |F| = a HW / 2, so M^2 = a^2 HW / 4 there and 0 elsewhere.  The largest
    window (9 x 9) gives the smallest local mean M^2 / 81, so var_hat =
    M^2 / 81 - s2 and rho = s2 / (M^2 / 81).  The output is rho times the
    input.  s2 defaults to the cosine's population variance a^2 / 2."""
    H, W, a = 48, 60, 1.7
    yy, xx = np.mgrid[0:H, 0:W]
    K = a * np.cos(2 * np.pi * (5 * yy / H + 9 * xx / W))
    s2 = a * a / 2 if sigma2 is None else sigma2
    M2 = a * a * H * W / 4
    assert M2 / 81 > s2
    rho = s2 / (M2 / 81)
    np.testing.assert_allclose(pipeline.wiener_dft(K, sigma2=sigma2), rho * K, rtol=0, atol=1e-12)


@pytest.mark.parametrize("axis", [0, 1])
@pytest.mark.parametrize("sigma2", [None, 0.2])
def test_wiener_dft_edge_bins_closed_form(axis, sigma2):
    """Windows cut by the edge of the frequency array (zero extension there).

    K = b + a cos(2 pi t / n) along `axis` has three non-zero DFT bins: DC with
    M^2 = b^2 N, and bins 1 and n-1 of that axis with M^2 = a^2 N / 4 each
    (N = H W).  With zero extension every window (3..9) centred on DC or on
    bin 1 holds DC and bin 1 but not bin n-1, so all window sums there are
    S = b^2 N + a^2 N / 4 and the smallest mean is S / 81; every window on
    bin n-1 holds only that bin, smallest mean a^2 N / 4 / 81.  (A periodic
    wrap would put bin n-1 in the windows of DC and bin 1 and vice versa.)
    With rho = s2 / max(s2, smallest mean), the real part of the inverse is
    b rho_0 + (a/2)(rho_1 + rho_{n-1}) cos(2 pi t / n).  s2 defaults to the
    population variance a^2 / 2."""
    H, W, a, b = 48, 60, 1.7, 0.9
    N = H * W
    yy, xx = np.mgrid[0:H, 0:W]
    t, n = (yy, H) if axis == 0 else (xx, W)
    cosine = np.cos(2 * np.pi * t / n)
    K = b + a * cosine
    s2 = a * a / 2 if sigma2 is None else sigma2
    S = b * b * N + a * a * N / 4
    rho_0 = rho_1 = s2 / max(s2, S / 81)
    rho_last = s2 / max(s2, a * a * N / 4 / 81)
    assert rho_1 != rho_last
    want = b * rho_0 + 0.5 * a * (rho_1 + rho_last) * cosine
    np.testing.assert_allclose(pipeline.wiener_dft(K, sigma2=sigma2), want, rtol=0, atol=1e-12)


def test_postprocess_order_for_colour():
    P = np.stack([_f((16, 24), 8 + c) for c in range(3)])
    got = pipeline.postprocess(P, pipeline.FIN_ZM | pipeline.FIN_LUMA)
    ref = pipeline.luma(np.stack([pipeline.zero_mean(P[c]) for c in range(3)]))
    np.testing.assert_allclose(got, ref, atol=1e-14)


# ---------------------------------------------------------------- correlation
@pytest.mark.parametrize("shape", [(6, 10), (12, 15), (16, 20)])
def test_fft_xcorr_equals_brute_force(shape):
    X, Y = _f(shape, 10), _f(shape, 11)
    Cb = correlate.xcorr_brute(X, Y)
    Cf = correlate.xcorr_fft(X, Y)
    assert np.max(np.abs(Cb - Cf)) <= 1e-12 * np.max(np.abs(Cb))


def test_xcorr_parseval():
    X, Y = _f((24, 30), 12), _f((24, 30), 13)
    C = correlate.xcorr_fft(X, Y)
    N = X.size
    rhs = np.sum(np.abs(np.fft.fft2(X)) ** 2 * np.abs(np.fft.fft2(Y)) ** 2) / N
    assert abs(np.sum(C ** 2) - rhs) <= 1e-12 * rhs


def test_shift_moves_argmax_peak():
    X = _f((40, 48), 14)
    t = (7, 13)
    Y = np.roll(X, t, axis=(0, 1))  # Y(y) = X(y - t): C peaks at s = -t
    r = correlate.pce(X, Y, correlate.PEAK_ARGMAX)
    assert r["peak"] == ((-t[0]) % 40, (-t[1]) % 48)
    assert r["pce"] > 1000


def test_pce_hand_computed_surface():
    """PCE from a given correlation surface: 12x12, peak 10 at the origin,
    one other non-zero value 2 at (6,6), outside the 11x11 block around the
    origin (rows/cols -5..5 wrap to 7..11 and 0..5); energy = 4/(144-121)."""
    C = np.zeros((12, 12))
    C[0, 0] = 10.0
    C[6, 6] = 2.0
    C[3, 3] = 5.0  # inside the neighbourhood: excluded from the energy
    r = correlate.pce(np.ones((12, 12)), np.ones((12, 12)), correlate.PEAK_FIXED_00, C=C)
    assert abs(r["pce"] - 100.0 / (4.0 / 23.0)) < 1e-9
    C[0, 0] = -10.0
    r = correlate.pce(np.ones((12, 12)), np.ones((12, 12)), correlate.PEAK_FIXED_00, C=C)
    assert abs(r["pce"] + 575.0) < 1e-9


def test_ncc_limits():
    X = _f((20, 30), 15)
    assert abs(correlate.pce(X, 3 * X + 7)["ncc"] - 1) < 1e-13
    assert abs(correlate.pce(X, -X)["ncc"] + 1) < 1e-13
    assert correlate.pce(X, -X)["pce"] < 0


def test_unmatched_pce_is_chi_square_one():
    """Independent white fields: C(0) is Gaussian with the same variance as the
    other shifts, so |PCE| ~ chi^2_1 (mean 1), the signed PCE is symmetric
    about 0, and neither comes near the threshold 60."""
    vals = [correlate.pce(_f((32, 32), 100 + 2 * i), _f((32, 32), 101 + 2 * i))["pce"]
            for i in range(300)]
    vals = np.array(vals)
    assert abs(np.mean(np.abs(vals)) - 1.0) < 0.2
    assert abs(np.mean(vals)) < 0.25
    assert np.max(np.abs(vals)) < 60


def test_matched_tiny_camera_above_threshold():
    """Tiny workload: a held-out frame of the same camera exceeds PCE 60,
    a frame of another camera does not (Sec. IV threshold)."""
    fr, _ = synth.tiny_camera(0, 9, 128, 128)
    other, _ = synth.tiny_camera(1, 1, 128, 128)
    K = pipeline.camera_fingerprint(fr[:8], 4)
    Wq, Iq = pipeline.query_residual(fr[8])
    Wu, Iu = pipeline.query_residual(other[0])
    assert correlate.pce(Wq, Iq * K)["pce"] > 60
    assert abs(correlate.pce(Wu, Iu * K)["pce"]) < 60


# ------------------------------------------------------------------ block-wise PCE (Sec. IV protocol)
def test_blocks_partition():
    X = np.arange(7 * 11, dtype=np.float64).reshape(7, 11)
    bl = correlate.blocks(X, 3)
    assert len(bl) == 2 * 3
    # row-major block order, remainder rows/columns dropped
    np.testing.assert_array_equal(bl[0], X[0:3, 0:3])
    np.testing.assert_array_equal(bl[2], X[0:3, 6:9])
    np.testing.assert_array_equal(bl[4], X[3:6, 3:6])
    assert sum(b.size for b in bl) == 6 * 9


def test_pce_blocks_locates_a_planted_block():
    """A fingerprint term that shares noise with the query in one block only
    gives a large PCE there and chi-square-sized values elsewhere."""
    g = np.random.default_rng(11)
    b = 64
    X = g.normal(0, 1, size=(2 * b, 3 * b))
    Y = g.normal(0, 1, size=X.shape)
    Y[b:2 * b, b:2 * b] = X[b:2 * b, b:2 * b] + 0.5 * g.normal(0, 1, size=(b, b))  # block 4
    p = correlate.pce_blocks(X, Y, b)
    assert p.shape == (6,)
    assert p[4] > 1000
    assert np.all(np.abs(np.delete(p, 4)) < 30)


def test_pce_blocks_one_block_is_the_whole_field():
    g = np.random.default_rng(12)
    X = g.normal(0, 1, size=(48, 48))
    Y = 0.3 * X + g.normal(0, 1, size=X.shape)
    p = correlate.pce_blocks(X, Y, 48)
    assert p.shape == (1,)
    assert p[0] == correlate.pce(X, Y, correlate.PEAK_FIXED_00)["pce"]
