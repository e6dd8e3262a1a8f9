"""Pins of the oracle's adjoint: finite differences on tiny inputs, the
scale identity of the level weights, and consistency with the forward
residual."""
import numpy as np
import pytest

import synth
from oracle import adjoint, pipeline


def _field(shape, k):
    return synth.random_field(shape, synth.CFG_TEST, 6000 + k)


def test_residual_matches_pipeline():
    x = synth.tiny_camera(0, 1, 48, 80, cfg=synth.CFG_TEST)[0][0, :, :, 0].astype(float)
    for lw in ((1, 1, 1, 1), (0.5, 2.0, 1.5, 0.7)):
        W1, _ = adjoint.residual_with_sensitivity(x, 3.0, lw)
        W2 = pipeline.denoise_residual(x, sigma0=3.0, level_weight=lw)
        np.testing.assert_allclose(W1, W2, atol=1e-12)


def test_pce_vjp_central_differences():
    x, y = _field((16, 20), 1), _field((16, 20), 2)
    y = y + 0.4 * x
    val, gx, gy = adjoint.pce_vjp(x, y, nbhd=5)
    for k in range(4):
        dx, dy = _field((16, 20), 10 + k), _field((16, 20), 20 + k)
        h = 1e-6
        fp = adjoint.pce_vjp(x + h * dx, y + h * dy, nbhd=5)[0]
        fm = adjoint.pce_vjp(x - h * dx, y - h * dy, nbhd=5)[0]
        fd = (fp - fm) / (2 * h)
        an = float(np.sum(gx * dx) + np.sum(gy * dy))
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1.0), (fd, an)


def test_residual_vjp_central_differences():
    """d<G, W(s)>/ds_l from the adjoint equals central differences in the
    per-level weights (no coefficient crosses m = s within the step)."""
    x = synth.patch_camera(0, 1, 64, 48)[0][0]
    G = _field((64, 48), 3)
    lw = np.array([1.0, 1.0, 1.0, 1.0])
    W0, sens = adjoint.residual_with_sensitivity(x, 3.0, lw)
    dLds = adjoint.residual_vjp_ds(G, sens)
    for l in range(4):
        h = 1e-6
        e = np.zeros(4)
        e[l] = h
        _, _, mp = adjoint.residual_with_sensitivity(x, 3.0, lw + e, want_masks=True)
        _, _, mm = adjoint.residual_with_sensitivity(x, 3.0, lw - e, want_masks=True)
        for a, b in zip(mp[l].values(), mm[l].values()):
            assert np.array_equal(a, b), "kink inside the step"
        Lp = np.sum(G * adjoint.residual_with_sensitivity(x, 3.0, lw + e)[0])
        Lm = np.sum(G * adjoint.residual_with_sensitivity(x, 3.0, lw - e)[0])
        fd = (Lp - Lm) / (2 * h) / 9.0  # d/ds_l with s_l = lambda_l * 9
        assert abs(fd - dLds[l]) <= 1e-5 * max(abs(dLds[l]), 1e-6), (l, fd, dLds[l])


def _diff_problem(H=64, W=64, ncam=2, nfp=8, nq=2):
    cams, qs, qc = [], [], []
    for c in range(ncam):
        p, _ = synth.patch_camera(c, nfp + nq, H, W)
        cams.append(p[:nfp])
        qs.extend(p[nfp:])
        qc.extend([c] * nq)
    return cams, np.stack(qs), qc


@pytest.mark.slow
def test_gap_loss_gradient_matches_central_differences():
    """The adjoint gradient of the matched-minus-unmatched PCE gap equals
    FP64 central differences (h = 1e-6) to 1e-5 relative at a kink-free
    point (all shrinkage masks identical at theta +- h)."""
    cams, qs, qc = _diff_problem()
    theta = np.array([3.0, 1.0, 1.0, 1.0, 1.0])
    L, g, _ = adjoint.gap_loss(theta, cams, qs, qc, d=4)
    h = 1e-6
    for k in range(5):
        e = np.zeros(5)
        e[k] = h
        mp = adjoint.kink_masks(theta + e, cams, qs, d=4)
        mm = adjoint.kink_masks(theta - e, cams, qs, d=4)
        assert np.array_equal(mp, mm), f"kink inside the step for component {k}"
        Lp = adjoint.gap_loss(theta + e, cams, qs, qc, d=4, want_grad=False)[0]
        Lm = adjoint.gap_loss(theta - e, cams, qs, qc, d=4, want_grad=False)[0]
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-5 * max(abs(g[k]), 1e-3 * abs(L)), (k, fd, g[k])


def test_level_weight_scale_identity():
    """s_l = lambda_l sigma0^2 gives sigma0 dL/dsigma0 = 2 sum_l lambda_l dL/dlambda_l."""
    cams, qs, qc = _diff_problem(H=48, W=48, nfp=4, nq=1)
    theta = np.array([2.5, 0.8, 1.3, 1.0, 0.6])
    _, g, _ = adjoint.gap_loss(theta, cams, qs, qc, d=2)
    lhs = theta[0] * g[0]
    rhs = 2.0 * float(np.dot(theta[1:], g[1:]))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1e-300) + 1e-300


def test_residual_cotangent_gives_positive_closed_form():
    """With the residual itself as cotangent (dL/dW = W) on a plane whose
    sides are multiples of 16 (no padding, so the DWT of W returns its
    residual coefficients r = c s / max(s, m)), every term of dL/ds_l is
    r [m > s] c / m = s (c / m)^2 [m > s] >= 0: dL/ds_l = s_l * sum of the
    squared sensitivities, and the sum of the terms' magnitudes equals it."""
    x = synth.patch_camera(1, 1, 96, 128)[0][0]
    lw = (1.0, 0.7, 1.3, 1.0)
    W, sens = adjoint.residual_with_sensitivity(x, 3.0, lw)
    ds, mag = adjoint.residual_vjp_ds(W, sens, want_abs=True)
    want = np.array([9.0 * lw[l] * sum(float(np.sum(v * v)) for v in sens[l].values()) for l in range(4)])
    np.testing.assert_allclose(ds, want, rtol=1e-12)
    np.testing.assert_allclose(mag, ds, rtol=1e-12)
    assert np.all(ds > 0)


def test_planted_level_one_error_is_caught_by_the_non_cancelling_check():
    """A level-1 sensitivity 1% off (the size of a mistake once seen in a
    GPU run) fails the per-level check of the residual cotangent
    (1e-4 of each level's own sum of term magnitudes), while every level of
    the correct sensitivities passes it."""
    from parity import components_ok

    x = synth.patch_camera(2, 1, 96, 128)[0][0]
    W, sens = adjoint.residual_with_sensitivity(x, 3.0)
    ref, mag = adjoint.residual_vjp_ds(W, sens, want_abs=True)
    assert np.all(components_ok(adjoint.residual_vjp_ds(W, sens), ref, mag))
    wrong = [dict(s) for s in sens]
    wrong[0] = {k: 1.01 * v for k, v in sens[0].items()}
    ok = components_ok(adjoint.residual_vjp_ds(W, wrong), ref, mag)
    assert not ok[0] and np.all(ok[1:])


def test_gap_loss_term_magnitudes_bound_the_gradient():
    """The per-component sums of term magnitudes bound the gradient's
    components (triangle inequality) and follow the same chain rule."""
    cams, qs, qc = _diff_problem(H=48, W=48, nfp=4, nq=1)
    theta = np.array([2.5, 0.8, 1.3, 1.0, 0.6])
    L, g, _, mag = adjoint.gap_loss(theta, cams, qs, qc, d=2, want_mag=True)
    L2, g2, _ = adjoint.gap_loss(theta, cams, qs, qc, d=2)
    assert L == L2 and np.array_equal(g, g2)
    assert np.all(mag >= np.abs(g))
    assert abs(theta[0] * mag[0] - 2.0 * float(np.dot(theta[1:], mag[1:]))) <= 1e-12 * theta[0] * mag[0]
