"""CPU checks of the attribution statistics (TPR / FPR at the PCE threshold
of 60, ROC and its area) against hand-computed cases."""
import numpy as np
import pytest

from paper_1909_04573_amd import evaluation as ev


def test_rates_at_threshold():
    assert ev.tpr([10, 61, 60, 200]) == 0.5  # strictly above 60
    assert ev.fpr([0, 5, 70]) == pytest.approx(1 / 3)
    assert ev.tpr([1, 2, 3], thr=1.5) == pytest.approx(2 / 3)


def test_roc_hand_case():
    f, t = ev.roc([5, 3], [4, 1])
    # thresholds 5, 4, 3, 1 (descending): (0,.5) (.5,.5) (.5,1) (1,1)
    np.testing.assert_allclose(f, [0, 0, 0.5, 0.5, 1.0])
    np.testing.assert_allclose(t, [0, 0.5, 0.5, 1.0, 1.0])


def test_auc_is_the_area_under_roc_and_a_rank_probability():
    g = np.random.default_rng(3)
    m = g.normal(2.0, 1.0, 200)
    u = g.normal(0.0, 1.0, 300)
    f, t = ev.roc(m, u)
    area = float(np.sum((f[1:] - f[:-1]) * (t[1:] + t[:-1]) / 2))
    assert ev.auc(m, u) == pytest.approx(area, abs=1e-12)
    brute = np.mean(m[:, None] > u[None, :]) + 0.5 * np.mean(m[:, None] == u[None, :])
    assert ev.auc(m, u) == pytest.approx(brute, abs=1e-12)


def test_auc_extremes_and_ties():
    assert ev.auc([3, 4], [1, 2]) == 1.0
    assert ev.auc([1, 2], [3, 4]) == 0.0
    assert ev.auc([1, 1], [1, 1]) == 0.5


def test_smooth_floor_and_aligned_window():
    """Brute force: the largest size <= n whose prime factors are 2, 3 and 5."""
    def smooth(m):
        for q in (2, 3, 5):
            while m % q == 0:
                m //= q
        return m == 1
    for n in range(1, 400):
        m = ev.smooth_floor(n)
        assert m <= n and smooth(m) and not any(smooth(k) for k in range(m + 1, n + 1))
    assert ev.aligned_window(1080, 1920, 8) == (1024, 1875)
    assert ev.aligned_window(256, 256, 3) == (250, 250)


def test_segment_stabiliser_draws():
    """Synthetic segment stabiliser: one translation per run of frames, drawn
    from a stream of its own (the per-frame stabiliser's draws and the frames
    of still segments are unchanged), and a frame's pattern is K rolled by its
    translation."""
    import synth
    import torch

    n, H, W = 25, 24, 32
    fr0, K, sh0 = synth.stabilized_video_torch(0, 1, n, H, W, k_std=0.02, max_shift=3, device="cpu",
                                                cfg=synth.CFG_TEST)
    fr1, K1, sh1 = synth.stabilized_video_torch(0, 1, n, H, W, k_std=0.02, max_shift=3, device="cpu",
                                                cfg=synth.CFG_TEST, segment=10)
    np.testing.assert_array_equal(K, K1)
    assert sh1.shape == (n, 2) and np.abs(sh1).max() <= 3
    for s in range(0, n, 10):
        assert (sh1[s:s + 10] == sh1[s]).all()
    assert len({tuple(r) for r in sh1[::10]}) > 1 or not sh1.any()
    # frames with the same translation under both models are identical (same scene, noise draws)
    for i in range(n):
        if (sh0[i] == sh1[i]).all():
            assert torch.equal(fr0[i], fr1[i])


def test_alignment_helpers_refuse_windows_outside_the_reference():
    """Argument checks of the alignment search run on the host before any
    device work."""
    import torch

    W = torch.zeros((2, 64, 64))
    with pytest.raises(ValueError, match="leaves the reference"):
        ev.segment_shifts(W, W, torch.zeros((64, 64)), max_shift=8, margin=4)
    with pytest.raises(ValueError, match="leaves the reference"):
        ev.segment_shifts(W, W, torch.zeros((56, 56)), max_shift=4, margin=8, origin=2)  # 6 + 4 + 48 > 56
    A = torch.zeros((1, 50, 50), dtype=torch.float64)
    with pytest.raises(ValueError, match="exceeds the window margin"):
        ev.aligned_fingerprint(W, np.array([[0, 0], [5, 0]]), A, A, 4)
    with pytest.raises(ValueError, match="exceed the window"):
        ev.aligned_fingerprint(W, np.zeros((2, 2), dtype=np.int64), torch.zeros((1, 60, 56)), A, 4)


def test_signed_lag_of_a_circular_correlation():
    """Index i of a circular correlation of length n is the lag i or i - n; a
    brute-force circular correlation of a shifted copy peaks at its shift."""
    assert [ev.signed_lag(i, 8) for i in range(8)] == [0, 1, 2, 3, 4, -3, -2, -1]
    assert ev.signed_lag(952, 960) == -8 and ev.signed_lag(480, 960) == 480 and ev.signed_lag(481, 960) == -479
    rng = np.random.default_rng(3)
    y = rng.normal(size=(12, 15))
    for sy, sx in [(3, -4), (-5, 2), (0, 7)]:
        x = np.roll(y, (-sy, -sx), axis=(0, 1))  # x(t) = y(t + s)
        # C(l) = sum_t x(t + l) y(t) peaks where t + l + s = t, at l = -s
        C = np.array([[np.sum(np.roll(x, (-a, -b), axis=(0, 1)) * y) for b in range(15)] for a in range(12)])
        r, c = np.unravel_index(np.argmax(C), C.shape)
        assert (ev.signed_lag(r, 12), ev.signed_lag(c, 15)) == (-sy, -sx)


def _oracle_library(monkeypatch):
    """Stand-ins for the two library calls of the segment searches, computed
    by the oracle on host tensors: the host logic around them (cut-out
    offsets, sign of the shifts, lag wrap, gate) is what these tests check."""
    import torch

    from oracle import correlate, resample
    from paper_1909_04573_amd import prnu

    def resample_bilinear(x, scale, oh, ow, oy=0, ox=0):
        a = x.double().numpy()
        out = [resample.bilinear(p, scale, oh, ow, oy, ox) for p in (a[None] if a.ndim == 2 else a)]
        t = torch.from_numpy(np.stack(out)).float()
        return t[0] if a.ndim == 2 else t

    def pce_match(X, Y, modulate=None, peak_mode=0, nbhd=11, want_ncc=True, want_peak=True):
        nx, ny = X.shape[0], Y.shape[0]
        P = np.zeros((nx, ny))
        pk = np.zeros((nx, ny, 2), dtype=np.int32)
        for q in range(nx):
            for j in range(ny):
                y = Y[j].double().numpy() * (modulate[q].double().numpy() if modulate is not None else 1.0)
                r = correlate.pce(X[q].double().numpy(), y, peak_mode, nbhd)
                P[q, j], pk[q, j] = r["pce"], r["peak"]
        return torch.from_numpy(P), None, torch.from_numpy(pk)

    monkeypatch.setattr(prnu, "resample_bilinear", resample_bilinear)
    monkeypatch.setattr(prnu, "pce_match", pce_match)


def _shifted_frames(shifts, H=40, W=40, seed=11):
    """Residuals whose sensor pattern is K rolled by each frame's shift."""
    import torch

    rng = np.random.default_rng(seed)
    K = rng.normal(size=(H, W))
    I = rng.uniform(50, 200, size=(len(shifts), H, W))
    Wr = np.stack([I[j] * np.roll(K, tuple(s), axis=(0, 1)) + rng.normal(0, 5.0, size=(H, W))
                   for j, s in enumerate(shifts)])
    return torch.from_numpy(Wr).float(), torch.from_numpy(I).float(), torch.from_numpy(K).float()


def test_segment_search_conventions_on_the_host(monkeypatch):
    _oracle_library(monkeypatch)
    true = np.array([[0, 0], [2, -1], [-2, 2], [1, 0]])
    Wr, I, K = _shifted_frames(true)
    est, P = ev.segment_shifts(Wr, I, K, max_shift=2, margin=6)
    np.testing.assert_array_equal(est, -true)
    assert P.shape == (4, 25) and P.max(axis=1).min() > 60
    # a reference whose pixel (0, 0) is frame pixel (3, 3)
    est_o, P_o = ev.segment_shifts(Wr, I, K[3:, 3:].contiguous(), max_shift=2, margin=6, origin=3)
    np.testing.assert_array_equal(est_o, -true)
    np.testing.assert_allclose(P_o, P)
    # the plane search finds the same translations from one correlation per frame
    est_p, pce_p = ev.segment_shifts_plane(Wr, I, K, max_shift=2, margin=6)
    np.testing.assert_array_equal(est_p, -true)
    assert pce_p.min() > 60


def test_segment_search_gate_keeps_the_zero_shift(monkeypatch):
    """Frames of another camera: no peak reaches the gate, every frame keeps
    the zero shift; without the gate the argmax moves them."""
    import torch

    _oracle_library(monkeypatch)
    Wr, I, _ = _shifted_frames(np.array([[1, 1], [-2, 0], [0, 2]]))
    other = torch.from_numpy(np.random.default_rng(99).normal(size=(40, 40))).float()
    est, P = ev.segment_shifts(Wr, I, other, max_shift=2, margin=6, pce_min=25.0)
    assert P.max() < 25 and not est.any()
    est_p, _ = ev.segment_shifts_plane(Wr, I, other, max_shift=2, margin=6, pce_min=25.0)
    assert not est_p.any()
    est_free, _ = ev.segment_shifts(Wr, I, other, max_shift=2, margin=6)
    assert est_free.any()


def test_aligned_fingerprint_lines_patterns_up(monkeypatch):
    """Frames whose pattern is K rolled by s_j, with their shifts estimated as
    -s_j, are all translated onto K's window from (M, M) before the MLE (the
    accumulation call is captured instead of run)."""
    import torch

    from paper_1909_04573_amd import prnu

    _oracle_library(monkeypatch)
    seen = {}
    monkeypatch.setattr(prnu, "fingerprint_accumulate", lambda fr, d, A, B, p=None, ws=None: seen.update(fr=fr, d=d))
    K = np.random.default_rng(5).normal(size=(30, 36))
    s = np.array([[0, 0], [2, -3], [-3, 1]])
    means = torch.from_numpy(np.stack([np.roll(K, tuple(v), axis=(0, 1)) for v in s])).float()
    M = 3
    A = torch.zeros((1, 24, 27), dtype=torch.float64)
    ev.aligned_fingerprint(means, -s, A, A, M)
    assert seen["d"] == 1 and tuple(seen["fr"].shape) == (3, 24, 27, 1)
    for j in range(3):
        np.testing.assert_array_equal(seen["fr"][j, :, :, 0].numpy(), K[M:M + 24, M:M + 27].astype(np.float32))


# ---------------------------------------------------------------- equivalence and variance model
def test_equal_variance_images_budget():
    """The SDA frame budget of Sec. III-B: no scene term gives m = n; the
    values of the simulated budget pin (s1^2 = 6, s2^2 = 2, d = 3, n = 20 ->
    m = 30); m grows linearly in d with slope n s2^2 / (s1^2 + s2^2)."""
    assert ev.equal_variance_images(50, 4.0, 0.0, 10) == 50.0
    assert ev.equal_variance_images(20, 6.0, 2.0, 3) == 30.0
    assert ev.equal_variance_images(20, 6.0, 2.0, 1) == 20.0
    a, b = ev.equal_variance_images(40, 3.0, 1.0, 5), ev.equal_variance_images(40, 3.0, 1.0, 6)
    assert abs((b - a) - 40 * 1.0 / 4.0) < 1e-12
    for bad in [(10, -1.0, 1.0, 2), (10, 0.0, 0.0, 2), (10, 1.0, 1.0, 0)]:
        with pytest.raises(ValueError):
            ev.equal_variance_images(*bad)


@pytest.mark.parametrize("s1,s2", [(4.0, 0.0), (3.25, 0.6), (1.0, 2.0)])
def test_variance_components_recover_generator_variances(s1, s2):
    """R residuals W_r = P + xi + psi_r with a scene term xi ~ N(0, s2) shared
    by all r and noise psi_r ~ N(0, s1) drawn per r: the estimator returns
    (s1, s2) within the sampling error of 256 x 256 pixels."""
    g = np.random.default_rng(1909)
    R, shape = 16, (256, 256)
    P = g.normal(0, 0.5, size=shape)
    xi = g.normal(0, np.sqrt(s2), size=shape)
    W = P + xi + g.normal(0, np.sqrt(s1), size=(R,) + shape)
    e1, e2 = ev.variance_components(W, P)
    assert abs(e1 / s1 - 1) < 0.02
    assert abs(e2 - s2) < 0.03 * max(s2, 1.0)


def test_variance_components_exact_cases():
    """No noise: s1 = 0 and s2 is the scene term's mean square exactly; the
    PRNU term itself contributes nothing; too few residuals are refused."""
    P = np.arange(12.0).reshape(3, 4)
    xi = np.array([[1.0, -1.0, 2.0, 0.0]] * 3)
    W = np.stack([P + xi] * 4)
    s1, s2 = ev.variance_components(W, P)
    assert s1 == 0.0 and s2 == pytest.approx(np.mean(xi ** 2))
    assert ev.variance_components(np.stack([P, P]), P) == (0.0, 0.0)
    with pytest.raises(ValueError):
        ev.variance_components(W[:1], P)
    with pytest.raises(ValueError):
        ev.variance_components(W, P[:2])


def test_equivalent_images_search():
    conv = {40: 0.26, 50: 0.5, 60: 0.7, 80: 0.95, 100: 0.99}
    sda = {50: 0.3, 75: 0.71, 100: 0.95, 125: 0.99}
    got = ev.equivalent_images(conv, sda)
    assert got == {40: 50, 50: 75, 60: 75, 80: 100, 100: 125}
    assert ev.equivalent_images({10: 1.0}, {50: 0.99, 100: 0.999}) == {10: None}
    assert ev.equivalent_images({10: 0.5}, {100: 0.5, 50: 0.5}) == {10: 50}  # ties reach, smallest m
    assert ev.equivalent_images({}, {50: 1.0}) == {}


# ---------------------------------------------------------------- rotations (stabilised video)
def _oracle_warp(monkeypatch):
    """Stand-in for prnu_warp_affine computed by the oracle on host tensors."""
    import torch

    from oracle import resample
    from paper_1909_04573_amd import prnu

    def warp_affine(x, mats, oh, ow):
        a = x.double().numpy()
        a = a[None] if a.ndim == 2 else a
        m = np.asarray(mats, dtype=np.float64).reshape(-1, 6)
        return torch.from_numpy(np.stack([resample.affine(a[k % len(a)], m[k], oh, ow) for k in range(len(m))])).float()

    monkeypatch.setattr(prnu, "warp_affine", warp_affine)


def _posed_frames(poses, H=56, W=56, seed=21):
    """Residuals whose pattern at frame pixel p is K(c + R(theta)(p - c) + d)."""
    import torch

    from oracle import resample

    rng = np.random.default_rng(seed)
    K = rng.normal(size=(H, W))
    I = rng.uniform(50, 200, size=(len(poses), H, W))
    Wr = []
    for j, (t, dy, dx) in enumerate(poses):
        m = ev.reference_pose_matrix(t, H, W, 0, 0)
        m[2] += dx
        m[5] += dy
        Wr.append(I[j] * resample.affine(K, m, H, W) + rng.normal(0, 5.0, size=(H, W)))
    return torch.from_numpy(np.stack(Wr)).float(), torch.from_numpy(I).float(), torch.from_numpy(K).float()


def test_pose_matrices_reduce_to_translations():
    """At angle 0 the reference cut-out is the crop from (margin - origin) and
    the alignment the translation of aligned_fingerprint; a pose and its
    alignment compose to the window's offset."""
    np.testing.assert_allclose(ev.reference_pose_matrix(0.0, 40, 50, 6, 2), [1, 0, 4, 0, 1, 4], atol=1e-12)
    np.testing.assert_allclose(ev.alignment_matrix(0.0, 2, -3, 40, 50, 5), [1, 0, 8, 0, 1, 3], atol=1e-12)
    t, dy, dx, H, W, M = 0.03, 2.0, -1.0, 60, 80, 7
    R = np.array(ev.reference_pose_matrix(t, H, W, 0, 0)).reshape(2, 3)
    R[:, 2] += (dx, dy)
    A = np.array(ev.alignment_matrix(t, dy, dx, H, W, M)).reshape(2, 3)
    comp = R[:, :2] @ A[:, :2], R[:, :2] @ A[:, 2] + R[:, 2]
    np.testing.assert_allclose(comp[0], np.eye(2), atol=1e-12)
    np.testing.assert_allclose(comp[1], [M, M], atol=1e-9)


def test_pose_search_recovers_rotations_and_translations(monkeypatch):
    """Frames rotated by angles of the candidate grid and translated by
    integers: every pose comes back exactly (on 56 x 56 frames neighbouring
    angles still correlate, so only the winner is checked); frames of
    another camera keep the zero pose under the gate."""
    _oracle_library(monkeypatch)
    _oracle_warp(monkeypatch)
    angles = [-0.08, -0.04, 0.0, 0.04, 0.08]
    true = np.array([[0.0, 0, 0], [0.04, 2, -1], [-0.08, -2, 2], [0.08, 1, 0], [-0.04, 0, -2]])
    Wr, I, K = _posed_frames(true)
    est, P = ev.segment_poses(Wr, I, K, angles, max_shift=3, margin=8)
    np.testing.assert_allclose(est, true, atol=1e-12)
    for j in range(len(true)):
        a = angles.index(true[j, 0])
        assert P[j, a] > 60 and P[j, a] == P[j].max()
    other = np.random.default_rng(77).normal(size=K.shape)
    import torch
    est_o, _ = ev.segment_poses(Wr, I, torch.from_numpy(other).float(), angles, max_shift=3, margin=8,
                                pce_min=25.0)
    assert not est_o.any()


def test_affine_alignment_lines_rotated_patterns_up(monkeypatch):
    """Smooth patterns posed by (theta, d) and aligned back with their poses
    match the reference window from (M, M) (interpolated twice: correlation
    above 0.999 on a smooth field); the accumulation call is captured."""
    import torch
    from scipy import ndimage

    from oracle import resample
    from paper_1909_04573_amd import prnu

    _oracle_warp(monkeypatch)
    seen = {}
    monkeypatch.setattr(prnu, "fingerprint_accumulate", lambda fr, d, A, B, p=None, ws=None: seen.update(fr=fr, d=d))
    H = W = 64
    K = ndimage.gaussian_filter(np.random.default_rng(9).normal(size=(H, W)), 3.0)
    poses = np.array([[0.0, 0, 0], [0.05, 2, -3], [-0.06, -3, 1]])
    frames = []
    for t, dy, dx in poses:
        m = ev.reference_pose_matrix(t, H, W, 0, 0)
        m[2] += dx
        m[5] += dy
        frames.append(resample.affine(K, m, H, W))
    M, h, w = 8, 48, 48
    A = torch.zeros((1, h, w), dtype=torch.float64)
    ev.aligned_fingerprint_affine(torch.from_numpy(np.stack(frames)).float(), poses, A, A, M)
    assert seen["d"] == 1 and tuple(seen["fr"].shape) == (3, h, w, 1)
    ref = K[M:M + h, M:M + w]
    np.testing.assert_allclose(seen["fr"][0, :, :, 0].numpy(), ref, atol=1e-6)
    for j in (1, 2):
        got = seen["fr"][j, :, :, 0].numpy().astype(np.float64)
        c = np.corrcoef(got[4:-4, 4:-4].ravel(), ref[4:-4, 4:-4].ravel())[0, 1]
        assert c > 0.999, c
