"""Pins of the oracle's bilinear resampling (mixed-media matching, Sec. V-B)."""
import numpy as np
from scipy import ndimage

from oracle import resample


def test_identity_at_scale_one():
    X = np.random.default_rng(1).normal(size=(13, 17))
    np.testing.assert_array_equal(resample.bilinear(X, 1.0, 13, 17), X)


def test_integer_offsets_at_scale_one_are_crops_with_edge_replication():
    """What the translation search of stabilised video relies on: at scale 1 an
    integer offset (oy, ox) reads X(y + oy, x + ox) exactly, clamped to the
    plane beyond its edges."""
    X = np.random.default_rng(4).normal(size=(15, 19))
    np.testing.assert_array_equal(resample.bilinear(X, 1.0, 9, 11, 3, 5), X[3:12, 5:16])
    Y = resample.bilinear(X, 1.0, 15, 19, 4, 2)
    rows = np.minimum(np.arange(15) + 4, 14)
    cols = np.minimum(np.arange(19) + 2, 18)
    np.testing.assert_array_equal(Y, X[np.ix_(rows, cols)])


def test_half_scale_is_the_two_by_two_mean():
    X = np.random.default_rng(2).normal(size=(12, 20))
    Y = resample.bilinear(X, 0.5, 6, 10)
    ref = X.reshape(6, 2, 10, 2).mean(axis=(1, 3))
    np.testing.assert_allclose(Y, ref, rtol=0, atol=1e-14)


def test_linear_ramps_are_reproduced():
    yy, xx = np.mgrid[0:40, 0:50].astype(np.float64)
    X = 3.0 * yy - 2.0 * xx + 7.0
    s, oy, ox = 0.73, 2, 3
    Y = resample.bilinear(X, s, 20, 25, oy, ox)
    fy = (np.arange(20) + oy + 0.5) / s - 0.5
    fx = (np.arange(25) + ox + 0.5) / s - 0.5
    ref = 3.0 * fy[:, None] - 2.0 * fx[None, :] + 7.0  # all inside the plane
    np.testing.assert_allclose(Y, ref, rtol=0, atol=1e-11)


def test_matches_scipy_order_one_with_edge_clamp():
    X = np.random.default_rng(3).normal(size=(31, 29))
    s, oh, ow, oy, ox = 1.37, 45, 41, 1, 4
    fy = (np.arange(oh) + oy + 0.5) / s - 0.5
    fx = (np.arange(ow) + ox + 0.5) / s - 0.5
    gy, gx = np.meshgrid(np.clip(fy, 0, 30), np.clip(fx, 0, 28), indexing="ij")
    ref = ndimage.map_coordinates(X, [gy, gx], order=1, mode="nearest")
    np.testing.assert_allclose(resample.bilinear(X, s, oh, ow, oy, ox), ref, rtol=0, atol=1e-12)


# ---------------------------------------------------------------- affine warp (stabilised video)
def test_affine_identity_and_integer_translation():
    X = np.random.default_rng(5).normal(size=(14, 18))
    np.testing.assert_array_equal(resample.affine(X, [1, 0, 0, 0, 1, 0], 14, 18), X)
    Y = resample.affine(X, [1, 0, 3, 0, 1, -2], 14, 18)  # column + 3, row - 2, edge replication
    rows = np.clip(np.arange(14) - 2, 0, 13)
    cols = np.clip(np.arange(18) + 3, 0, 17)
    np.testing.assert_array_equal(Y, X[np.ix_(rows, cols)])


def test_affine_quarter_turns_are_exact_permutations():
    """A rotation by 90 degrees about the centre of a square plane lands every
    output pixel on a source pixel: the result is np.rot90 exactly (up to the
    last bit of the trigonometric matrix)."""
    X = np.random.default_rng(6).normal(size=(11, 11))
    for k, th in ((1, np.pi / 2), (2, np.pi), (3, 3 * np.pi / 2)):
        Y = resample.affine(X, resample.rotation(th, 1.0, 11, 11, 11, 11), 11, 11)
        np.testing.assert_allclose(Y, np.rot90(X, k), rtol=0, atol=1e-12)


def test_affine_scale_and_crop_is_the_bilinear_resampler():
    """The mixed-media resampler is the affine warp with m0 = m4 = 1/s and the
    pixel-centre offsets; compared with the independently pinned bilinear()."""
    X = np.random.default_rng(7).normal(size=(33, 27))
    s, oh, ow, oy, ox = 0.61, 19, 15, 2, 1
    M = [1 / s, 0.0, (ox + 0.5) / s - 0.5, 0.0, 1 / s, (oy + 0.5) / s - 0.5]
    np.testing.assert_allclose(resample.affine(X, M, oh, ow), resample.bilinear(X, s, oh, ow, oy, ox),
                               rtol=0, atol=1e-12)


def test_affine_reproduces_planes_inside_and_matches_scipy():
    """A linear field is reproduced exactly where the samples stay inside the
    plane; a random plane matches scipy's order-1 map_coordinates with the
    same clamped coordinates (rotation, zoom and shear)."""
    yy, xx = np.mgrid[0:40, 0:44].astype(np.float64)
    X = 2.5 * xx - 1.25 * yy + 3.0
    M = resample.rotation(0.3, 1.2, 40, 44, 20, 22, ty=1.5, tx=-2.0)
    Y = resample.affine(X, M, 20, 22)
    oy, ox = np.mgrid[0:20, 0:22].astype(np.float64)
    u = M[0] * ox + M[1] * oy + M[2]
    v = M[3] * ox + M[4] * oy + M[5]
    assert u.min() > 0 and u.max() < 43 and v.min() > 0 and v.max() < 39
    np.testing.assert_allclose(Y, 2.5 * u - 1.25 * v + 3.0, rtol=0, atol=1e-11)
    R = np.random.default_rng(8).normal(size=(29, 31))
    for M in ([0.9, 0.2, 1.5, -0.1, 1.1, -0.7], resample.rotation(-0.05, 0.98, 29, 31, 29, 31, 0.4, -1.3)):
        Z = resample.affine(R, M, 25, 27)
        oy, ox = np.mgrid[0:25, 0:27].astype(np.float64)
        u = np.clip(M[0] * ox + M[1] * oy + M[2], 0, 30)
        v = np.clip(M[3] * ox + M[4] * oy + M[5], 0, 28)
        ref = ndimage.map_coordinates(R, [v, u], order=1, mode="nearest")
        np.testing.assert_allclose(Z, ref, rtol=0, atol=1e-12)


def test_rotation_matrix_maps_centres_and_composes():
    """rotation() sends the output centre to the input centre plus the
    translation, and a rotation by a then by b equals one by a + b."""
    M = resample.rotation(0.2, 1.1, 30, 40, 20, 24, ty=1.0, tx=2.0)
    cx, cy = (24 - 1) / 2, (20 - 1) / 2
    assert np.isclose(M[0] * cx + M[1] * cy + M[2], (40 - 1) / 2 + 2.0)
    assert np.isclose(M[3] * cx + M[4] * cy + M[5], (30 - 1) / 2 + 1.0)
    A = np.array(resample.rotation(0.1, 1.0, 9, 9, 9, 9)).reshape(2, 3)
    B = np.array(resample.rotation(0.25, 1.0, 9, 9, 9, 9)).reshape(2, 3)
    C = np.array(resample.rotation(0.35, 1.0, 9, 9, 9, 9)).reshape(2, 3)
    comp = A[:, :2] @ B[:, :2], A[:, :2] @ B[:, 2] + A[:, 2]
    np.testing.assert_allclose(comp[0], C[:, :2], atol=1e-14)
    np.testing.assert_allclose(comp[1], C[:, 2], atol=1e-12)
