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
