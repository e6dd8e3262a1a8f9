"""Tolerances shared by the GPU parity tests.

The FP32 path is held to 1e-4 relative against the FP64 oracle.  For arrays
the scale is the reference's largest magnitude: every element must satisfy
|got - ref| <= rtol * max|ref| (a residual or fingerprint has no meaningful
per-element relative error where it crosses zero), and the whole array
|got - ref|_2 <= rtol * |ref|_2.  PCE values use 1e-4 relative where
|ref| >= 1 and 1e-4 absolute below (an unmatched PCE sits near 0).
Gradient components are checked one by one, each against its own bound
(its own magnitude, or the sum of the magnitudes of the terms it adds up).
"""
import numpy as np

RTOL = 1e-4


def assert_scaled(got, ref, rtol=RTOL, what="array"):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, (what, got.shape, ref.shape)
    assert np.all(np.isfinite(got)), f"{what}: non-finite output"
    scale = float(np.max(np.abs(ref)))
    err = float(np.max(np.abs(got - ref)))
    assert err <= rtol * scale, f"{what}: max|err| {err:.3e} > {rtol:g} * max|ref| {scale:.3e}"
    l2 = float(np.linalg.norm(got - ref))
    nr = float(np.linalg.norm(ref))
    assert l2 <= rtol * nr, f"{what}: |err|_2 {l2:.3e} > {rtol:g} * |ref|_2 {nr:.3e}"
    return err / scale if scale > 0 else 0.0


def assert_pce(got, ref, rtol=RTOL, what="pce"):
    got = np.asarray(got, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    for g, r in zip(got, ref):
        tol = rtol * abs(r) if abs(r) >= 1.0 else rtol
        assert abs(g - r) <= tol, f"{what}: gpu {g!r} oracle {r!r}"


def components_ok(got, ref, bound, rtol=RTOL):
    """True where |got - ref| <= rtol * bound, component by component."""
    got = np.asarray(got, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    bound = np.asarray(bound, dtype=np.float64).ravel()
    return np.abs(got - ref) <= rtol * bound


def assert_components(got, ref, bound, rtol=RTOL, what="gradient"):
    ok = components_ok(got, ref, bound, rtol)
    rel = np.abs(np.asarray(got, np.float64).ravel() - np.asarray(ref, np.float64).ravel()) / np.maximum(
        np.asarray(bound, np.float64).ravel(), 1e-300)
    assert np.all(ok), f"{what}: gpu {np.asarray(got)} oracle {np.asarray(ref)} err/bound {rel} (rtol {rtol:g})"
