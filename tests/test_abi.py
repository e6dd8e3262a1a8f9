"""CPU checks of the C ABI: the library loads, exports every function the
header declares, its host-side filter matches the oracle's, and argument
validation rejects bad calls before anything is enqueued (no GPU needed)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from oracle import filters

pytest.importorskip("torch")
from paper_1909_04573_amd import prnu  # noqa: E402

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "prnu.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(prnu_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(prnu.LIB_PATH):
        pytest.fail("libprnu.so is not built (python -m paper_1909_04573_amd.build)")
    return prnu.lib()


def test_exports_every_declared_symbol(lib):
    declared = _declared()
    assert declared, "no declarations parsed"
    assert sorted(prnu.EXPORTS) == declared
    out = subprocess.run(["nm", "-D", "--defined-only", prnu.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (prnu_[a-z0-9_]+)", out))
    missing = [s for s in declared if s not in exported]
    assert not missing, missing
    for s in declared:
        getattr(lib, s)


@pytest.mark.parametrize("taps", [2, 4, 8, 12, 16, 20])
def test_host_filter_matches_oracle(lib, taps):
    got = np.array(prnu.filter_coefficients(taps))
    np.testing.assert_allclose(got, filters.lowpass(taps), rtol=0, atol=2e-15)


def test_default_params(lib):
    p = prnu.DenoiseParams()
    lib.prnu_default_denoise_params(ctypes.byref(p))
    assert (p.sigma0, p.levels, p.taps, list(p.level_weight)) == (3.0, 4, 16, [1.0] * 4)


def _ws_size(fn, *args):
    n = ctypes.c_size_t(0)
    rc = fn(*args, ctypes.byref(n))
    return rc, n.value


def test_workspace_queries(lib):
    p = prnu.denoise_params()
    rc, n = _ws_size(lib.prnu_denoise_residual_workspace_size, 4, 1080, 1920, ctypes.byref(p))
    assert rc == 0 and n >= 4 * 1088 * 1920 * 4
    rc, n8 = _ws_size(lib.prnu_fingerprint_accumulate_workspace_size, 400, 1080, 1920, 3, 50, ctypes.byref(p))
    assert rc == 0 and n8 > 0
    rc, n1 = _ws_size(lib.prnu_fingerprint_accumulate_workspace_size, 400, 1080, 1920, 3, 1, ctypes.byref(p))
    assert rc == 0 and n1 == 4 * n8  # batches of 32 SDA frames at d = 1, all 8 at d = 50
    rc, n12 = _ws_size(lib.prnu_fingerprint_accumulate_workspace_size, 400, 1080, 1920, 3, 12, ctypes.byref(p))
    assert rc == 0 and n12 == n1  # 34 SDA frames: batches of 32 either way
    rc, n = _ws_size(lib.prnu_fingerprint_finalize_workspace_size, 3, 1080, 1920, 7)
    assert rc == 0 and n > 1080 * 1920 * 16
    rc, n = _ws_size(lib.prnu_pce_match_workspace_size, 50, 4, 1080, 1920, 1)
    assert rc == 0 and n > 50 * 1080 * 1920 * 8
    rc, n = _ws_size(lib.prnu_query_residual_workspace_size, 50, 1080, 1920, 3, ctypes.byref(p), 7)
    assert rc == 0 and n > 0


def test_validation_rejects_before_enqueue(lib):
    p = prnu.denoise_params()
    P = ctypes.byref(p)
    fake = ctypes.c_void_p(0x100000)  # never dereferenced: every call below fails validation
    out = ctypes.c_void_p(0x200000)
    sda = lambda fr, dt, n, C, stride, d, sums, means: lib.prnu_sda_average(fr, dt, n, 16, 16, C, stride, d, sums,
                                                                             means, None, None, None)
    assert sda(None, 0, 8, 1, 0, 1, fake, fake) == prnu.PRNU_E_INVAL
    assert sda(fake, 0, 8, 2, 0, 1, None, fake) == prnu.PRNU_E_INVAL
    assert sda(fake, 0, 8, 1, 0, 0, None, fake) == prnu.PRNU_E_INVAL
    assert sda(fake, 1, 8, 1, 0, 1, fake, None) == prnu.PRNU_E_INVAL
    assert sda(fake, 9, 8, 1, 0, 1, None, fake) == prnu.PRNU_E_INVAL
    # frame strides: shorter than a frame, not a multiple of the sample size, negative, overflowing
    assert sda(fake, 0, 8, 1, 255, 1, None, fake) == prnu.PRNU_E_INVAL
    assert sda(fake, 2, 8, 1, 16 * 16 * 4 + 2, 1, None, fake) == prnu.PRNU_E_INVAL
    assert sda(fake, 0, 8, 1, -256, 1, None, fake) == prnu.PRNU_E_INVAL
    assert sda(fake, 0, 8, 1, (1 << 62), 1, None, fake) == prnu.PRNU_E_INVAL
    assert "frame_stride_bytes" in lib.prnu_last_error().decode()
    assert lib.prnu_denoise_residual(fake, 1, 15, 64, P, fake, fake, 1 << 30, None) == prnu.PRNU_E_INVAL
    assert lib.prnu_denoise_residual(fake, 1, 64, 64, P, out, fake, 16, None) == prnu.PRNU_E_WORKSPACE
    assert lib.prnu_denoise_residual(fake, 0, 64, 64, P, fake, fake, 1 << 30, None) == prnu.PRNU_E_INVAL
    bad = prnu.denoise_params(taps=6)
    assert lib.prnu_denoise_residual(fake, 1, 64, 64, ctypes.byref(bad), out, fake, 1 << 30, None) == \
        prnu.PRNU_E_UNSUPPORTED
    bad = prnu.denoise_params(levels=5)
    assert lib.prnu_denoise_residual(fake, 1, 64, 64, ctypes.byref(bad), out, fake, 1 << 30, None) == \
        prnu.PRNU_E_INVAL
    bad = prnu.denoise_params(sigma0=float("nan"))
    assert lib.prnu_denoise_residual(fake, 1, 64, 64, ctypes.byref(bad), out, fake, 1 << 30, None) == \
        prnu.PRNU_E_INVAL
    misaligned = ctypes.c_void_p(0x100010)
    assert lib.prnu_denoise_residual(fake, 1, 64, 64, P, out, misaligned, 1 << 30, None) == \
        prnu.PRNU_E_WORKSPACE
    assert lib.prnu_fingerprint_accumulate(fake, 0, 8, 64, 64, 1, 0, 1, P, 7, fake, fake, None, fake, 1 << 30,
                                           None) == prnu.PRNU_E_INVAL
    assert lib.prnu_fingerprint_accumulate(fake, 0, 8, 64, 64, 1, 0, 1, P, 0, None, fake, None, fake, 1 << 30,
                                           None) == prnu.PRNU_E_INVAL
    assert lib.prnu_fingerprint_accumulate(fake, 0, 8, 64, 64, 1, 64 * 64 - 1, 1, P, 0, fake, fake, None, fake,
                                           1 << 30, None) == prnu.PRNU_E_INVAL
    assert lib.prnu_fingerprint_finalize(fake, fake, 0, 1, 17, 64, 4, -1.0, fake, fake, 1 << 30,
                                         None) == prnu.PRNU_E_UNSUPPORTED  # 17 is not 5-smooth
    assert lib.prnu_fingerprint_finalize(fake, fake, 0, 1, 64, 64, 8, -1.0, fake, fake, 1 << 30,
                                         None) == prnu.PRNU_E_INVAL
    pp = prnu.PceParams(0, 11)
    assert lib.prnu_pce_match(fake, 1, fake, 1, 11, 64, None, ctypes.byref(pp), fake, None, None, fake,
                              1 << 30, None) == prnu.PRNU_E_INVAL
    assert lib.prnu_pce_match(fake, 1, fake, 1, 14, 64, None, ctypes.byref(pp), fake, None, None, fake,
                              1 << 30, None) == prnu.PRNU_E_UNSUPPORTED  # 7 is a factor of 14
    pp = prnu.PceParams(2, 11)
    assert lib.prnu_pce_match(fake, 1, fake, 1, 64, 64, None, ctypes.byref(pp), fake, None, None, fake,
                              1 << 30, None) == prnu.PRNU_E_INVAL
    assert "peak mode" in lib.prnu_last_error().decode()
    assert lib.prnu_query_residual(fake, 0, 1, 64, 64, 3, P, 16, fake, None, fake, 1 << 30,
                                   None) == prnu.PRNU_E_INVAL


def test_extract_blocks_validation(lib):
    fake = ctypes.c_void_p(0x1000)
    ok = (fake, 2, 64, 80, 16, fake, None)
    bad = [
        (None, 2, 64, 80, 16, fake, None), (fake, 2, 64, 80, 16, None, None), (fake, 0, 64, 80, 16, fake, None),
        (fake, 2, 0, 80, 16, fake, None), (fake, 2, 64, 80, 0, fake, None), (fake, 2, 64, 80, 65, fake, None),
        (fake, 2, 64, 1 << 16, 16, fake, None),
    ]
    for args in bad:
        assert lib.prnu_extract_blocks(*args) == prnu.PRNU_E_INVAL, args
    assert "prnu_extract_blocks" in lib.prnu_last_error().decode()
    assert len(ok) == 7


def test_resample_validation(lib):
    fake = ctypes.c_void_p(0x1000)
    bad = [
        (None, 1, 8, 8, 0.5, 0, 0, 4, 4, fake, None), (fake, 1, 8, 8, 0.5, 0, 0, 4, 4, None, None),
        (fake, 0, 8, 8, 0.5, 0, 0, 4, 4, fake, None), (fake, 1, 8, 8, 0.0, 0, 0, 4, 4, fake, None),
        (fake, 1, 8, 8, float("nan"), 0, 0, 4, 4, fake, None), (fake, 1, 8, 8, 0.5, -1, 0, 4, 4, fake, None),
        (fake, 1, 8, 8, 0.5, 0, 0, 0, 4, fake, None), (fake, 1, 0, 8, 0.5, 0, 0, 4, 4, fake, None),
    ]
    for args in bad:
        assert lib.prnu_resample_bilinear(*args) == prnu.PRNU_E_INVAL, args


def test_noalloc_validation(lib):
    """The no-allocation residual call rejects bad arguments, and a plane whose
    wavelet pyramid exceeds the static scratch, on the host before any device
    work."""
    p = prnu.denoise_params()
    P = ctypes.byref(p)
    fake = ctypes.c_void_p(0x100000)
    out = ctypes.c_void_p(0x200000)
    f = lib.prnu_denoise_residual_noalloc
    assert f(None, 1, 64, 64, P, out, None) == prnu.PRNU_E_INVAL
    assert f(fake, 1, 64, 64, P, fake, None) == prnu.PRNU_E_INVAL  # resid aliases img
    assert f(fake, 0, 64, 64, P, out, None) == prnu.PRNU_E_INVAL
    assert f(fake, 1, 15, 64, P, out, None) == prnu.PRNU_E_INVAL
    bad = prnu.denoise_params(taps=6)
    assert f(fake, 1, 64, 64, ctypes.byref(bad), out, None) == prnu.PRNU_E_UNSUPPORTED
    assert f(fake, 1, 4096, 4096, P, out, None) == prnu.PRNU_E_INVAL
    assert "static scratch" in lib.prnu_last_error().decode()


def test_warp_affine_validation(lib):
    """The affine warp rejects null pointers and bad sizes on the host."""
    fake = ctypes.c_void_p(0x100000)
    out = ctypes.c_void_p(0x200000)
    m = ctypes.c_void_p(0x300000)
    f = lib.prnu_warp_affine
    assert f(None, 1, 16, 16, m, 1, 8, 8, out, None) == prnu.PRNU_E_INVAL
    assert f(fake, 1, 16, 16, None, 1, 8, 8, out, None) == prnu.PRNU_E_INVAL
    assert f(fake, 1, 16, 16, m, 1, 8, 8, None, None) == prnu.PRNU_E_INVAL
    assert f(fake, 0, 16, 16, m, 1, 8, 8, out, None) == prnu.PRNU_E_INVAL
    assert f(fake, 1, 16, 16, m, 0, 8, 8, out, None) == prnu.PRNU_E_INVAL
    assert f(fake, 1, 16, 16, m, 70000, 8, 8, out, None) == prnu.PRNU_E_INVAL
    assert f(fake, 1, 0, 16, m, 1, 8, 8, out, None) == prnu.PRNU_E_INVAL
    assert f(fake, 1, 16, 16, m, 1, 8, 40000, out, None) == prnu.PRNU_E_INVAL


def test_host_sources_under_sanitizers(host_check):
    """The validation, workspace carving, filter design and error text of the
    host sources run clean under ASan + UBSan (the same rejections as above,
    from C), and the sanitizers are live: a planted heap over-read and a
    planted signed overflow in the check program are reported."""
    from paper_1909_04573_amd import build

    rc, out = host_check("abi")
    assert rc == 0 and "0 failed" in out, out
    assert "Sanitizer" not in out and "runtime error" not in out, out
    syms = subprocess.run(["nm", os.path.join(os.path.dirname(build.HOST_CHECK), "api.cpp.o")],
                          capture_output=True, text=True).stdout
    assert "__asan_report_load" in syms and "__ubsan_handle" in syms
    rc, out = host_check("plant-heap")
    assert rc != 0 and "AddressSanitizer: heap-buffer-overflow" in out, out
    rc, out = host_check("plant-ub")
    assert rc != 0 and "runtime error: signed integer overflow" in out, out


def test_gap_f64_validation(lib):
    """The FP64 gap rejects bad sizes, a DFT size with a factor 7, even
    neighbourhoods, negative theta and a short workspace on the host."""
    fake = ctypes.c_void_p(0x100000)
    out = ctypes.c_void_p(0x200000)
    qc = ctypes.c_void_p(0x300000)
    n = ctypes.c_size_t(0)
    ws_size = lib.prnu_pce_gap_f64_workspace_size
    assert ws_size(2, 8, 4, 64, 64, 4, 16, 11, ctypes.byref(n)) == 0 and n.value > 0
    assert ws_size(0, 8, 4, 64, 64, 4, 16, 11, ctypes.byref(n)) == prnu.PRNU_E_INVAL
    assert ws_size(2, 8, 4, 64, 70, 4, 16, 11, ctypes.byref(n)) == prnu.PRNU_E_UNSUPPORTED  # 7 divides 70
    assert ws_size(2, 8, 4, 64, 64, 4, 16, 10, ctypes.byref(n)) == prnu.PRNU_E_INVAL
    assert ws_size(2, 8, 4, 64, 64, 4, 6, 11, ctypes.byref(n)) == prnu.PRNU_E_UNSUPPORTED
    th = (ctypes.c_double * 5)(3.0, 1.0, 1.0, 1.0, 1.0)
    f = lib.prnu_pce_gap_f64
    assert f(None, 2, 8, fake, 4, qc, 64, 64, 4, 16, 11, th, out, None, fake, 1 << 30, None) == prnu.PRNU_E_INVAL
    assert f(fake, 2, 8, fake, 4, qc, 64, 64, 4, 16, 11, th, out, None, fake, 16, None) == prnu.PRNU_E_WORKSPACE
    bad = (ctypes.c_double * 5)(3.0, -1.0, 1.0, 1.0, 1.0)
    assert f(fake, 2, 8, fake, 4, qc, 64, 64, 4, 16, 11, bad, out, None, fake, 1 << 30, None) == prnu.PRNU_E_INVAL
    assert "theta" in lib.prnu_last_error().decode()
