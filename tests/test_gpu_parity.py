"""GPU parity: every C-ABI entry point against the FP64 oracle on seeded
synthetic inputs (element by element), at small sizes that span several
tiles with ragged tails and at the 1080p video size."""
import sys

import numpy as np
import pytest

import synth
from oracle import correlate, pipeline, resample, sda
from parity import RTOL, assert_pce, assert_scaled

torch = pytest.importorskip("torch")
from paper_1909_04573_amd import prnu  # noqa: E402

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    d = torch.device("cuda:0")
    prnu.lib()
    return d


def up(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def down(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _u8(shape, key):
    return synth.rng(synth.CFG_TEST, 5000 + key).integers(0, 256, size=shape, dtype=np.uint8)


# ------------------------------------------------------------------ SDA
@pytest.mark.parametrize("n,H,W,C,d", [(8, 256, 256, 1, 4), (8, 256, 256, 1, 1), (10, 72, 104, 3, 4),
                                       (7, 17, 33, 3, 3), (5, 16, 16, 1, 2), (12, 1080, 1920, 3, 5)])
def test_sda_u8_bit_exact(dev, n, H, W, C, d):
    _log(f"sda u8 n={n} {H}x{W}x{C} d={d}")
    fr = _u8((n, H, W, C), n * 131 + H)
    sums, means = prnu.sda_average(up(fr, dev), d)
    rs, _ = sda.sda_sums(fr, d)
    rm = sda.sda_means_f32(fr, d)
    np.testing.assert_array_equal(down(sums), rs)
    np.testing.assert_array_equal(down(means).view(np.uint32), rm.view(np.uint32))


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_sda_float_frames(dev, dtype):
    _log(f"sda {dtype}")
    g = synth.rng(synth.CFG_TEST, 5100)
    fr = g.uniform(0, 255, size=(9, 40, 56, 1)).astype(np.float32)
    t = up(fr, dev)
    if dtype == "bf16":
        t = t.to(torch.bfloat16)
        fr = t.float().cpu().numpy()
    _, means = prnu.sda_average(t, 4, want_sums=False)
    ref = sda.sda_means(fr.astype(np.float64), 4).astype(np.float32)
    np.testing.assert_array_equal(down(means).view(np.uint32), ref.view(np.uint32))


def _spaced(fr, layout, dev):
    """The frames fr [n][H][W][C] (numpy or a device tensor) as a device view
    whose frames are dense but spaced apart: every other frame of a buffer,
    or one frame per slot of H*W*C + pad samples."""
    t = fr if isinstance(fr, torch.Tensor) else up(fr, dev)
    n, H, W, C = t.shape
    hwc = H * W * C
    if layout == "every_other":
        buf = torch.zeros((2 * n, H, W, C), dtype=t.dtype, device=dev)
        buf[::2] = t
        return buf[::2]
    pad = {"slot_pad64": 64, "slot_pad3": 3}[layout]
    buf = torch.zeros((n, hwc + pad), dtype=t.dtype, device=dev)
    buf[:, :hwc] = t.reshape(n, -1)
    return buf.as_strided((n, H, W, C), (hwc + pad, W * C, C, 1))


@pytest.mark.parametrize("layout", ["every_other", "slot_pad64", "slot_pad3"])
@pytest.mark.parametrize("C", [1, 3])
def test_sda_spaced_frames_and_counts(dev, layout, C):
    """Frames spaced apart in memory (frame_stride_bytes) give the oracle's
    exact sums and means; counts[g] are the group sizes n_i (Sec. III-B),
    the last group shorter.  slot_pad3 makes the stride odd: the one-pixel
    path instead of the dword-quad path."""
    n, H, W, d = 11, 40, 56, 4
    _log(f"sda spaced {layout} C={C}")
    fr = _u8((n, H, W, C), 70 + C)
    sums, means, counts = prnu.sda_average(_spaced(fr, layout, dev), d, want_counts=True)
    rs, rc = sda.sda_sums(fr, d)
    np.testing.assert_array_equal(down(sums), rs)
    np.testing.assert_array_equal(down(means).view(np.uint32), sda.sda_means_f32(fr, d).view(np.uint32))
    np.testing.assert_array_equal(down(counts), rc)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_sda_nonfinite_flag(dev, dtype):
    """A NaN or infinite sample sets PRNU_STATUS_NONFINITE (its group's mean
    is not finite, the others are unchanged); finite frames leave the word
    clear.  Spaced float frames give the dense result."""
    _log(f"sda non-finite {dtype}")
    g = synth.rng(synth.CFG_TEST, 5200)
    fr = g.uniform(0, 255, size=(9, 24, 40, 3)).astype(np.float32)
    tdt = torch.float32 if dtype == "f32" else torch.bfloat16
    st = torch.zeros(1, dtype=torch.int32, device=dev)
    t = up(fr, dev).to(tdt)
    _, m0 = prnu.sda_average(t, 4, want_sums=False, status=st)
    assert int(down(st)[0]) == 0
    _, m1 = prnu.sda_average(_spaced(t, "slot_pad3", dev), 4, want_sums=False)
    np.testing.assert_array_equal(down(m1).view(np.uint32), down(m0).view(np.uint32))
    for bad in (float("nan"), float("inf"), -float("inf")):
        st.zero_()
        t2 = t.clone()
        t2[5, 7, 11, 2] = bad
        _, m2 = prnu.sda_average(t2, 4, want_sums=False, status=st)
        assert int(down(st)[0]) == prnu.STATUS_NONFINITE
        m2, m0h = down(m2), down(m0)
        assert not np.isfinite(m2[1, 2, 7, 11])
        mask = np.ones(m2.shape, bool)
        mask[1, 2, 7, 11] = False
        np.testing.assert_array_equal(m2[mask], m0h[mask])


# ------------------------------------------------------------------ denoiser
DENOISE_CASES = [
    (256, 256, 16, 4, (1, 1, 1, 1)),
    (96, 160, 16, 4, (1, 1, 1, 1)),
    (17, 33, 16, 4, (1, 1, 1, 1)),
    (200, 136, 8, 4, (1, 1, 1, 1)),
    (64, 64, 16, 2, (1, 1, 1, 1)),
    (128, 96, 16, 4, (0.5, 1.5, 2.0, 0.25)),
    (130, 1000, 16, 3, (1, 1, 1, 1)),
]


@pytest.mark.parametrize("H,W,taps,levels,lw", DENOISE_CASES)
def test_denoise_residual(dev, H, W, taps, levels, lw):
    _log(f"denoise {H}x{W} taps={taps} levels={levels} lw={lw}")
    g = synth.rng(synth.CFG_TEST, 5200 + H)
    img = np.stack([synth.textured_scene(H, W, g, sigma=3.0) + g.normal(0, 2, (H, W)),
                    g.uniform(0, 255, (H, W))]).astype(np.float32)
    p = prnu.denoise_params(3.0, levels, taps, lw)
    got = down(prnu.denoise_residual(up(img, dev), p))
    for k in range(2):
        ref = pipeline.denoise_residual(img[k].astype(np.float64), sigma0=3.0, levels=levels, taps=taps,
                                        level_weight=lw)
        assert_scaled(got[k], ref, what=f"W[{k}]")


def test_denoise_residual_1080p(dev):
    _log("denoise 1080x1920")
    fr, _ = synth.video_camera(0, 1, 1080, 1920, 1, cfg=synth.CFG_TEST)
    img = fr[0, :, :, 0].astype(np.float32)
    got = down(prnu.denoise_residual(up(img, dev)))
    ref = pipeline.denoise_residual(img.astype(np.float64))
    assert_scaled(got, ref, what="W 1080p")


# ------------------------------------------------------------------ MLE accumulation
ACC_CASES = [
    ("tiny d=1", 8, 256, 256, 1, 1),
    ("tiny d=4", 8, 256, 256, 1, 4),
    ("rgb ragged remainder", 10, 72, 104, 3, 4),
    ("rgb d=1 frames read in place", 10, 72, 104, 3, 1),
    ("d=3", 9, 64, 80, 1, 3),
    ("many batches", 80, 48, 48, 1, 2),  # 40 SDA frames: a batch of 32 and a ragged one of 8
]


def _frames_for(n, H, W, C, key):
    if C == 1:
        fr, _ = synth.tiny_camera(key, n, H, W, cfg=synth.CFG_TEST)
    else:
        fr, _ = synth.video_camera(key, n, H, W, C, cfg=synth.CFG_TEST)
    return fr


@pytest.mark.parametrize("name,n,H,W,C,d", ACC_CASES)
def test_fingerprint_accumulate(dev, name, n, H, W, C, d):
    _log(f"accumulate {name}")
    fr = _frames_for(n, H, W, C, 7)
    A, B = prnu.new_accumulators(C, H, W, device=dev)
    prnu.fingerprint_accumulate(up(fr, dev), d, A, B)
    Ar, Br = pipeline.fingerprint_accumulate(fr, d)
    assert_scaled(down(A), Ar, what="A")
    assert_scaled(down(B), Br, rtol=1e-7, what="B")
    if d in (1, 2, 4):  # means are exact in float32: B is exact
        np.testing.assert_array_equal(down(B), Br)


@pytest.mark.parametrize("mode", [prnu.ACC_KAHAN_F32, prnu.ACC_F32])
def test_accumulator_modes(dev, mode):
    _log(f"accumulate mode {mode}")
    fr = _frames_for(24, 64, 64, 1, 8)
    A, B = prnu.new_accumulators(1, 64, 64, mode, device=dev)
    prnu.fingerprint_accumulate(up(fr, dev), 1, A, B, acc_mode=mode)
    Ar, Br = pipeline.fingerprint_accumulate(fr, 1)
    a, b = down(A), down(B)
    if mode == prnu.ACC_KAHAN_F32:
        a = a[0].astype(np.float64) + a[1]
        b = b[0].astype(np.float64) + b[1]
        assert_scaled(b, Br, rtol=1e-9, what="B kahan")
    else:
        assert_scaled(b, Br, rtol=1e-6, what="B f32")
    assert_scaled(a, Ar, what="A")
    K = down(prnu.fingerprint_finalize(A, B, mode, flags=0))
    assert_scaled(K, pipeline.mle_ratio(Ar, Br)[0], what="K")


def test_streaming_calls_add_up(dev):
    _log("accumulate streaming")
    fr = _frames_for(16, 64, 64, 1, 9)
    t = up(fr, dev)
    A1, B1 = prnu.new_accumulators(1, 64, 64, device=dev)
    prnu.fingerprint_accumulate(t, 4, A1, B1)
    A2, B2 = prnu.new_accumulators(1, 64, 64, device=dev)
    prnu.fingerprint_accumulate(t[:8].contiguous(), 4, A2, B2)
    prnu.fingerprint_accumulate(t[8:].contiguous(), 4, A2, B2)
    np.testing.assert_allclose(down(A2), down(A1), rtol=0, atol=1e-12 * float(np.abs(down(A1)).max()))
    np.testing.assert_array_equal(down(B2), down(B1))


@pytest.mark.parametrize("layout,d", [("every_other", 1), ("slot_pad3", 1), ("slot_pad64", 3)])
def test_accumulate_spaced_frames(dev, layout, d):
    """Spaced frames accumulate exactly as the same frames packed densely
    (at d = 1 the spaced u8 frames go through the SDA kernel instead of being
    read in place: same values, same arithmetic)."""
    _log(f"accumulate spaced {layout} d={d}")
    fr = _frames_for(7, 72, 104, 3, 12)
    A0, B0 = prnu.new_accumulators(3, 72, 104, device=dev)
    prnu.fingerprint_accumulate(up(fr, dev), d, A0, B0)
    A1, B1 = prnu.new_accumulators(3, 72, 104, device=dev)
    prnu.fingerprint_accumulate(_spaced(fr, layout, dev), d, A1, B1)
    np.testing.assert_array_equal(down(A1), down(A0))
    np.testing.assert_array_equal(down(B1), down(B0))


def test_accumulator_state_counts_and_flag(dev):
    """The accumulator state counts the frames and SDA frames folded in, over
    calls and over the call's internal batches (40 SDA frames at d = 1 cross
    a batch), and collects the non-finite-input flag of float frames."""
    _log("accumulator state")
    fr = _frames_for(57, 64, 64, 1, 13)
    t = up(fr, dev)
    A, B = prnu.new_accumulators(1, 64, 64, device=dev)
    st = prnu.new_acc_state(dev)
    prnu.fingerprint_accumulate(t[:40], 1, A, B, state=st)
    assert down(st).tolist() == [40, 40, 0]
    prnu.fingerprint_accumulate(t[40:], 5, A, B, state=st)
    assert down(st).tolist() == [57, 44, 0]  # 17 frames in groups of 5: 4 SDA frames
    ff = up(fr.astype(np.float32), dev)
    st2 = prnu.new_acc_state(dev)
    A2, B2 = prnu.new_accumulators(1, 64, 64, device=dev)
    prnu.fingerprint_accumulate(ff[:10], 2, A2, B2, state=st2)
    assert down(st2).tolist() == [10, 5, 0]
    ff[3, 5, 6, 0] = float("nan")
    prnu.fingerprint_accumulate(ff[:10], 2, A2, B2, state=st2)
    assert down(st2).tolist() == [20, 10, prnu.STATUS_NONFINITE]


def test_depth_one_u8_frames_read_in_place(dev):
    """At d = 1 the u8 frames are read in place (no means written); the same
    frames as float32 go through the SDA kernel: identical accumulators."""
    _log("d=1 u8 in place vs f32 frames")
    fr = _frames_for(7, 72, 104, 3, 11)
    A8, B8 = prnu.new_accumulators(3, 72, 104, device=dev)
    prnu.fingerprint_accumulate(up(fr, dev), 1, A8, B8)
    Af, Bf = prnu.new_accumulators(3, 72, 104, device=dev)
    prnu.fingerprint_accumulate(up(fr.astype(np.float32), dev), 1, Af, Bf)
    np.testing.assert_array_equal(down(A8), down(Af))
    np.testing.assert_array_equal(down(B8), down(Bf))


@pytest.mark.parametrize("mode", [prnu.ACC_F64, prnu.ACC_KAHAN_F32, prnu.ACC_F32])
def test_depth_one_u8_intensity_energy_exact(dev, mode):
    """At d = 1 on u8 frames B = sum_i I_i^2 is a sum of integers below 2^24
    (33 frames, across the 32-frame fold batch): every accumulator mode holds
    it exactly (the compensation plane stays zero)."""
    _log(f"d=1 u8 B exact mode {mode}")
    fr = _frames_for(33, 40, 72, 3, 12)
    A, B = prnu.new_accumulators(3, 40, 72, mode, device=dev)
    prnu.fingerprint_accumulate(up(fr, dev), 1, A, B, acc_mode=mode)
    ref = np.sum(fr.astype(np.int64) ** 2, axis=0).transpose(2, 0, 1).astype(np.float64)
    b = down(B).astype(np.float64)
    if mode == prnu.ACC_KAHAN_F32:
        np.testing.assert_array_equal(b[1], 0.0)
        b = b[0]
    np.testing.assert_array_equal(b, ref)


def test_depth_one_equals_per_frame_residuals(dev):
    """d = 1 is the conventional estimator: A equals sum_i W_i I_i built from
    the standalone residual call on each frame."""
    _log("d=1 vs residual entry point")
    fr = _frames_for(6, 64, 96, 1, 10)
    A, B = prnu.new_accumulators(1, 64, 96, device=dev)
    prnu.fingerprint_accumulate(up(fr, dev), 1, A, B)
    img = fr[:, :, :, 0].astype(np.float32)
    Wr = down(prnu.denoise_residual(up(img, dev))).astype(np.float64)
    Aw = np.sum(Wr * img, axis=0)
    np.testing.assert_allclose(down(A)[0], Aw, rtol=0, atol=1e-9 * np.abs(Aw).max())


# ------------------------------------------------------------------ finalize
@pytest.mark.parametrize("C,H,W,flags", [
    (1, 256, 256, prnu.ZM), (1, 256, 256, prnu.ZM | prnu.WIENER), (3, 120, 160, prnu.ZM | prnu.LUMA),
    (3, 120, 160, prnu.ZM | prnu.LUMA | prnu.WIENER), (3, 96, 128, prnu.ZM), (1, 100, 75, prnu.WIENER),
    (1, 37, 53, prnu.ZM), (3, 1080, 1920, prnu.ZM | prnu.LUMA | prnu.WIENER), (3, 45, 75, prnu.LUMA),
    (3, 45, 75, 0), (1, 45, 75, 0)])
def test_fingerprint_finalize(dev, C, H, W, flags):
    _log(f"finalize C={C} {H}x{W} flags={flags}")
    g = synth.rng(synth.CFG_TEST, 5300 + H + C)
    B = g.uniform(1e4, 6e4, size=(C, H, W))
    B[0, 0, 0] = 0.0  # zero denominator -> K = 0
    A = B * (g.normal(0, 0.01, size=(C, H, W)) + 0.002 * np.cos(np.arange(W) * 0.7)[None, None, :])
    K = down(prnu.fingerprint_finalize(up(A, dev), up(B, dev), flags=flags))
    ref = pipeline.finalize(A, B, flags)
    assert_scaled(K, ref, what="K")


def test_finalize_fixed_sigma(dev):
    g = synth.rng(synth.CFG_TEST, 5350)
    B = g.uniform(1e4, 6e4, size=(1, 120, 150))
    A = B * g.normal(0, 0.01, size=B.shape)
    K = down(prnu.fingerprint_finalize(up(A, dev), up(B, dev), flags=prnu.ZM | prnu.WIENER, sigma_wf=0.004))
    ref = pipeline.finalize(A, B, pipeline.FIN_ZM | pipeline.FIN_WIENER, sigma_wf=0.004)
    assert_scaled(K, ref, what="K fixed sigma")


# ------------------------------------------------------------------ queries
@pytest.mark.parametrize("n,H,W,C,flags", [(3, 120, 160, 3, 7), (2, 256, 256, 1, 7), (2, 72, 104, 3, 3),
                                           (1, 64, 64, 1, 0), (2, 45, 75, 3, 3), (2, 45, 75, 3, 2)])
def test_query_residual(dev, n, H, W, C, flags):
    _log(f"query n={n} {H}x{W}x{C} flags={flags}")
    fr = _frames_for(n, H, W, C, 11)
    Wq, Iq = prnu.query_residual(up(fr, dev), flags=flags)
    Wq, Iq = down(Wq), down(Iq)
    for k in range(n):
        Wr, Ir = pipeline.query_residual(fr[k], flags=flags)
        assert_scaled(Wq[k], Wr, what=f"Wq[{k}]")
        assert_scaled(Iq[k], Ir, rtol=1e-6, what=f"Iq[{k}]")


# ------------------------------------------------------------------ PCE / NCC
def _pce_ref(X, Y, mod, mode):
    out = np.zeros((len(X), len(Y)))
    ncc = np.zeros_like(out)
    peaks = np.zeros(out.shape + (2,), np.int64)
    Cs = {}
    for q in range(len(X)):
        for j in range(len(Y)):
            y = Y[j] * mod[q] if mod is not None else Y[j]
            r = correlate.pce(X[q], y, mode)
            out[q, j], ncc[q, j] = r["pce"], r["ncc"]
            peaks[q, j] = r["peak"]
            Xc, Yc = X[q] - X[q].mean(), y - y.mean()
            Cs[q, j] = correlate.xcorr_fft(Xc, Yc)
    return out, ncc, peaks, Cs


@pytest.mark.parametrize("h,w,mode,modulated", [
    (64, 80, 0, False), (64, 80, 1, True), (120, 160, 0, True), (256, 256, 1, False),
    (30, 36, 1, True), (45, 75, 0, True), (36, 50, 0, False), (1080, 1920, 0, True),
    (1080, 1920, 0, False)])
def test_pce_match(dev, h, w, mode, modulated):
    _log(f"pce {h}x{w} mode={mode} modulated={modulated}")
    g = synth.rng(synth.CFG_TEST, 5400 + h)
    nx, ny = 2, 3
    X = g.normal(0, 1, size=(nx, h, w)).astype(np.float32)
    Y = g.normal(0, 1, size=(ny, h, w)).astype(np.float32)
    Y[0] = (0.3 * X[0] + g.normal(0, 1, size=(h, w))).astype(np.float32)  # matched with query 0
    if mode == 1:
        Y[1] = np.roll(X[1], (5, 9), axis=(0, 1)) + g.normal(0, 1, size=(h, w)).astype(np.float32)
    mod = g.uniform(50, 200, size=(nx, h, w)).astype(np.float32) if modulated else None
    if modulated and mode == 1:
        mod[1] = 1.0
    pce, ncc, peak = prnu.pce_match(up(X, dev), up(Y, dev), up(mod, dev) if modulated else None, peak_mode=mode)
    rp, rn, rpk, Cs = _pce_ref(X.astype(np.float64), Y.astype(np.float64),
                               mod.astype(np.float64) if modulated else None, mode)
    pce, ncc, peak = down(pce), down(ncc), down(peak)
    np.testing.assert_allclose(ncc, rn, rtol=0, atol=1e-5)
    for q in range(nx):
        for j in range(ny):
            if tuple(peak[q, j]) != tuple(rpk[q, j]):
                # a different maximum is only acceptable if the oracle's surface
                # holds (within float32 rounding) the same maximal value there
                C = Cs[q, j]
                assert C[tuple(peak[q, j])] >= C.max() - 1e-5 * np.abs(C).max(), (q, j, peak[q, j], rpk[q, j])
                continue
            assert_pce(pce[q, j], rp[q, j], what=f"pce[{q},{j}]")
    assert pce[0, 0] > 60
    if mode == 1:
        assert tuple(peak[1, 1]) == ((-5) % h, (-9) % w)


@pytest.mark.parametrize("nx,ny,h,w,modulated", [
    (3, 16, 36, 150, True), (2, 17, 40, 64, False), (1, 33, 24, 200, True), (4, 5, 72, 96, False)])
def test_pce_fixed_many_fingerprints(dev, nx, ny, h, w, modulated):
    """Fixed-peak PCE with three or more fingerprints per query (the direct sums
    then run on the matrix cores in groups of 16, ragged tiles)."""
    _log(f"pce many fingerprints nx={nx} ny={ny} {h}x{w} modulated={modulated}")
    g = synth.rng(synth.CFG_TEST, 5700 + ny)
    X = g.normal(0, 1, size=(nx, h, w)).astype(np.float32)
    Y = g.normal(0, 1, size=(ny, h, w)).astype(np.float32)
    for q in range(nx):
        Y[(3 * q) % ny] = (0.4 * X[q] + g.normal(0, 1, size=(h, w))).astype(np.float32)
    mod = g.uniform(50, 200, size=(nx, h, w)).astype(np.float32) if modulated else None
    pce, ncc, _ = prnu.pce_match(up(X, dev), up(Y, dev), up(mod, dev) if modulated else None, peak_mode=0)
    rp, rn, _, _ = _pce_ref(X.astype(np.float64), Y.astype(np.float64),
                            mod.astype(np.float64) if modulated else None, 0)
    # without the NCC the matrix-core sums skip sum y^2 only: the PCE is bit-identical
    pce_only, _, _ = prnu.pce_match(up(X, dev), up(Y, dev), up(mod, dev) if modulated else None, peak_mode=0,
                                    want_ncc=False, want_peak=False)
    pce, ncc = down(pce), down(ncc)
    np.testing.assert_array_equal(down(pce_only), pce)
    np.testing.assert_allclose(ncc, rn, rtol=0, atol=1e-5)
    for q in range(nx):
        for j in range(ny):
            assert_pce(pce[q, j], rp[q, j], what=f"pce[{q},{j}]")
        assert pce[q, (3 * q) % ny] > 60


@pytest.mark.parametrize("h,w", [(512, 512), (720, 1280), (2160, 3840)])
def test_compiled_transform_sizes(dev, h, w):
    """Frame sizes whose row, half-row and column transforms run compile-time
    kernels (1080x1920 is covered above): fixed-peak PCE of one modulated
    query against three fingerprints, and the DFT-domain Wiener of one plane."""
    _log(f"compiled transform sizes {h}x{w}")
    g = synth.rng(synth.CFG_TEST, 5900 + h)
    X = g.normal(0, 1, size=(1, h, w)).astype(np.float32)
    Y = g.normal(0, 1, size=(3, h, w)).astype(np.float32)
    Y[1] = (0.2 * X[0] + g.normal(0, 1, size=(h, w))).astype(np.float32)
    mod = g.uniform(50, 200, size=(1, h, w)).astype(np.float32)
    pce, _, _ = prnu.pce_match(up(X, dev), up(Y, dev), up(mod, dev), peak_mode=0, want_ncc=False,
                               want_peak=False)
    pce = down(pce)
    for j in range(3):
        r = correlate.pce(X[0].astype(np.float64), Y[j].astype(np.float64) * mod[0], correlate.PEAK_FIXED_00)
        assert_pce(pce[0, j], r["pce"], what=f"pce[0,{j}] {h}x{w}")
    assert pce[0, 1] > 60
    B = g.uniform(1e4, 6e4, size=(1, h, w))
    A = B * g.normal(0, 0.01, size=(1, h, w))
    K = down(prnu.fingerprint_finalize(up(A, dev), up(B, dev), flags=prnu.ZM | prnu.WIENER))
    assert_scaled(K, pipeline.finalize(A, B, pipeline.FIN_ZM | pipeline.FIN_WIENER), what=f"K {h}x{w}")


@pytest.mark.parametrize("n,H,W,b", [(3, 37, 53, 16), (2, 1080, 1920, 500), (1, 64, 64, 64), (4, 20, 30, 1)])
def test_extract_blocks_exact(dev, n, H, W, b):
    """Block gather of the block-wise protocol: bit-exact copies, block-major."""
    _log(f"extract blocks n={n} {H}x{W} b={b}")
    g = synth.rng(synth.CFG_TEST, 6000 + H)
    x = g.normal(0, 1, size=(n, H, W)).astype(np.float32)
    got = down(prnu.extract_blocks(up(x, dev), b))
    ref = np.stack([np.stack(correlate.blocks(x[p], b)) for p in range(n)], axis=1)
    assert got.shape == ref.shape
    np.testing.assert_array_equal(got, ref)


def test_pce_blocks_vs_oracle(dev):
    """Block-wise fixed-peak PCE (block k of each query against block k of each
    fingerprint, query intensity x fingerprint) against the oracle; the pairs
    that share noise in some blocks stand out only there."""
    _log("block-wise PCE")
    g = synth.rng(synth.CFG_TEST, 6100)
    nx, ny, H, W, b = 2, 3, 600, 1100, 250
    X = g.normal(0, 1, size=(nx, H, W)).astype(np.float32)
    Y = g.normal(0, 1, size=(ny, H, W)).astype(np.float32)
    mod = g.uniform(50, 200, size=(nx, H, W)).astype(np.float32)
    for blk in (2, 5):  # query 0 and fingerprint 1 share noise in blocks 2 and 5
        r, c = divmod(blk, W // b)
        sl = (slice(r * b, (r + 1) * b), slice(c * b, (c + 1) * b))
        Y[1][sl] = (0.3 * X[0][sl] / mod[0][sl] * 100 + g.normal(0, 1, size=(b, b))).astype(np.float32)
    got = down(prnu.pce_blocks(up(X, dev), up(Y, dev), up(mod, dev), b))
    assert got.shape == ((H // b) * (W // b), nx, ny)
    for q in range(nx):
        for j in range(ny):
            ref = correlate.pce_blocks(X[q].astype(np.float64), Y[j].astype(np.float64) * mod[q], b)
            for k in range(len(ref)):
                assert_pce(got[k, q, j], ref[k], what=f"block {k} pce[{q},{j}]")
    assert got[2, 0, 1] > 60 and got[5, 0, 1] > 60
    assert abs(got[0, 0, 1]) < 60


@pytest.mark.parametrize("n,H,W,scale,oh,ow,oy,ox", [
    (2, 64, 96, 0.5, 32, 48, 0, 0), (1, 37, 53, 1.37, 60, 70, 3, 5), (3, 120, 200, 0.73, 80, 140, 2, 1),
    (1, 2200, 3900, 0.5, 1080, 1920, 37, 61), (1, 17, 19, 2.0, 40, 40, 0, 0), (2, 40, 56, 1.0, 36, 50, 6, 9)])
def test_resample_bilinear_vs_oracle(dev, n, H, W, scale, oh, ow, oy, ox):
    """Resizing and cropping of a query for mixed-media matching: downsampling,
    upsampling, crop offsets and clamped edges against the oracle."""
    _log(f"resample {n}x{H}x{W} scale {scale} -> {oh}x{ow} at ({oy},{ox})")
    g = synth.rng(synth.CFG_TEST, 6200 + H)
    x = g.normal(0, 1, size=(n, H, W)).astype(np.float32)
    got = down(prnu.resample_bilinear(up(x, dev), scale, oh, ow, oy, ox))
    for p in range(n):
        ref = resample.bilinear(x[p].astype(np.float64), scale, oh, ow, oy, ox)
        np.testing.assert_allclose(got[p], ref, rtol=0, atol=2e-6 * np.abs(ref).max())


@pytest.mark.parametrize("n_src,H,W,oh,ow", [(1, 64, 96, 50, 70), (2, 120, 200, 120, 200), (1, 1080, 1920, 960, 1800)])
def test_warp_affine_vs_oracle(dev, n_src, H, W, oh, ow):
    """The affine warp of stabilised video against the oracle: rotations by
    small and large angles, zooms, shear, translations (some leave the plane:
    clamped edges), each output plane with its own matrix; plane k samples
    source k % n_src.  Bilinear weights in float32 from double coordinates:
    2e-6 of the plane's scale."""
    _log(f"warp affine {n_src}x{H}x{W} -> {oh}x{ow}")
    g = synth.rng(synth.CFG_TEST, 6300 + H)
    x = g.normal(0, 1, size=(n_src, H, W)).astype(np.float32)
    mats = [resample.rotation(0.0, 1.0, H, W, oh, ow),
            resample.rotation(0.0175, 1.0, H, W, oh, ow, 2.5, -3.0),
            resample.rotation(-0.3, 1.07, H, W, oh, ow),
            resample.rotation(1.2, 0.8, H, W, oh, ow, -7.0, 11.0),
            [0.95, 0.12, 3.3, -0.08, 1.04, -2.1],
            resample.rotation(np.pi / 2, 1.0, H, W, oh, ow)]
    got = down(prnu.warp_affine(up(x, dev), np.array(mats), oh, ow))
    assert got.shape == (len(mats), oh, ow)
    for k, M in enumerate(mats):
        ref = resample.affine(x[k % n_src].astype(np.float64), M, oh, ow)
        np.testing.assert_allclose(got[k], ref, rtol=0, atol=2e-6 * np.abs(ref).max())


def test_pce_fixed_query_chunks(dev):
    """Enough pairs that the direct sums run in several chunks of queries."""
    _log("pce query chunks")
    g = synth.rng(synth.CFG_TEST, 5800)
    nx, ny, h, w = 300, 256, 16, 20
    X = g.normal(0, 1, size=(nx, h, w)).astype(np.float32)
    Y = g.normal(0, 1, size=(ny, h, w)).astype(np.float32)
    pce, _, _ = prnu.pce_match(up(X, dev), up(Y, dev), None, peak_mode=0, want_ncc=False, want_peak=False)
    pce = down(pce)
    # oracle via the FFT of every pair (fixed peak at (0,0), 11x11 excluded)
    Xc = X.astype(np.float64) - X.mean(axis=(1, 2), keepdims=True)
    Yc = Y.astype(np.float64) - Y.mean(axis=(1, 2), keepdims=True)
    FX, FY = np.fft.fft2(Xc), np.fft.fft2(Yc)
    sel = [q for q in range(0, nx, 7)] + [nx - 1]
    for q in sel:
        C = np.real(np.fft.ifft2(FX[q][None] * np.conj(FY)))  # [ny][h][w]
        c0 = C[:, 0, 0]
        Ct = C.copy()
        rows = [d % h for d in range(-5, 6)]
        cols = [d % w for d in range(-5, 6)]
        Ct[:, np.array(rows)[:, None], np.array(cols)[None, :]] = 0.0
        E = (Ct ** 2).sum(axis=(1, 2)) / (h * w - 121)
        ref = np.sign(c0) * c0 * c0 / E
        for j in range(ny):
            assert_pce(pce[q, j], ref[j], what=f"pce[{q},{j}]")


def test_pce_fixed_peak_offsets_and_nbhd(dev):
    """Fixed-peak path with fields far from zero mean and a 7x7 neighbourhood."""
    g = synth.rng(synth.CFG_TEST, 5600)
    h, w = 72, 96
    X = (g.normal(0, 1, size=(2, h, w)) + 50.0).astype(np.float32)
    Y = (g.normal(0, 1, size=(2, h, w)) - 20.0).astype(np.float32)
    Y[1] = (0.5 * (X[1] - 50.0) + g.normal(0, 1, size=(h, w)) + 3.0).astype(np.float32)
    mod = g.uniform(0.5, 2.0, size=(2, h, w)).astype(np.float32)
    for m in (None, mod):
        for nb in (7, 11):
            pce, ncc, _ = prnu.pce_match(up(X, dev), up(Y, dev), up(m, dev) if m is not None else None, nbhd=nb)
            pce, ncc = down(pce), down(ncc)
            for q in range(2):
                for j in range(2):
                    y = Y[j].astype(np.float64) * (m[q] if m is not None else 1.0)
                    r = correlate.pce(X[q].astype(np.float64), y, correlate.PEAK_FIXED_00, nbhd=nb)
                    assert_pce(pce[q, j], r["pce"], what=f"pce[{q},{j}] nbhd={nb}")
                    assert abs(ncc[q, j] - r["ncc"]) < 1e-5


def test_pce_nbhd_and_wrap(dev):
    """Peak near the corner: the 11x11 block wraps around both edges."""
    g = synth.rng(synth.CFG_TEST, 5500)
    h, w = 48, 60
    X = g.normal(0, 1, size=(1, h, w)).astype(np.float32)
    Y = np.roll(X, (2, -3), axis=(1, 2)).astype(np.float32)
    pce, _, peak = prnu.pce_match(up(X, dev), up(Y, dev), peak_mode=prnu.PEAK_ARGMAX, nbhd=7)
    r = correlate.pce(X[0].astype(np.float64), Y[0].astype(np.float64), correlate.PEAK_ARGMAX, nbhd=7)
    assert tuple(down(peak)[0, 0]) == r["peak"]
    assert_pce(down(pce)[0, 0], r["pce"])


# ------------------------------------------------------------------ end to end
@pytest.mark.parametrize("d", [1, 4])
def test_tiny_workload_end_to_end(dev, d):
    """Tiny workload: one camera, 256x256 gray, 8 frames, SDA depth d, query
    frames from the same and from a second camera."""
    _log(f"e2e tiny d={d}")
    fr, _ = synth.tiny_camera(0, 9, 256, 256)
    other, _ = synth.tiny_camera(1, 1, 256, 256)
    A, B = prnu.new_accumulators(1, 256, 256, device=dev)
    prnu.fingerprint_accumulate(up(fr[:8], dev), d, A, B)
    K = prnu.fingerprint_finalize(A, B)
    q = np.concatenate([fr[8:9], other])
    Wq, Iq = prnu.query_residual(up(q, dev))
    pce, _, _ = prnu.pce_match(Wq, K.unsqueeze(0), modulate=Iq)
    Kr = pipeline.camera_fingerprint(fr[:8], d)
    assert_scaled(down(K), Kr, what="K")
    ref = []
    for f in q:
        Wr, Ir = pipeline.query_residual(f)
        ref.append(correlate.pce(Wr, Ir * Kr)["pce"])
    assert_pce(down(pce)[:, 0], ref)
    assert down(pce)[0, 0] > 60 and abs(down(pce)[1, 0]) < 60


def test_video_1080p_rgb_sample(dev):
    """1080p RGB video camera (the video workload's frame shape), 40 frames at
    SDA depth 20, in the same launch configuration the benchmark uses; one
    query from the camera and one from another camera."""
    _log("e2e 1080p rgb d=20")
    fr, _ = synth.video_camera(0, 41, 1080, 1920, 3)
    other, _ = synth.video_camera(1, 1, 1080, 1920, 3)
    A, B = prnu.new_accumulators(3, 1080, 1920, device=dev)
    prnu.fingerprint_accumulate(up(fr[:40], dev), 20, A, B)
    K = prnu.fingerprint_finalize(A, B)
    q = np.concatenate([fr[40:41], other])
    Wq, Iq = prnu.query_residual(up(q, dev))
    pce, _, _ = prnu.pce_match(Wq, K.unsqueeze(0), modulate=Iq)
    Kr = pipeline.camera_fingerprint(fr[:40], 20)
    assert_scaled(down(K), Kr, what="K 1080p")
    ref = []
    for f in q:
        Wr, Ir = pipeline.query_residual(f)
        ref.append(correlate.pce(Wr, Ir * Kr)["pce"])
    assert_pce(down(pce)[:, 0], ref)
    _log(f"1080p pce gpu {down(pce)[:, 0]} oracle {ref}")


def test_stabilised_segments_aligned(dev):
    """Segment-constant stabiliser (Sec. V-E): the alignment search finds each
    segment's translation against the camera's pattern, and the aligned MLE
    fingerprint correlates with K better than the unaligned one."""
    from paper_1909_04573_amd import evaluation as ev

    _log("stabilised segments: alignment search")
    H = W = 256
    fr, K, sh = synth.stabilized_video_torch(1, 0, 80, H, W, k_std=0.02, max_shift=3, device=dev,
                                             cfg=synth.CFG_TEST, segment=10)
    seg = sh[::10]
    assert np.any(seg != 0) and np.any(np.all(seg == 0, axis=1))
    _, means = prnu.sda_average(fr, 10, want_sums=False)
    means = means[:, 0].contiguous()
    Wr = prnu.denoise_residual(means)
    Kt = torch.from_numpy(K.astype(np.float32)).to(dev)
    est, P = ev.segment_shifts(Wr, means, Kt, max_shift=3, margin=8)
    # the pattern of a frame shifted by (sy, sx) is K rolled by (sy, sx): candidate (-sy, -sx)
    np.testing.assert_array_equal(est, -seg)
    est_p, pce_p = ev.segment_shifts_plane(Wr, means, Kt, max_shift=3, margin=8)
    np.testing.assert_array_equal(est_p, -seg)
    # the same peak; the planes differ in which side carries the modulation and the mean
    assert np.all(pce_p > 0.5 * P.max(axis=1)) and np.all(pce_p < 2.0 * P.max(axis=1))
    M = 3
    assert ev.aligned_window(H, W, M) == (250, 250)
    A, B = prnu.new_accumulators(1, 250, 250, device=dev)
    ev.aligned_fingerprint(means, est, A, B, M)
    Ka = down(prnu.fingerprint_finalize(A, B, flags=0))  # pixel (0, 0) is frame pixel (M, M)
    A0, B0 = prnu.new_accumulators(1, H, W, device=dev)
    prnu.fingerprint_accumulate(fr, 10, A0, B0)
    K0 = down(prnu.fingerprint_finalize(A0, B0, flags=0))
    c, ca = slice(8, H - 8), slice(8 - M, H - 8 - M)
    corr = lambda a, s: float(np.corrcoef(a[s, s].ravel(), K[c, c].ravel())[0, 1])
    print(f"corr aligned {corr(Ka, ca):.3f} unaligned {corr(K0, c):.3f}", flush=True)
    assert corr(Ka, ca) > corr(K0, c) + 0.1


def test_stabilised_rotations_aligned(dev):
    """Stabiliser that rotates and translates each segment (Sec. II-B, V-E):
    the pose search finds every segment's angle (from the candidate grid) and
    translation against the camera's pattern, and the MLE over the frames
    warped back correlates with K better than the unaligned fingerprint."""
    from paper_1909_04573_amd import evaluation as ev

    _log("stabilised rotations: pose search")
    H = W = 256
    degs = (-2.0, -1.0, 1.0, 2.0)
    fr, K, poses = synth.stabilized_video_affine_torch(1, 0, 80, H, W, k_std=0.02, max_shift=3, angles_deg=degs,
                                                       segment=10, device=dev, cfg=synth.CFG_TEST)
    seg = poses[::10]
    assert np.any(seg[:, 0] != 0) and np.any(np.all(seg == 0, axis=1))
    _, means = prnu.sda_average(fr, 10, want_sums=False)
    means = means[:, 0].contiguous()
    Wr = prnu.denoise_residual(means)
    Kt = torch.from_numpy(K.astype(np.float32)).to(dev)
    angles = list(np.deg2rad((-2.0, -1.0, 0.0, 1.0, 2.0)))
    est, P = ev.segment_poses(Wr, means, Kt, angles, max_shift=3, margin=28)  # 200 x 200 DFT window
    # pattern at p is K(c + R(theta)(p - c) - s): the pose search reports (theta, -sy, -sx)
    np.testing.assert_allclose(est[:, 0], seg[:, 0], atol=1e-12)
    np.testing.assert_array_equal(est[:, 1:], -seg[:, 1:])
    M, h = 12, 225
    A, B = prnu.new_accumulators(1, h, h, device=dev)
    ev.aligned_fingerprint_affine(means, est, A, B, M)
    Ka = down(prnu.fingerprint_finalize(A, B, flags=0))  # pixel (0, 0) is frame pixel (M, M)
    A0, B0 = prnu.new_accumulators(1, H, W, device=dev)
    prnu.fingerprint_accumulate(fr, 10, A0, B0)
    K0 = down(prnu.fingerprint_finalize(A0, B0, flags=0))
    c, ca = slice(16, 16 + 200), slice(16 - M, 16 - M + 200)
    corr = lambda a, s: float(np.corrcoef(a[s, s].ravel(), K[c, c].ravel())[0, 1])
    print(f"corr aligned {corr(Ka, ca):.3f} unaligned {corr(K0, c):.3f}", flush=True)
    assert corr(Ka, ca) > corr(K0, c) + 0.1
