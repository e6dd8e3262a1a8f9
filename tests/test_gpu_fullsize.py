"""GPU parity at the workloads' full frame sizes, against the FP64 oracle.

* 4000x3000 BF16 stills with block-quantisation noise (the precision
  workload's size): SDA depth 1 and 3 through the MLE, zero-mean and the
  DFT-domain Wiener (transform lengths 3000 and 4000, rows padded to 3008),
  then the fixed-peak PCE of a matched and an unmatched query.
* The batched path with one grey camera per resolution of the batched
  workload (1280x720, 1920x1080, 3840x2160), mixed SDA depths and a round
  budget that forces several rounds.
* The per-frame (depth 1) RGB 1080p path that reads u8 frames in place, with
  33 frames: a full accumulation batch of 32 and a ragged one.

The oracle runs on the host; each case holds its oracle work to a few
seconds to a few tens of seconds there.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import correlate, pipeline
from parity import assert_pce, assert_scaled

torch = pytest.importorskip("torch")
from paper_1909_04573_amd import prnu  # noqa: E402

pytestmark = pytest.mark.gpu

ZW = pipeline.FIN_ZM | pipeline.FIN_WIENER


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    prnu.lib()
    return torch.device("cuda:0")


def up(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def down(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


# ------------------------------------------------------------------ 4000 x 3000 BF16 stills
SH, SW = 3000, 4000


@pytest.fixture(scope="module")
def stills(dev):
    """Three fingerprint stills and a held-out still of camera 0, one still of
    camera 1, stored as BF16 on the device; the oracle reads the same
    BF16-decoded values.  The query residuals' oracle values are computed once."""
    _log("stills 4000x3000: synthesis")
    fr, _ = synth.still_camera(0, 4, SH, SW)
    other, _ = synth.still_camera(1, 1, SH, SW)
    tb = up(np.concatenate([fr, other]).astype(np.float32), dev).to(torch.bfloat16).contiguous()
    dec = tb.float().cpu().numpy().astype(np.float64)
    _log("stills 4000x3000: oracle query residuals")
    qref = [pipeline.query_residual(f, flags=ZW) for f in dec[3:5]]
    return tb, dec, qref, {}


@pytest.mark.parametrize("d,mode", [(1, prnu.ACC_F64), (3, prnu.ACC_F64), (3, prnu.ACC_KAHAN_F32)])
def test_stills_4000x3000_bf16(dev, stills, d, mode):
    tb, dec, qref, cache = stills
    _log(f"stills 4000x3000 bf16 d={d} mode={mode}")
    A, B = prnu.new_accumulators(1, SH, SW, mode, device=dev)
    prnu.fingerprint_accumulate(tb[:3], d, A, B, acc_mode=mode)
    K = prnu.fingerprint_finalize(A, B, mode, flags=prnu.ZM | prnu.WIENER)
    Wq, Iq = prnu.query_residual(tb[3:5], flags=prnu.ZM | prnu.WIENER)
    pce, _, _ = prnu.pce_match(Wq, K.unsqueeze(0), modulate=Iq)
    a, b = down(A), down(B)
    if mode == prnu.ACC_KAHAN_F32:
        a = a[0].astype(np.float64) + a[1]
        b = b[0].astype(np.float64) + b[1]
    if d not in cache:
        _log(f"stills 4000x3000: oracle fingerprint d={d}")
        Ar, Br = pipeline.fingerprint_accumulate(dec[:3], d)
        Kr = pipeline.finalize(Ar, Br, ZW)
        ref = [correlate.pce(Wr, Ir * Kr)["pce"] for Wr, Ir in qref]
        cache[d] = (Ar, Br, Kr, ref)
    Ar, Br, Kr, ref = cache[d]
    assert_scaled(a, Ar, what="A")
    assert_scaled(b, Br, rtol=1e-7, what="B")
    assert_scaled(K.cpu().numpy(), Kr, what="K")
    wq = down(Wq)
    for k, (Wr, Ir) in enumerate(qref):
        assert_scaled(wq[k], Wr, what=f"Wq[{k}]")
        assert_scaled(down(Iq)[k], Ir, rtol=1e-6, what=f"Iq[{k}]")
    _log(f"  pce gpu {down(pce)[:, 0]} oracle {ref}")
    assert_pce(down(pce)[:, 0], ref)


# ------------------------------------------------------------------ batched, one camera per resolution
BATCH_CAMS = [(5, 720, 1280, 1, 2), (4, 1080, 1920, 1, 1), (6, 2160, 3840, 1, 4)]


def test_batched_resolutions_several_rounds(dev):
    """720p (3 SDA frames, the last of one frame), 1080p at depth 1 and 2160p
    (a group of 4 and a short one of 2) under a 64 MiB round budget: the
    2160p jobs alone exceed it, so the schedule runs four rounds, some
    holding jobs of two cameras."""
    _log("batched 720p/1080p/2160p: synthesis")
    frames = [synth.video_camera(60 + k, n, H, W, C, cfg=synth.CFG_TEST)[0]
              for k, (n, H, W, C, _) in enumerate(BATCH_CAMS)]
    cams = []
    for fr, (n, H, W, C, d) in zip(frames, BATCH_CAMS):
        A, B = prnu.new_accumulators(C, H, W, device=dev)
        cams.append((up(fr, dev), d, A, B))
    _log("batched 720p/1080p/2160p: graph launch")
    b = prnu.Batch(cams, flags=prnu.BATCH_GRAPH | prnu.BATCH_ZERO_ACC, round_bytes=64 << 20)
    b.launch()
    info = b.info()
    b.close()
    torch.cuda.synchronize()
    assert info["rounds"] >= 3, info
    assert info["sda_frames"] == sum(-(-n // d) for n, *_, d in BATCH_CAMS)
    for k, (fr, (n, H, W, C, d), (_, _, A, B)) in enumerate(zip(frames, BATCH_CAMS, cams)):
        _log(f"batched: oracle camera {k} ({H}x{W}, {n} frames, d={d})")
        Ar, Br = pipeline.fingerprint_accumulate(fr, d)
        assert_scaled(down(A), Ar, what=f"A cam{k}")
        assert_scaled(down(B), Br, rtol=1e-7, what=f"B cam{k}")


# ------------------------------------------------------------------ RGB 1080p, depth 1, frames read in place
def test_rgb_1080p_depth_one_33_frames(dev):
    """The conventional (depth 1) estimator on 33 RGB 1080p u8 frames, which
    are read in place: identical accumulators to the same frames given as
    float32 (those go through the SDA kernel), and the G channel's sums
    against the oracle (33 plane denoises on the host)."""
    _log("rgb 1080p d=1 x33: synthesis")
    fr, _ = synth.video_camera(70, 33, 1080, 1920, 3, cfg=synth.CFG_TEST)
    A8, B8 = prnu.new_accumulators(3, 1080, 1920, device=dev)
    prnu.fingerprint_accumulate(up(fr, dev), 1, A8, B8)
    Af, Bf = prnu.new_accumulators(3, 1080, 1920, device=dev)
    prnu.fingerprint_accumulate(up(fr.astype(np.float32), dev), 1, Af, Bf)
    a8, b8 = down(A8), down(B8)
    np.testing.assert_array_equal(a8, down(Af))
    np.testing.assert_array_equal(b8, down(Bf))
    _log("rgb 1080p d=1 x33: oracle, channel 1")
    Ar, Br = pipeline.fingerprint_accumulate(fr[:, :, :, 1:2], 1)
    assert_scaled(a8[1], Ar[0], what="A[G]")
    np.testing.assert_array_equal(b8[1], Br[0])  # integer-valued squares: exact in FP64
