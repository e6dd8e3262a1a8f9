"""The no-allocation residual call (static per-GPU scratch) against the
workspace call and the oracle: two calls in a row, the second on a smaller
input, and a batch that needs several passes through the scratch."""
import ctypes
import sys

import numpy as np
import pytest

import synth
from oracle import pipeline
from parity import assert_scaled

torch = pytest.importorskip("torch")
from paper_1909_04573_amd import prnu  # noqa: E402

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    prnu.lib()
    return torch.device("cuda:0")


def _planes(seed, n, H, W, dev):
    fr, _ = synth.tiny_camera(seed, n, H, W)
    return torch.from_numpy(fr[..., 0].astype(np.float32)).to(dev)


def _noalloc(x, p=None):
    """Through the C ABI: only the input, the output and the stream."""
    out = torch.full_like(x, float("nan"))
    pp = p or prnu.denoise_params()
    rc = prnu.lib().prnu_denoise_residual_noalloc(ctypes.c_void_p(x.data_ptr()), x.shape[0], x.shape[1],
                                                   x.shape[2], ctypes.byref(pp), ctypes.c_void_p(out.data_ptr()),
                                                   ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == prnu.PRNU_OK, prnu.lib().prnu_last_error().decode()
    return out


def test_noalloc_matches_workspace_call_twice(dev):
    big = _planes(11, 3, 1080, 1920, dev)    # six 1080p pyramids fit: one pass
    small = _planes(12, 2, 200, 328, dev)    # smaller, after the big call filled the scratch
    for k, x in enumerate((big, small)):
        _log(f"noalloc call {k}: {tuple(x.shape)}")
        got = _noalloc(x)
        ref = prnu.denoise_residual(x)
        torch.cuda.synchronize()
        assert torch.isfinite(got).all()
        assert torch.equal(got, ref), f"call {k}: differs from the workspace call"
        g = got.cpu().numpy()
        assert_scaled(g[0], pipeline.denoise_residual(x[0].cpu().numpy().astype(np.float64)), what=f"call {k} W[0]")


def test_noalloc_several_passes_and_params(dev):
    """Seven 1080p planes (more than one pass through the scratch) with 8
    taps, 3 levels and level weights."""
    x = _planes(13, 7, 1080, 1920, dev)
    p = prnu.denoise_params(taps=8, levels=3, level_weight=(0.5, 1.5, 2.0, 1.0))
    _log("noalloc: 7 x 1080p, 8 taps, 3 levels")
    got = _noalloc(x, p)
    ref = prnu.denoise_residual(x, p)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    assert_scaled(got[6].cpu().numpy(), pipeline.denoise_residual(x[6].cpu().numpy().astype(np.float64), taps=8,
                                                                  levels=3, level_weight=(0.5, 1.5, 2.0, 1.0)),
                  what="W[6]")
