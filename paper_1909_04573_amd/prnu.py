"""Python binding of libprnu.so (ctypes; argument marshalling only).

Every function passes device pointers of torch tensors, the current HIP
stream and a workspace tensor to the C ABI declared in include/prnu.h; all
computation happens in the library's HIP kernels.  The library must have been
built (``python -m paper_1909_04573_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libprnu.so")

PRNU_OK, PRNU_E_INVAL, PRNU_E_UNSUPPORTED, PRNU_E_WORKSPACE, PRNU_E_HIP = 0, -1, -2, -3, -4
U8, BF16, F32 = 0, 1, 2
ACC_F64, ACC_KAHAN_F32, ACC_F32 = 0, 1, 2
ZM, LUMA, WIENER = 1, 2, 4
STATUS_NONFINITE = 1
PEAK_FIXED_00, PEAK_ARGMAX = 0, 1

_DT = {torch.uint8: U8, torch.bfloat16: BF16, torch.float32: F32}

# Every symbol the header declares (checked by the CPU test suite).
EXPORTS = (
    "prnu_last_error", "prnu_version", "prnu_default_denoise_params", "prnu_filter_coefficients",
    "prnu_sda_average",
    "prnu_denoise_residual_workspace_size", "prnu_denoise_residual", "prnu_denoise_residual_noalloc",
    "prnu_fingerprint_accumulate_workspace_size", "prnu_fingerprint_accumulate",
    "prnu_fingerprint_finalize_workspace_size", "prnu_fingerprint_finalize",
    "prnu_query_residual_workspace_size", "prnu_query_residual",
    "prnu_pce_match_workspace_size", "prnu_pce_match", "prnu_extract_blocks", "prnu_resample_bilinear",
    "prnu_warp_affine",
    "prnu_timing_enable", "prnu_timing_report",
    "prnu_postprocess_workspace_size", "prnu_postprocess",
    "prnu_denoise_ckpt_floats", "prnu_denoise_residual_ckpt",
    "prnu_denoise_residual_vjp_workspace_size", "prnu_denoise_residual_vjp",
    "prnu_pce_vjp_workspace_size", "prnu_pce_vjp",
    "prnu_pce_gap_f64_workspace_size", "prnu_pce_gap_f64",
    "prnu_batch_workspace_size", "prnu_batch_create", "prnu_batch_launch", "prnu_batch_info_get",
    "prnu_batch_destroy", "prnu_fingerprint_batch",
    "prnu_get_tile", "prnu_set_tile", "prnu_autotune_workspace_size", "prnu_autotune",
)
TILE_FWD, TILE_INV, TILE_MLE, TILE_SEG = 0, 1, 2, 3
BATCH_ZERO_ACC, BATCH_GRAPH = 1, 2


class PrnuError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libprnu error {code}: {msg}")
        self.code = code


class DenoiseParams(ctypes.Structure):
    _fields_ = [("sigma0", ctypes.c_float), ("levels", ctypes.c_int), ("taps", ctypes.c_int),
                ("level_weight", ctypes.c_float * 4)]


class PceParams(ctypes.Structure):
    _fields_ = [("peak_mode", ctypes.c_int), ("nbhd", ctypes.c_int)]


class Camera(ctypes.Structure):
    _fields_ = [("frames", ctypes.c_void_p), ("n_frames", ctypes.c_int), ("H", ctypes.c_int),
                ("W", ctypes.c_int), ("C", ctypes.c_int), ("group", ctypes.c_int),
                ("A", ctypes.c_void_p), ("B", ctypes.c_void_p)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int), ("launches", ctypes.c_int), ("jobs", ctypes.c_int64),
                ("sda_frames", ctypes.c_int64), ("padded_pixels", ctypes.c_int64),
                ("input_bytes", ctypes.c_int64)]


_lib = None
_P, _I, _F, _S, _L = ctypes.c_void_p, ctypes.c_int, ctypes.c_float, ctypes.c_size_t, ctypes.c_int64
_DP = ctypes.POINTER(DenoiseParams)


def lib() -> ctypes.CDLL:
    """Load libprnu.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1909_04573_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    L.prnu_last_error.restype = ctypes.c_char_p
    L.prnu_version.restype = ctypes.c_char_p
    L.prnu_default_denoise_params.argtypes = [_DP]
    L.prnu_filter_coefficients.argtypes = [_I, ctypes.POINTER(ctypes.c_double)]
    L.prnu_sda_average.argtypes = [_P, _I, _I, _I, _I, _I, _L, _I, _P, _P, _P, _P, _P]
    L.prnu_denoise_residual_workspace_size.argtypes = [_I, _I, _I, _DP, ctypes.POINTER(_S)]
    L.prnu_denoise_residual.argtypes = [_P, _I, _I, _I, _DP, _P, _P, _S, _P]
    L.prnu_denoise_residual_noalloc.argtypes = [_P, _I, _I, _I, _DP, _P, _P]
    L.prnu_fingerprint_accumulate_workspace_size.argtypes = [_I, _I, _I, _I, _I, _DP, ctypes.POINTER(_S)]
    L.prnu_fingerprint_accumulate.argtypes = [_P, _I, _I, _I, _I, _I, _L, _I, _DP, _I, _P, _P, _P, _P, _S, _P]
    L.prnu_fingerprint_finalize_workspace_size.argtypes = [_I, _I, _I, _I, ctypes.POINTER(_S)]
    L.prnu_fingerprint_finalize.argtypes = [_P, _P, _I, _I, _I, _I, _I, _F, _P, _P, _S, _P]
    L.prnu_query_residual_workspace_size.argtypes = [_I, _I, _I, _I, _DP, _I, ctypes.POINTER(_S)]
    L.prnu_query_residual.argtypes = [_P, _I, _I, _I, _I, _I, _DP, _I, _P, _P, _P, _S, _P]
    L.prnu_pce_match_workspace_size.argtypes = [_I, _I, _I, _I, _I, ctypes.POINTER(_S)]
    L.prnu_pce_match.argtypes = [_P, _I, _P, _I, _I, _I, _P, ctypes.POINTER(PceParams), _P, _P, _P, _P,
                                 _S, _P]
    L.prnu_extract_blocks.argtypes = [_P, _I, _I, _I, _I, _P, _P]
    L.prnu_resample_bilinear.argtypes = [_P, _I, _I, _I, ctypes.c_double, _I, _I, _I, _I, _P, _P]
    L.prnu_warp_affine.argtypes = [_P, _I, _I, _I, _P, _I, _I, _I, _P, _P]
    L.prnu_postprocess_workspace_size.argtypes = [_I, _I, _I, _I, _I, ctypes.POINTER(_S)]
    L.prnu_postprocess.argtypes = [_P, _I, _I, _I, _I, _I, _F, _P, _P, _S, _P]
    L.prnu_denoise_ckpt_floats.argtypes = [_I, _I, _I, ctypes.POINTER(_S)]
    L.prnu_denoise_residual_ckpt.argtypes = [_P, _I, _I, _I, _DP, _P, _P, _P, _S, _P]
    L.prnu_denoise_residual_vjp_workspace_size.argtypes = [_I, _I, _I, _DP, ctypes.POINTER(_S)]
    L.prnu_denoise_residual_vjp.argtypes = [_P, ctypes.c_int64, _P, _P, _I, _I, _I, _DP, _P, _P, _P, _S, _P]
    L.prnu_pce_vjp_workspace_size.argtypes = [_I, _I, _I, _I, ctypes.POINTER(_S)]
    L.prnu_pce_vjp.argtypes = [_P, _I, _P, _I, _I, _I, _P, _I, _P, _P, _P, _P, _P, _S, _P]
    L.prnu_pce_gap_f64_workspace_size.argtypes = [_I, _I, _I, _I, _I, _I, _I, _I, ctypes.POINTER(_S)]
    L.prnu_pce_gap_f64.argtypes = [_P, _I, _I, _P, _I, _P, _I, _I, _I, _I, _I, ctypes.POINTER(ctypes.c_double),
                                   _P, _P, _P, _S, _P]
    _CP = ctypes.POINTER(Camera)
    L.prnu_batch_workspace_size.argtypes = [_CP, _I, _DP, _S, ctypes.POINTER(_S)]
    L.prnu_batch_create.argtypes = [_CP, _I, _I, _DP, _I, _I, _S, _P, _S, _P, ctypes.POINTER(_P)]
    L.prnu_batch_launch.argtypes = [_P, _P]
    L.prnu_batch_info_get.argtypes = [_P, ctypes.POINTER(BatchInfo)]
    L.prnu_batch_destroy.argtypes = [_P]
    L.prnu_fingerprint_batch.argtypes = [_CP, _I, _I, _DP, _I, _S, _P, _S, _P]
    L.prnu_get_tile.argtypes = [_I, _I, _I, _I]
    L.prnu_set_tile.argtypes = [_I, _I, _I, _I, _I]
    L.prnu_autotune_workspace_size.argtypes = [_I, _I, _I, _DP, ctypes.POINTER(_S)]
    L.prnu_autotune.argtypes = [_I, _I, _I, _DP, _P, _S, _P, ctypes.POINTER(_I)]
    L.prnu_timing_enable.argtypes = [_I]
    L.prnu_timing_report.argtypes = [ctypes.c_char_p, _S, ctypes.POINTER(_S)]
    _lib = L
    return L


def _check(rc: int):
    if rc != PRNU_OK:
        raise PrnuError(rc, lib().prnu_last_error().decode())


def denoise_params(sigma0: float = 3.0, levels: int = 4, taps: int = 16, level_weight=(1, 1, 1, 1)):
    p = DenoiseParams()
    p.sigma0, p.levels, p.taps = float(sigma0), int(levels), int(taps)
    for i in range(4):
        p.level_weight[i] = float(level_weight[i])
    return p


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(dev):
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _cuda(t: torch.Tensor, name: str) -> torch.Tensor:
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _frames(frames: torch.Tensor, strided: bool = False):
    """(frames [n][H][W][C], dtype code, n, H, W, C[, frame stride in bytes]).
    With strided=True the frames may be a view whose frames are dense but
    spaced further apart (e.g. big[::k] or the first frames of a padded
    buffer); the stride is 0 when the frames are dense."""
    if not frames.is_cuda:
        raise ValueError("frames must be a device tensor")
    if frames.dtype not in _DT:
        raise ValueError("frames must be uint8, bfloat16 or float32")
    if frames.dim() == 3:
        frames = frames.unsqueeze(-1)
    if frames.dim() != 4:
        raise ValueError("frames must be [n][H][W] or [n][H][W][C]")
    n, H, W, C = frames.shape
    if not strided:
        _cuda(frames, "frames")
        return frames, _DT[frames.dtype], n, H, W, C
    if not frames[0].is_contiguous():
        raise ValueError("each frame must be contiguous")
    dense = H * W * C
    s0 = frames.stride(0) if n > 1 else dense
    if s0 < dense:
        raise ValueError("frames overlap")
    stride = 0 if s0 == dense else s0 * frames.element_size()
    return frames, _DT[frames.dtype], n, H, W, C, stride


def workspace(nbytes: int, device) -> torch.Tensor:
    ws = torch.empty(max(int(nbytes), 256) + 256, dtype=torch.uint8, device=device)
    off = (-ws.data_ptr()) % 256
    return ws[off:off + max(int(nbytes), 256)]


def version() -> str:
    return lib().prnu_version().decode()


def filter_coefficients(taps: int):
    """Host-side Daubechies low-pass filter used by the kernels (float64 list)."""
    buf = (ctypes.c_double * taps)()
    _check(lib().prnu_filter_coefficients(taps, buf))
    return list(buf)


def sda_average(frames: torch.Tensor, group: int, want_sums: bool = True, want_means: bool = True,
                want_counts: bool = False, status: torch.Tensor | None = None):
    """SDA frames: returns (sums int64 [g][C][H][W] or None, means f32
    [g][C][H][W] or None), plus counts int32 [g] with want_counts.  Frames
    may be spaced apart (a view with dense frames).  ``status``: optional
    int32 device word that PRNU_STATUS_NONFINITE is ORed into."""
    frames, dt, n, H, W, C, stride = _frames(frames, strided=True)
    g = (n + group - 1) // group
    dev = frames.device
    sums = torch.empty((g, C, H, W), dtype=torch.int32, device=dev) if want_sums and dt == U8 else None
    means = torch.empty((g, C, H, W), dtype=torch.float32, device=dev) if want_means else None
    counts = torch.empty(g, dtype=torch.int32, device=dev) if want_counts else None
    if status is not None:
        _cuda(status, "status")
        if status.dtype != torch.int32 or status.numel() != 1:
            raise ValueError("status must be one int32 device word")
    _check(lib().prnu_sda_average(_ptr(frames), dt, n, H, W, C, stride, int(group), _ptr(sums), _ptr(means),
                                  _ptr(counts), _ptr(status), _stream(dev)))
    if sums is not None:
        sums = sums.to(torch.int64) & 0xFFFFFFFF
    return (sums, means, counts) if want_counts else (sums, means)


def denoise_residual(img: torch.Tensor, params: DenoiseParams | None = None) -> torch.Tensor:
    """W = I - F(I) of float planes [n][H][W] (or [H][W])."""
    _cuda(img, "img")
    if img.dtype != torch.float32:
        raise ValueError("img must be float32")
    squeeze = img.dim() == 2
    x = img.unsqueeze(0) if squeeze else img
    n, H, W = x.shape
    p = params or denoise_params()
    nbytes = _S()
    _check(lib().prnu_denoise_residual_workspace_size(n, H, W, ctypes.byref(p), ctypes.byref(nbytes)))
    ws = workspace(nbytes.value, x.device)
    out = torch.empty_like(x)
    _check(lib().prnu_denoise_residual(_ptr(x), n, H, W, ctypes.byref(p), _ptr(out), _ptr(ws),
                                       ws.numel(), _stream(x.device)))
    return out[0] if squeeze else out


def denoise_residual_noalloc(img: torch.Tensor, out: torch.Tensor, params: DenoiseParams | None = None):
    """W = I - F(I) of float planes [n][H][W] into `out`, with the library's
    static per-GPU scratch (no workspace, nothing allocated by the call)."""
    _cuda(img, "img")
    _cuda(out, "out")
    if img.dtype != torch.float32 or img.dim() != 3 or out.shape != img.shape or out.dtype != torch.float32:
        raise ValueError("img and out must be float32 [n][H][W] of one shape")
    n, H, W = img.shape
    p = params or denoise_params()
    _check(lib().prnu_denoise_residual_noalloc(_ptr(img), n, H, W, ctypes.byref(p), _ptr(out), _stream(img.device)))
    return out


def new_accumulators(C: int, H: int, W: int, acc_mode: int = ACC_F64, device="cuda"):
    """Zeroed (A, B) accumulators in the layout of ``acc_mode``."""
    if acc_mode == ACC_F64:
        shape, dt = (C, H, W), torch.float64
    elif acc_mode == ACC_KAHAN_F32:
        shape, dt = (2, C, H, W), torch.float32
    else:
        shape, dt = (C, H, W), torch.float32
    return torch.zeros(shape, dtype=dt, device=device), torch.zeros(shape, dtype=dt, device=device)


def new_acc_state(device) -> torch.Tensor:
    """Zeroed prnu_acc_state as int64 [3]: frames, SDA frames, status bits
    (the low 32 bits of the third word)."""
    return torch.zeros(3, dtype=torch.int64, device=device)


def fingerprint_accumulate(frames: torch.Tensor, group: int, A: torch.Tensor, B: torch.Tensor,
                           params: DenoiseParams | None = None, acc_mode: int = ACC_F64,
                           ws: torch.Tensor | None = None, state: torch.Tensor | None = None):
    """A += sum W*I, B += sum I^2 over the SDA frames of ``frames`` (in place).
    Frames may be spaced apart (a view with dense frames).  ``state`` (from
    new_acc_state) counts the frames and SDA frames folded in and collects
    the non-finite-input flag."""
    frames, dt, n, H, W, C, stride = _frames(frames, strided=True)
    _cuda(A, "A")
    _cuda(B, "B")
    if state is not None:
        _cuda(state, "state")
        if state.dtype != torch.int64 or state.numel() != 3:
            raise ValueError("state must be int64 [3] (new_acc_state)")
    p = params or denoise_params()
    nbytes = _S()
    _check(lib().prnu_fingerprint_accumulate_workspace_size(n, H, W, C, int(group), ctypes.byref(p),
                                                            ctypes.byref(nbytes)))
    if ws is None or ws.numel() < nbytes.value:
        ws = workspace(nbytes.value, frames.device)
    _check(lib().prnu_fingerprint_accumulate(_ptr(frames), dt, n, H, W, C, stride, int(group), ctypes.byref(p),
                                             int(acc_mode), _ptr(A), _ptr(B), _ptr(state), _ptr(ws), ws.numel(),
                                             _stream(frames.device)))
    return A, B


def fingerprint_accumulate_workspace_size(n, H, W, C, group, params: DenoiseParams | None = None) -> int:
    p = params or denoise_params()
    nbytes = _S()
    _check(lib().prnu_fingerprint_accumulate_workspace_size(n, H, W, C, int(group), ctypes.byref(p),
                                                            ctypes.byref(nbytes)))
    return nbytes.value


def fingerprint_finalize(A: torch.Tensor, B: torch.Tensor, acc_mode: int = ACC_F64,
                         flags: int = ZM | LUMA | WIENER, sigma_wf: float = -1.0,
                         out: torch.Tensor | None = None) -> torch.Tensor:
    """K = A/B then zero-mean / luma / DFT Wiener per ``flags`` (into ``out`` if given)."""
    _cuda(A, "A")
    _cuda(B, "B")
    shape = A.shape[-3:]
    C, H, W = int(shape[0]), int(shape[1]), int(shape[2])
    nbytes = _S()
    _check(lib().prnu_fingerprint_finalize_workspace_size(C, H, W, int(flags), ctypes.byref(nbytes)))
    ws = workspace(nbytes.value, A.device)
    nout = 1 if (C == 3 and flags & LUMA) else C
    shape = (nout, H, W) if nout > 1 else (H, W)
    if out is not None:
        _cuda(out, "out")
        if tuple(out.shape) != shape or out.dtype != torch.float32:
            raise ValueError(f"out must be float32 {shape}")
        K = out
    else:
        K = torch.empty(shape, dtype=torch.float32, device=A.device)
    _check(lib().prnu_fingerprint_finalize(_ptr(A), _ptr(B), int(acc_mode), C, H, W, int(flags),
                                           float(sigma_wf), _ptr(K), _ptr(ws), ws.numel(), _stream(A.device)))
    return K


def query_residual(frames: torch.Tensor, params: DenoiseParams | None = None,
                   flags: int = ZM | LUMA | WIENER, want_intensity: bool = True):
    """Residuals of query frames, post-processed like fingerprints; and their luma."""
    frames, dt, n, H, W, C = _frames(frames)
    p = params or denoise_params()
    nbytes = _S()
    _check(lib().prnu_query_residual_workspace_size(n, H, W, C, ctypes.byref(p), int(flags),
                                                    ctypes.byref(nbytes)))
    ws = workspace(nbytes.value, frames.device)
    nout = 1 if (C == 3 and flags & LUMA) else C
    Wq = torch.empty((n, nout, H, W) if nout > 1 else (n, H, W), dtype=torch.float32, device=frames.device)
    Iq = torch.empty((n, H, W), dtype=torch.float32, device=frames.device) if want_intensity else None
    _check(lib().prnu_query_residual(_ptr(frames), dt, n, H, W, C, ctypes.byref(p), int(flags), _ptr(Wq),
                                     _ptr(Iq), _ptr(ws), ws.numel(), _stream(frames.device)))
    return Wq, Iq


def pce_match(X: torch.Tensor, Y: torch.Tensor, modulate: torch.Tensor | None = None,
              peak_mode: int = PEAK_FIXED_00, nbhd: int = 11, want_ncc: bool = True,
              want_peak: bool = True):
    """PCE [nx][ny] (float64), NCC and peak (row, col) of every (query, fingerprint) pair."""
    _cuda(X, "X")
    _cuda(Y, "Y")
    if X.dtype != torch.float32 or Y.dtype != torch.float32:
        raise ValueError("X and Y must be float32")
    if X.dim() == 2:
        X = X.unsqueeze(0)
    if Y.dim() == 2:
        Y = Y.unsqueeze(0)
    nx, h, w = X.shape
    ny = Y.shape[0]
    if tuple(Y.shape[1:]) != (h, w):
        raise ValueError("X and Y planes differ in size")
    if modulate is not None:
        _cuda(modulate, "modulate")
        if modulate.dim() == 2:
            modulate = modulate.unsqueeze(0)
        if tuple(modulate.shape) != (nx, h, w) or modulate.dtype != torch.float32:
            raise ValueError("modulate must be float32 [nx][h][w]")
    nbytes = _S()
    _check(lib().prnu_pce_match_workspace_size(nx, ny, h, w, int(modulate is not None), ctypes.byref(nbytes)))
    ws = workspace(nbytes.value, X.device)
    pp = PceParams(int(peak_mode), int(nbhd))
    dev = X.device
    pce = torch.empty((nx, ny), dtype=torch.float64, device=dev)
    ncc = torch.empty((nx, ny), dtype=torch.float64, device=dev) if want_ncc else None
    peak = torch.empty((nx, ny, 2), dtype=torch.int32, device=dev) if want_peak else None
    _check(lib().prnu_pce_match(_ptr(X), nx, _ptr(Y), ny, h, w, _ptr(modulate), ctypes.byref(pp), _ptr(pce),
                                _ptr(ncc), _ptr(peak), _ptr(ws), ws.numel(), _stream(dev)))
    return pce, ncc, peak


def extract_blocks(x: torch.Tensor, b: int) -> torch.Tensor:
    """Disjoint b x b blocks of planes [n][H][W] (or [H][W]), block-major
    [(H//b)*(W//b)][n][b][b]; rows and columns past the last whole block are
    not used."""
    _cuda(x, "x")
    if x.dtype != torch.float32:
        raise ValueError("x must be float32")
    if x.dim() == 2:
        x = x.unsqueeze(0)
    x = x.contiguous()
    n, H, W = (int(v) for v in x.shape)
    nb = (H // b) * (W // b) if b > 0 else 0
    out = torch.empty((max(nb, 1), n, max(b, 1), max(b, 1)), dtype=torch.float32, device=x.device)
    _check(lib().prnu_extract_blocks(_ptr(x), n, H, W, int(b), _ptr(out), _stream(x.device)))
    return out


def warp_affine(x: torch.Tensor, matrices, out_h: int, out_w: int) -> torch.Tensor:
    """Planes [n_src][H][W] (or [H][W]) warped by n affine matrices (rows of 6:
    column = m0 x + m1 y + m2, row = m3 x + m4 y + m5 of output pixel (y, x);
    a float64 tensor or array [n][6], or one matrix) into [n][out_h][out_w];
    output plane k samples source plane k % n_src."""
    _cuda(x, "x")
    if x.dtype != torch.float32:
        raise ValueError("x must be float32")
    x = (x.unsqueeze(0) if x.dim() == 2 else x).contiguous()
    m = torch.as_tensor(matrices, dtype=torch.float64).reshape(-1, 6).to(x.device).contiguous()
    n_src, H, W = (int(v) for v in x.shape)
    n = int(m.shape[0])
    out = torch.empty((n, int(out_h), int(out_w)), dtype=torch.float32, device=x.device)
    _check(lib().prnu_warp_affine(_ptr(x), n_src, H, W, _ptr(m), n, int(out_h), int(out_w), _ptr(out),
                                  _stream(x.device)))
    return out


def resample_bilinear(x: torch.Tensor, scale: float, out_h: int, out_w: int, oy: int = 0,
                      ox: int = 0) -> torch.Tensor:
    """Planes [n][H][W] (or [H][W]) resampled by `scale` (pixel centres, edges
    clamped) into [n][out_h][out_w], starting at output pixel (oy, ox)."""
    _cuda(x, "x")
    if x.dtype != torch.float32:
        raise ValueError("x must be float32")
    squeeze = x.dim() == 2
    if squeeze:
        x = x.unsqueeze(0)
    x = x.contiguous()
    n, H, W = (int(v) for v in x.shape)
    out = torch.empty((n, int(out_h), int(out_w)), dtype=torch.float32, device=x.device)
    _check(lib().prnu_resample_bilinear(_ptr(x), n, H, W, float(scale), int(oy), int(ox), int(out_h), int(out_w),
                                        _ptr(out), _stream(x.device)))
    return out[0] if squeeze else out


def pce_blocks(X: torch.Tensor, Y: torch.Tensor, modulate: torch.Tensor | None = None, b: int = 500,
               nbhd: int = 11):
    """Block-wise fixed-peak PCE: query planes X [nx][H][W] against fingerprints
    Y [ny][H][W] (optionally X's modulation [nx][H][W]), block k of a query
    against block k of each fingerprint.  Returns float64 [nblocks][nx][ny]."""
    Xb = extract_blocks(X, b)
    Yb = extract_blocks(Y, b)
    Mb = extract_blocks(modulate, b) if modulate is not None else None
    out = []
    for k in range(Xb.shape[0]):
        p, _, _ = pce_match(Xb[k], Yb[k], Mb[k] if Mb is not None else None, peak_mode=PEAK_FIXED_00, nbhd=nbhd,
                            want_ncc=False, want_peak=False)
        out.append(p)
    return torch.stack(out)


def timing_enable(on: bool = True):
    """Start (or stop) bracketing every kernel launch with HIP events."""
    _check(lib().prnu_timing_enable(1 if on else 0))


def timing_report() -> dict:
    """{kernel name: (launches, total ms, algorithmic bytes, algorithmic flops)} since timing_enable."""
    need = _S()
    _check(lib().prnu_timing_report(None, 0, ctypes.byref(need)))
    buf = ctypes.create_string_buffer(need.value + 64)
    _check(lib().prnu_timing_report(buf, len(buf), None))
    out = {}
    for line in buf.value.decode().splitlines():
        name, n, ms, b, fl = line.split("\t")
        out[name] = (int(n), float(ms), float(b), float(fl))
    return out


def postprocess(planes: torch.Tensor, C: int = 1, flags: int = ZM, sigma_wf: float = -1.0) -> torch.Tensor:
    """Zero-mean / luma / DFT-Wiener of planes [n][C][H][W] (or [n][H][W] for C = 1)."""
    _cuda(planes, "planes")
    if planes.dtype != torch.float32:
        raise ValueError("planes must be float32")
    H, W = int(planes.shape[-2]), int(planes.shape[-1])
    n = planes.numel() // (C * H * W)
    nbytes = _S()
    _check(lib().prnu_postprocess_workspace_size(n, C, H, W, int(flags), ctypes.byref(nbytes)))
    ws = workspace(nbytes.value, planes.device)
    nout = 1 if (C == 3 and flags & LUMA) else C
    out = torch.empty((n, nout, H, W) if nout > 1 else (n, H, W), dtype=torch.float32, device=planes.device)
    _check(lib().prnu_postprocess(_ptr(planes), n, C, H, W, int(flags), float(sigma_wf), _ptr(out), _ptr(ws),
                                  ws.numel(), _stream(planes.device)))
    return out


def denoise_residual_ckpt(img: torch.Tensor, params: DenoiseParams | None = None):
    """Residuals of planes [n][H][W] and the shrinkage sensitivities the adjoint needs."""
    _cuda(img, "img")
    if img.dtype != torch.float32 or img.dim() != 3:
        raise ValueError("img must be float32 [n][H][W]")
    n, H, W = img.shape
    p = params or denoise_params()
    per = _S()
    _check(lib().prnu_denoise_ckpt_floats(H, W, p.levels, ctypes.byref(per)))
    nbytes = _S()
    _check(lib().prnu_denoise_residual_workspace_size(n, H, W, ctypes.byref(p), ctypes.byref(nbytes)))
    ws = workspace(nbytes.value, img.device)
    out = torch.empty_like(img)
    ckpt = torch.empty((n, per.value), dtype=torch.float32, device=img.device)
    _check(lib().prnu_denoise_residual_ckpt(_ptr(img), n, H, W, ctypes.byref(p), _ptr(out), _ptr(ckpt), _ptr(ws),
                                            ws.numel(), _stream(img.device)))
    return out, ckpt


def denoise_residual_vjp(gW: torch.Tensor, ckpt: torch.Tensor, params: DenoiseParams | None = None,
                         mul: torch.Tensor | None = None, div: torch.Tensor | None = None,
                         dLds: torch.Tensor | None = None) -> torch.Tensor:
    """dL/ds_l (float64 [levels]) summed over n planes; gW is [n][H][W] or one
    [H][W] plane broadcast over n = ckpt.shape[0] planes, scaled by mul/div."""
    _cuda(gW, "gW")
    _cuda(ckpt, "ckpt")
    p = params or denoise_params()
    n = int(ckpt.shape[0])
    H, W = int(gW.shape[-2]), int(gW.shape[-1])
    stride = 0 if gW.dim() == 2 else H * W
    if gW.dim() == 3 and gW.shape[0] != n:
        raise ValueError("gW and ckpt disagree on the number of planes")
    nbytes = _S()
    _check(lib().prnu_denoise_residual_vjp_workspace_size(n, H, W, ctypes.byref(p), ctypes.byref(nbytes)))
    ws = workspace(nbytes.value, gW.device)
    if dLds is None:
        dLds = torch.zeros(p.levels, dtype=torch.float64, device=gW.device)
    _check(lib().prnu_denoise_residual_vjp(_ptr(gW), stride, _ptr(mul), _ptr(div), n, H, W, ctypes.byref(p),
                                           _ptr(ckpt), _ptr(dLds), _ptr(ws), ws.numel(), _stream(gW.device)))
    return dLds


def pce_gap_f64(theta, cam_frames: torch.Tensor, queries: torch.Tensor, query_cam, d: int = 8, nbhd: int = 11,
                taps: int = 16):
    """FP64 mode of the differentiated chain: (loss, dL/dtheta [5], PCE [nq][ncam])
    of the matched-minus-unmatched PCE gap, everything in double on the GPU.
    theta = (sigma0, lambda_1..4); cam_frames float32 [ncam][m][H][W];
    queries float32 [nq][H][W]; query_cam: camera of each query."""
    _cuda(cam_frames, "cam_frames")
    _cuda(queries, "queries")
    if cam_frames.dtype != torch.float32 or queries.dtype != torch.float32:
        raise ValueError("cam_frames and queries must be float32")
    if cam_frames.dim() != 4 or queries.dim() != 3 or tuple(queries.shape[1:]) != tuple(cam_frames.shape[2:]):
        raise ValueError("cam_frames [ncam][m][H][W] and queries [nq][H][W] of one frame size")
    ncam, m, H, W = (int(v) for v in cam_frames.shape)
    nq = int(queries.shape[0])
    dev = queries.device
    qc = torch.as_tensor(list(query_cam), dtype=torch.int32).to(dev)
    if qc.numel() != nq:
        raise ValueError("query_cam needs one camera per query")
    th = (ctypes.c_double * 5)(*[float(v) for v in theta])
    nbytes = _S()
    _check(lib().prnu_pce_gap_f64_workspace_size(ncam, m, nq, H, W, int(d), int(taps), int(nbhd),
                                                 ctypes.byref(nbytes)))
    ws = workspace(nbytes.value, dev)
    out = torch.zeros(6, dtype=torch.float64, device=dev)
    pce = torch.zeros((nq, ncam), dtype=torch.float64, device=dev)
    _check(lib().prnu_pce_gap_f64(_ptr(cam_frames), ncam, m, _ptr(queries), nq, _ptr(qc), H, W, int(d), int(taps),
                                  int(nbhd), th, _ptr(out), _ptr(pce), _ptr(ws), ws.numel(), _stream(dev)))
    o = out.cpu().numpy()
    return float(o[0]), o[1:6].copy(), pce.cpu().numpy()


def pce_vjp(X: torch.Tensor, Y: torch.Tensor, weights: torch.Tensor, modulate: torch.Tensor | None = None,
            nbhd: int = 11):
    """(PCE [nx][ny], dL/dX, dL/dY) for L = sum weights * PCE, fixed peak."""
    for t, name in ((X, "X"), (Y, "Y"), (weights, "weights")):
        _cuda(t, name)
    nx, h, w = X.shape
    ny = Y.shape[0]
    nbytes = _S()
    _check(lib().prnu_pce_vjp_workspace_size(nx, ny, h, w, ctypes.byref(nbytes)))
    ws = workspace(nbytes.value, X.device)
    pce = torch.empty((nx, ny), dtype=torch.float64, device=X.device)
    gX, gY = torch.empty_like(X), torch.empty_like(Y)
    _check(lib().prnu_pce_vjp(_ptr(X), nx, _ptr(Y), ny, h, w, _ptr(modulate), int(nbhd), _ptr(weights), _ptr(pce),
                              _ptr(gX), _ptr(gY), _ptr(ws), ws.numel(), _stream(X.device)))
    return pce, gX, gY


# ---------------------------------------------------------------------------
# Batched accumulation over many cameras and the tile autotuner.

def _cameras(cams):
    """cams: sequence of (frames [n][H][W] or [n][H][W][C], group, A, B); one dtype."""
    arr = (Camera * len(cams))()
    dts = set()
    dev = None
    for i, (frames, group, A, B) in enumerate(cams):
        frames, dt, n, H, W, C = _frames(frames)
        _cuda(A, "A")
        _cuda(B, "B")
        dts.add(dt)
        dev = frames.device
        arr[i] = Camera(frames.data_ptr(), n, H, W, C, int(group), A.data_ptr(), B.data_ptr())
    if len(dts) != 1:
        raise ValueError("all cameras of a batch must share one frame dtype")
    return arr, dts.pop(), dev


def batch_workspace_size(cams, params: DenoiseParams | None = None, round_bytes: int = 0) -> int:
    arr, _, _ = _cameras(cams)
    p = params or denoise_params()
    nbytes = _S()
    _check(lib().prnu_batch_workspace_size(arr, len(cams), ctypes.byref(p), int(round_bytes),
                                           ctypes.byref(nbytes)))
    return nbytes.value


class Batch:
    """A planned batch (prnu_batch_create): ``launch()`` enqueues the whole
    schedule on the current stream (one graph launch with BATCH_GRAPH)."""

    def __init__(self, cams, params: DenoiseParams | None = None, acc_mode: int = ACC_F64,
                 flags: int = BATCH_GRAPH | BATCH_ZERO_ACC, round_bytes: int = 0, ws: torch.Tensor | None = None):
        self._h = None
        arr, dt, dev = _cameras(cams)
        p = params or denoise_params()
        nbytes = _S()
        _check(lib().prnu_batch_workspace_size(arr, len(cams), ctypes.byref(p), int(round_bytes),
                                               ctypes.byref(nbytes)))
        if ws is None or ws.numel() < nbytes.value:
            ws = workspace(nbytes.value, dev)
        self.ws, self.device, self.cams = ws, dev, list(cams)  # keep the buffers alive
        h = ctypes.c_void_p()
        _check(lib().prnu_batch_create(arr, len(cams), dt, ctypes.byref(p), int(acc_mode), int(flags),
                                       int(round_bytes), _ptr(ws), ws.numel(), _stream(dev), ctypes.byref(h)))
        self._h = h

    def launch(self):
        _check(lib().prnu_batch_launch(self._h, _stream(self.device)))

    def info(self) -> dict:
        bi = BatchInfo()
        _check(lib().prnu_batch_info_get(self._h, ctypes.byref(bi)))
        return {k: getattr(bi, k) for k, _ in BatchInfo._fields_}

    def close(self):
        if self._h is not None and self._h.value:
            torch.cuda.synchronize(self.device)
            _check(lib().prnu_batch_destroy(self._h))
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fingerprint_batch(cams, params: DenoiseParams | None = None, acc_mode: int = ACC_F64, round_bytes: int = 0,
                      ws: torch.Tensor | None = None):
    """A += sum W*I, B += sum I^2 for every camera of ``cams`` (one schedule, no graph)."""
    arr, dt, dev = _cameras(cams)
    p = params or denoise_params()
    nbytes = _S()
    _check(lib().prnu_batch_workspace_size(arr, len(cams), ctypes.byref(p), int(round_bytes),
                                           ctypes.byref(nbytes)))
    if ws is None or ws.numel() < nbytes.value:
        ws = workspace(nbytes.value, dev)
    _check(lib().prnu_fingerprint_batch(arr, len(cams), dt, ctypes.byref(p), int(acc_mode), int(round_bytes),
                                        _ptr(ws), ws.numel(), _stream(dev)))


def get_tile(kind: int, taps: int, hk: int, wk: int) -> int:
    return int(lib().prnu_get_tile(int(kind), int(taps), int(hk), int(wk)))


def set_tile(kind: int, taps: int, hk: int, wk: int, tile: int):
    _check(lib().prnu_set_tile(int(kind), int(taps), int(hk), int(wk), int(tile)))


def set_tiles(H: int, W: int, tiles, taps: int = 16, levels: int = 4):
    """Applies a list in autotune's layout (forward 1..4, -, inverse 2..4, MLE,
    and from entry 12 on the forward levels' segment targets) to the level
    geometries of H x W frames; 0 entries and a missing tail are left as they
    are."""
    Hp, Wp = -(-int(H) // 16) * 16, -(-int(W) // 16) * 16
    for l in range(1, levels + 1):
        if tiles[l - 1]:
            set_tile(TILE_FWD, taps, Hp >> l, Wp >> l, tiles[l - 1])
        if len(tiles) > 12 + l - 1 and tiles[12 + l - 1]:
            set_tile(TILE_SEG, taps, Hp >> l, Wp >> l, tiles[12 + l - 1])
    for l in range(2, levels + 1):
        if tiles[4 + l - 1]:
            set_tile(TILE_INV, taps, Hp >> l, Wp >> l, tiles[4 + l - 1])
    if tiles[8]:
        set_tile(TILE_MLE, taps, Hp >> 1, Wp >> 1, tiles[8])


def autotune(H: int, W: int, C: int = 1, params: DenoiseParams | None = None, device="cuda"):
    """Times both tile sizes of every level kernel (and the forward levels'
    segment targets) for H x W x C frames and keeps the fastest; returns the
    16 choices (forward 1..4, inverse 1..4, MLE, -, -, -, segment targets of
    forward 1..4)."""
    p = params or denoise_params()
    nbytes = _S()
    _check(lib().prnu_autotune_workspace_size(int(H), int(W), int(C), ctypes.byref(p), ctypes.byref(nbytes)))
    dev = torch.device(device)
    ws = workspace(nbytes.value, dev)
    out = (ctypes.c_int * 16)()
    _check(lib().prnu_autotune(int(H), int(W), int(C), ctypes.byref(p), _ptr(ws), ws.numel(), _stream(dev), out))
    return list(out)
