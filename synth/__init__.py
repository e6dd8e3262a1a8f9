"""Seeded synthetic camera data for the SDA fingerprint path.

Frames follow the sensor output model of Sec. II-A, Eq. (1): the recorded
image is the clean scene plus the scene modulated by the multiplicative PRNU
factor K plus additive noise, then rounded (half to even) and clipped to the
8-bit range.  Nothing here denoises, averages or correlates: this module only
makes inputs.  It is shared by the tests, the benchmark and the CPU oracle's
callers, and it contains none of the fingerprint method's arithmetic.

Streams: every draw comes from ``numpy.random.Generator(Philox)`` keyed by a
master seed and a tuple of integers (config, camera, frame, ...), so any
frame of any synthetic camera can be regenerated on its own.

The device variant (``video_frames_torch``) draws its noise with torch's
generator on the GPU; it follows the same recipe but not the same random
stream, and callers that need an oracle result on it read its frames back.
"""
from __future__ import annotations

import numpy as np

MASTER_SEED = 190904573

# Config ids used as the first stream key.
CFG_TINY, CFG_VIDEO, CFG_BATCH, CFG_DIFF, CFG_STILL, CFG_EVAL, CFG_TEST = 0, 1, 2, 3, 4, 5, 99


def rng(*keys: int) -> np.random.Generator:
    """Independent generator for the stream named by ``keys``."""
    ss = np.random.SeedSequence([MASTER_SEED, *[int(k) & 0xFFFFFFFF for k in keys]])
    return np.random.Generator(np.random.Philox(ss))


def gaussian_blur(x: np.ndarray, sigma: float) -> np.ndarray:
    """Gaussian low-pass of a 2-D field (reflect boundary, 4-sigma support)."""
    from scipy.ndimage import gaussian_filter

    return gaussian_filter(x, sigma=sigma, mode="reflect", truncate=4.0)


def camera_prnu(shape, std: float, *keys: int) -> np.ndarray:
    """PRNU factor K ~ N(0, std^2), one value per sensor element (and channel)."""
    return rng(*keys).normal(0.0, std, size=shape)


def flat_scene(H: int, W: int, g: np.random.Generator, sigma: float = 8.0) -> np.ndarray:
    """Uniform[40,220] field blurred with sigma px: a nearly flat scene (std ~2 DN)."""
    return gaussian_blur(g.uniform(40.0, 220.0, size=(H, W)), sigma)


def stretch(x: np.ndarray, lo: float = 40.0, hi: float = 220.0) -> np.ndarray:
    """Affine re-stretch of a field to [lo, hi]."""
    mn, mx = float(x.min()), float(x.max())
    if mx <= mn:
        return np.full_like(x, 0.5 * (lo + hi))
    return lo + (hi - lo) * (x - mn) / (mx - mn)


def textured_scene(H: int, W: int, g: np.random.Generator, sigma: float = 8.0) -> np.ndarray:
    """Blurred uniform field re-stretched to [40,220]: a textured scene."""
    return stretch(flat_scene(H, W, g, sigma))


def quantize_u8(x: np.ndarray) -> np.ndarray:
    """Round half to even, clip to [0,255], store as uint8."""
    return np.clip(np.rint(x), 0, 255).astype(np.uint8)


def sensor_frame(I0: np.ndarray, K: np.ndarray, noise_std: float, g: np.random.Generator,
                 quantize: bool = True) -> np.ndarray:
    """I = I0 + I0*K + psi with psi ~ N(0, noise_std^2) (Sec. II-A, Eq. (1))."""
    I = I0 * (1.0 + K) + g.normal(0.0, noise_std, size=I0.shape)
    return quantize_u8(I) if quantize else I


def tiny_camera(cam: int, n_frames: int, H: int = 256, W: int = 256, k_std: float = 0.02,
                noise_std: float = 2.0, textured: bool = False, cfg: int = CFG_TINY,
                first_frame: int = 0):
    """Grayscale camera of the tiny workload.

    Returns (frames uint8 [n][H][W][1], K float64 [H][W]).  Each frame has a new
    scene: Uniform[40,220] blurred with sigma = 8 px (flat), or the same field
    re-stretched to [40,220] (textured variant).
    """
    K = camera_prnu((H, W), k_std, cfg, cam, 0xC0FFEE)
    out = np.empty((n_frames, H, W, 1), np.uint8)
    for i in range(n_frames):
        g = rng(cfg, cam, 1 + first_frame + i)
        I0 = textured_scene(H, W, g) if textured else flat_scene(H, W, g)
        out[i, :, :, 0] = sensor_frame(I0, K, noise_std, g)
    return out, K


def video_texture(H: int, W: int, C: int, *keys: int) -> np.ndarray:
    """Per-camera base texture, twice the frame size, per channel: U[0,1] blurred
    with sigma = 2 px and stretched to [40,220].  Shape [2H][2W][C]."""
    g = rng(*keys)
    tex = np.empty((2 * H, 2 * W, C))
    for c in range(C):
        tex[:, :, c] = stretch(gaussian_blur(g.uniform(0.0, 1.0, size=(2 * H, 2 * W)), 2.0))
    return tex


def crop_walk(n: int, H: int, W: int, g: np.random.Generator, step: float = 3.0):
    """Random-walk integer crop offsets inside a [2H][2W] texture."""
    y, x = H // 2, W // 2
    offs = np.empty((n, 2), np.int64)
    for i in range(n):
        y = int(np.clip(round(y + g.normal(0.0, step)), 0, H))
        x = int(np.clip(round(x + g.normal(0.0, step)), 0, W))
        offs[i] = (y, x)
    return offs


def video_camera(cam: int, n_frames: int, H: int, W: int, C: int = 3, k_std: float = 0.01,
                 noise_std: float = 2.0, cfg: int = CFG_VIDEO, first_frame: int = 0):
    """Video-shaped camera: frames are random-walk crops of a per-camera texture
    with a per-frame brightness jitter U[0.7,1.3], PRNU and N(0, 2^2) noise.

    Returns (frames uint8 [n][H][W][C], K float64 [H][W][C]).
    """
    K = camera_prnu((H, W, C), k_std, cfg, cam, 0xC0FFEE)
    tex = video_texture(H, W, C, cfg, cam, 0x7E7)
    offs = crop_walk(first_frame + n_frames, H, W, rng(cfg, cam, 0x3A1C))[first_frame:]
    out = np.empty((n_frames, H, W, C), np.uint8)
    for i in range(n_frames):
        g = rng(cfg, cam, 1 + first_frame + i)
        b = g.uniform(0.7, 1.3)
        y, x = offs[i]
        I0 = b * tex[y:y + H, x:x + W, :]
        out[i] = sensor_frame(I0, K, noise_std, g)
    return out, K


def video_frames_torch(cam: int, n_frames: int, H: int, W: int, C: int = 3, k_std: float = 0.01,
                       noise_std: float = 2.0, device="cuda", cfg: int = CFG_VIDEO, out=None,
                       first_frame: int = 0):
    """Same recipe as :func:`video_camera`, drawn on the device for large volumes.

    Texture, K, offsets and brightness come from the numpy streams above; the
    per-pixel noise is drawn with a seeded torch generator on ``device``.
    Returns a uint8 tensor [n][H][W][C] on ``device`` (written into ``out`` if
    given) and K as float64 numpy.
    """
    import torch

    K = camera_prnu((H, W, C), k_std, cfg, cam, 0xC0FFEE)
    tex = torch.from_numpy(video_texture(H, W, C, cfg, cam, 0x7E7)).to(device=device, dtype=torch.float32)
    offs = crop_walk(first_frame + n_frames, H, W, rng(cfg, cam, 0x3A1C))[first_frame:]
    bright = rng(cfg, cam, 0xB16).uniform(0.7, 1.3, size=first_frame + n_frames)[first_frame:]
    Kt = torch.from_numpy(K).to(device=device, dtype=torch.float32)
    gen = torch.Generator(device=device)
    gen.manual_seed((MASTER_SEED * 1000003 + cfg * 7919 + cam * 104729 + first_frame) % (2**63))
    if out is None:
        out = torch.empty((n_frames, H, W, C), dtype=torch.uint8, device=device)
    noise = torch.empty((H, W, C), dtype=torch.float32, device=device)
    for i in range(n_frames):
        y, x = int(offs[i, 0]), int(offs[i, 1])
        I0 = tex[y:y + H, x:x + W, :] * float(bright[i])
        noise.normal_(0.0, noise_std, generator=gen)
        I = I0 * (1.0 + Kt) + noise
        out[i] = torch.round(I).clamp_(0, 255).to(torch.uint8)
    return out, K


def random_field(shape, *keys: int, std: float = 1.0) -> np.ndarray:
    """White Gaussian field (for correlation tests)."""
    return rng(*keys).normal(0.0, std, size=shape)


# ---------------------------------------------------------------- stills with block-DCT quantisation
def dct8_matrix() -> np.ndarray:
    """Orthonormal 8-point DCT-II matrix D (rows = frequencies)."""
    D = np.zeros((8, 8))
    for u in range(8):
        a = np.sqrt(1.0 / 8.0) if u == 0 else np.sqrt(2.0 / 8.0)
        for x in range(8):
            D[u, x] = a * np.cos((2 * x + 1) * u * np.pi / 16.0)
    return D


def quant_table() -> np.ndarray:
    """Synthetic quantisation steps q(u, v) = 2 + u + v (not JPEG's table)."""
    u = np.arange(8)
    return 2.0 + u[:, None] + u[None, :]


def block_quantise(I: np.ndarray) -> np.ndarray:
    """8x8 block DCT-II, rounding of every coefficient to a multiple of
    q(u, v), inverse DCT, clip to [0, 255] (H and W multiples of 8)."""
    H, W = I.shape
    D, Q = dct8_matrix(), quant_table()
    B = I.reshape(H // 8, 8, W // 8, 8).transpose(0, 2, 1, 3)
    C = D @ B @ D.T
    C = np.rint(C / Q) * Q
    R = (D.T @ C @ D).transpose(0, 2, 1, 3).reshape(H, W)
    return np.clip(R, 0.0, 255.0)


def still_camera(cam: int, n: int, H: int, W: int, k_std: float = 0.005, noise_std: float = 2.0,
                 cfg: int = CFG_STILL, first_frame: int = 0):
    """Grayscale stills: a new blurred texture per still (U[0,1] blurred with
    sigma 2 px, stretched to [40,220]), PRNU, N(0, 2^2) noise, 8x8 block
    quantisation noise.  Returns (float64 frames [n][H][W][1] before storage
    rounding, K)."""
    K = camera_prnu((H, W), k_std, cfg, cam, 0xC0FFEE)
    out = np.empty((n, H, W, 1))
    for i in range(n):
        g = rng(cfg, cam, 1 + first_frame + i)
        I0 = stretch(gaussian_blur(g.uniform(0.0, 1.0, size=(H, W)), 2.0))
        out[i, :, :, 0] = block_quantise(sensor_frame(I0, K, noise_std, g, quantize=False))
    return out, K


def still_frames_torch(cam: int, n: int, H: int, W: int, k_std: float = 0.005, noise_std: float = 2.0,
                       device="cuda", cfg: int = CFG_STILL, first_frame: int = 0):
    """Device version of :func:`still_camera` (same recipe, torch's RNG for the
    per-pixel draws).  Returns float32 frames [n][H][W][1] before storage
    rounding, and K (float64 numpy)."""
    import torch

    K = camera_prnu((H, W), k_std, cfg, cam, 0xC0FFEE)
    Kt = torch.from_numpy(K).to(device=device, dtype=torch.float32)
    gen = torch.Generator(device=device)
    gen.manual_seed((MASTER_SEED * 7 + cfg * 7919 + cam * 104729 + first_frame) % (2**63))
    D = torch.from_numpy(dct8_matrix()).to(device=device, dtype=torch.float32)
    DT = torch.from_numpy(np.ascontiguousarray(dct8_matrix().T)).to(device=device, dtype=torch.float32)
    Q = torch.from_numpy(quant_table()).to(device=device, dtype=torch.float32)
    r = 8
    x = torch.arange(-r, r + 1, device=device, dtype=torch.float32)
    kern = torch.exp(-0.5 * (x / 2.0) ** 2)
    kern = kern / kern.sum()
    out = torch.empty((n, H, W, 1), dtype=torch.float32, device=device)
    for i in range(n):
        u = torch.rand((1, 1, H, W), generator=gen, device=device)
        u = torch.nn.functional.pad(u, (r, r, r, r), mode="reflect")
        u = torch.nn.functional.conv2d(u, kern.view(1, 1, 1, -1))
        u = torch.nn.functional.conv2d(u, kern.view(1, 1, -1, 1))[0, 0]
        I0 = 40.0 + 180.0 * (u - u.min()) / (u.max() - u.min())
        I = I0 * (1.0 + Kt) + noise_std * torch.randn((H, W), generator=gen, device=device)
        B = I.reshape(H // 8, 8, W // 8, 8).permute(0, 2, 1, 3)
        B = B.contiguous()
        C = torch.round(torch.matmul(torch.matmul(D, B), DT) / Q) * Q
        R = torch.matmul(torch.matmul(DT, C.contiguous()), D)
        out[i, :, :, 0] = R.permute(0, 2, 1, 3).reshape(H, W).clamp_(0.0, 255.0)
    return out, K


def patch_camera(cam: int, n: int, H: int = 512, W: int = 512, k_std: float = 0.015, kappa: float = 0.03,
                 cfg: int = CFG_DIFF, first_frame: int = 0):
    """Float patches for the differentiable workload: random-walk crops of a
    per-camera texture (as for video), PRNU K ~ N(0, k_std^2) and signal-
    dependent noise of variance kappa * I0 (about 2 DN at I0 = 130).
    Returns (float64 patches [n][H][W], K)."""
    K = camera_prnu((H, W), k_std, cfg, cam, 0xC0FFEE)
    tex = video_texture(H, W, 1, cfg, cam, 0x7E7)[:, :, 0]
    offs = crop_walk(first_frame + n, H, W, rng(cfg, cam, 0x3A1C), step=16.0)[first_frame:]
    out = np.empty((n, H, W))
    for i in range(n):
        g = rng(cfg, cam, 1 + first_frame + i)
        y, x = offs[i]
        I0 = tex[y:y + H, x:x + W]
        out[i] = I0 * (1.0 + K) + g.normal(0.0, 1.0, size=I0.shape) * np.sqrt(kappa * I0)
    return out, K


def _eval_scene(gen, H: int, W: int, kind: str, device):
    """One scene of the attribution generator: 'flat' = a 9 x 16 grid of
    U[100, 160] values, bicubic-upsampled; 'textured' = U[0,1] blurred with
    sigma 2 px, stretched to [40, 220]."""
    import torch

    if kind == "flat":
        grid = 100.0 + 60.0 * torch.rand((1, 1, 9, 16), generator=gen, device=device)
        return torch.nn.functional.interpolate(grid, size=(H, W), mode="bicubic", align_corners=False)[0, 0]
    r = 8
    x = torch.arange(-r, r + 1, device=device, dtype=torch.float32)
    kern = torch.exp(-0.5 * (x / 2.0) ** 2)
    kern = kern / kern.sum()
    u = torch.rand((1, 1, H, W), generator=gen, device=device)
    u = torch.nn.functional.pad(u, (r, r, r, r), mode="reflect")
    u = torch.nn.functional.conv2d(u, kern.view(1, 1, 1, -1))
    u = torch.nn.functional.conv2d(u, kern.view(1, 1, -1, 1))[0, 0]
    return 40.0 + 180.0 * (u - u.min()) / (u.max() - u.min())


def _eval_generator(cam: int, cfg: int, first_frame: int, kind: str, device):
    import torch

    gen = torch.Generator(device=device)
    gen.manual_seed((MASTER_SEED * 11 + cfg * 7919 + cam * 104729 + first_frame * 31 +
                     (0 if kind == "flat" else 17)) % (2**63))
    return gen


def eval_frames_torch(cam: int, n: int, H: int, W: int, kind: str = "flat", k_std: float = 0.0008,
                      noise_std: float = 2.0, device="cuda", cfg: int = CFG_EVAL, first_frame: int = 0):
    """Gray images for the attribution protocol (flat vs textured scenes, a
    new scene per image), drawn on the device: PRNU K ~ N(0, k_std^2) per
    camera, N(0, noise_std^2) noise, rint, clip.  Returns (uint8 [n][H][W][1]
    on device, K float64 [H][W])."""
    import torch

    K = camera_prnu((H, W), k_std, cfg, cam, 0xC0FFEE)
    Kt = torch.from_numpy(K).to(device=device, dtype=torch.float32)
    gen = _eval_generator(cam, cfg, first_frame, kind, device)
    out = torch.empty((n, H, W, 1), dtype=torch.uint8, device=device)
    for i in range(n):
        I0 = _eval_scene(gen, H, W, kind, device)
        I = I0 * (1.0 + Kt) + noise_std * torch.randn((H, W), generator=gen, device=device)
        out[i, :, :, 0] = torch.round(I).clamp_(0, 255).to(torch.uint8)
    return out, K


def eval_scene_realizations(cam: int, R: int, H: int, W: int, kind: str = "textured", k_std: float = 0.0008,
                            noise_std: float = 2.0, device="cuda", cfg: int = CFG_EVAL):
    """R images of ONE scene of the attribution generator (same I0 and K,
    independent noise), to separate the residual's noise term from its scene
    term.  Returns (uint8 [R][H][W] on device, I0 float32 [H][W] on device,
    K float64 [H][W])."""
    import torch

    K = camera_prnu((H, W), k_std, cfg, cam, 0xC0FFEE)
    Kt = torch.from_numpy(K).to(device=device, dtype=torch.float32)
    gen = _eval_generator(cam, cfg, 1 << 20, kind, device)
    I0 = _eval_scene(gen, H, W, kind, device)
    out = torch.empty((R, H, W), dtype=torch.uint8, device=device)
    for i in range(R):
        I = I0 * (1.0 + Kt) + noise_std * torch.randn((H, W), generator=gen, device=device)
        out[i] = torch.round(I).clamp_(0, 255).to(torch.uint8)
    return out, I0, K


def mixed_media_camera_torch(cam: int, n_video: int, n_still: int, Hs: int = 2250, Ws: int = 4000,
                             oy: int = 0, ox: int = 0, Hv: int = 1080, Wv: int = 1920, k_std: float = 0.001,
                             noise_std: float = 2.0, video_noise: float = 1.0, device="cuda",
                             cfg: int = CFG_EVAL):
    """A camera that records full-resolution stills and half-resolution video.

    The sensor has PRNU K ~ N(0, k_std^2) at Hs x Ws.  A still is a textured
    scene at sensor resolution (as in eval_frames_torch) times (1 + K) plus
    N(0, noise_std^2), rounded.  A video frame is a sensor frame (same model)
    reduced 2 x 2 (the in-camera downscale by 0.5, pixel centres), cropped at
    (oy, ox) to Hv x Wv, plus N(0, video_noise^2), rounded.  Returns (video
    uint8 [n_video][Hv][Wv][1], stills uint8 [n_still][Hs][Ws][1], K float64
    [Hs][Ws]) with the frames on `device`."""
    import torch

    K = camera_prnu((Hs, Ws), k_std, cfg, cam, 0x5E45)
    Kt = torch.from_numpy(K).to(device=device, dtype=torch.float32)
    gen = _eval_generator(cam, cfg, 1 << 21, "textured", device)
    video = torch.empty((n_video, Hv, Wv, 1), dtype=torch.uint8, device=device)
    stills = torch.empty((n_still, Hs, Ws, 1), dtype=torch.uint8, device=device)
    for i in range(n_video):
        S = _eval_scene(gen, Hs, Ws, "textured", device) * (1.0 + Kt)
        S = S + noise_std * torch.randn((Hs, Ws), generator=gen, device=device)
        half = S[: Hs // 2 * 2, : Ws // 2 * 2].reshape(Hs // 2, 2, Ws // 2, 2).mean(dim=(1, 3))
        v = half[oy:oy + Hv, ox:ox + Wv] + video_noise * torch.randn((Hv, Wv), generator=gen, device=device)
        video[i, :, :, 0] = torch.round(v).clamp_(0, 255).to(torch.uint8)
    for i in range(n_still):
        S = _eval_scene(gen, Hs, Ws, "textured", device) * (1.0 + Kt)
        S = S + noise_std * torch.randn((Hs, Ws), generator=gen, device=device)
        stills[i, :, :, 0] = torch.round(S).clamp_(0, 255).to(torch.uint8)
    return video, stills, K


def stabilized_video_affine_torch(cam: int, vid: int, n: int, H: int = 1080, W: int = 1920,
                                  k_std: float = 0.0004, p_still: float = 0.3, max_shift: int = 8,
                                  angles_deg=(-1.0, -0.5, 0.5, 1.0), segment: int = 30, noise_std: float = 2.0,
                                  device="cuda", cfg: int = CFG_EVAL, K=None):
    """A stabilised gray video whose stabiliser holds one pose per run of
    `segment` frames: with probability p_still none, otherwise a rotation
    about the frame centre by an angle drawn from `angles_deg` and an integer
    translation uniform in [-max_shift, max_shift]^2 (Sec. II-B: stabilisers
    shift, rotate and zoom frames).  A frame with pose (theta, sy, sx) sees
    the sensor pattern at frame pixel p as K(c + R(theta) (p - c) - s), c the
    frame centre, sampled bilinearly (torch grid_sample, edges clamped); the
    scene is the video generator's random-walk crop of a per-video texture.
    I = I0 (1 + pattern) + N(0, noise_std^2), rounded.  K defaults to the
    camera's PRNU of the stabilised workload.  Returns (uint8 [n][H][W][1]
    on device, K float64 [H][W], poses float64 [n][3] = (theta in radians,
    sy, sx))."""
    import torch
    import torch.nn.functional as F

    if K is None:
        K = camera_prnu((H, W), k_std, cfg, cam, 0x57AB)
    Kt = torch.from_numpy(np.asarray(K)).to(device=device, dtype=torch.float32)[None, None]
    g = rng(cfg, cam, 0x57AB, vid)
    tex = torch.from_numpy(stretch(gaussian_blur(g.uniform(0.0, 1.0, size=(2 * H, 2 * W)), 2.0))).to(
        device=device, dtype=torch.float32)
    offs = crop_walk(n, H, W, g)
    bright = g.uniform(0.7, 1.3, size=n)
    gs = rng(cfg, cam, 0x57AB, vid, 0xAFF)
    nseg = (n + segment - 1) // segment
    still = gs.uniform(size=nseg) < p_still
    th = np.deg2rad(np.asarray(angles_deg, dtype=np.float64))[gs.integers(0, len(angles_deg), size=nseg)]
    sh = gs.integers(-max_shift, max_shift + 1, size=(nseg, 2)).astype(np.float64)
    th[still] = 0.0
    sh[still] = 0.0
    poses = np.repeat(np.concatenate([th[:, None], sh], axis=1), segment, axis=0)[:n]
    gen = torch.Generator(device=device)
    gen.manual_seed((MASTER_SEED * 19 + cfg * 7919 + cam * 104729 + vid * 131) % (2**63))
    yy, xx = torch.meshgrid(torch.arange(H, dtype=torch.float64, device=device),
                            torch.arange(W, dtype=torch.float64, device=device), indexing="ij")
    cy, cx = (H - 1) / 2.0, (W - 1) / 2.0
    out = torch.empty((n, H, W, 1), dtype=torch.uint8, device=device)
    pat = None
    for i in range(n):
        if i % segment == 0:
            t, sy, sx = (float(v) for v in poses[i])
            u = cx + np.cos(t) * (xx - cx) - np.sin(t) * (yy - cy) - sx
            v = cy + np.sin(t) * (xx - cx) + np.cos(t) * (yy - cy) - sy
            u = u.clamp(0, W - 1) / (W - 1) * 2 - 1  # grid_sample's [-1, 1] with corner alignment
            v = v.clamp(0, H - 1) / (H - 1) * 2 - 1
            grid = torch.stack([u, v], dim=-1)[None].to(torch.float32)
            pat = F.grid_sample(Kt, grid, mode="bilinear", padding_mode="border", align_corners=True)[0, 0]
        y, x = int(offs[i, 0]), int(offs[i, 1])
        I = tex[y:y + H, x:x + W] * float(bright[i]) * (1.0 + pat)
        I = I + noise_std * torch.randn((H, W), generator=gen, device=device)
        out[i, :, :, 0] = torch.round(I).clamp_(0, 255).to(torch.uint8)
    return out, K, poses


def stabilized_video_torch(cam: int, vid: int, n: int, H: int = 1080, W: int = 1920, k_std: float = 0.0004,
                           p_still: float = 0.3, max_shift: int = 8, noise_std: float = 2.0, device="cuda",
                           cfg: int = CFG_EVAL, segment: int = 0):
    """A digitally stabilised gray video: the scene is a random-walk crop of a
    per-video texture (as in the video generator); each frame's sensor
    pattern reaches the output translated by the stabiliser, by (0, 0) with
    probability p_still and otherwise by an integer shift uniform in
    [-max_shift, max_shift]^2 (a translation-only stand-in for the in-camera
    warps).  With segment > 0 the translation is drawn once per run of
    `segment` frames (a stabiliser whose correction holds over a segment),
    from a stream of its own, so the per-frame draws are unchanged.
    I = I0 (1 + K shifted) + N(0, noise_std^2), rounded; the pattern of a
    frame with shift (sy, sx) is K rolled by (sy, sx).  Returns (uint8
    [n][H][W][1] on device, K float64 [H][W], shifts int [n][2])."""
    import torch

    K = camera_prnu((H, W), k_std, cfg, cam, 0x57AB)
    Kt = torch.from_numpy(K).to(device=device, dtype=torch.float32)
    g = rng(cfg, cam, 0x57AB, vid)
    tex = torch.from_numpy(stretch(gaussian_blur(g.uniform(0.0, 1.0, size=(2 * H, 2 * W)), 2.0))).to(
        device=device, dtype=torch.float32)
    offs = crop_walk(n, H, W, g)
    bright = g.uniform(0.7, 1.3, size=n)
    still = g.uniform(size=n) < p_still
    shifts = g.integers(-max_shift, max_shift + 1, size=(n, 2))
    shifts[still] = 0
    if segment > 0:
        gs = rng(cfg, cam, 0x57AB, vid, 0x5E6)
        nseg = (n + segment - 1) // segment
        sstill = gs.uniform(size=nseg) < p_still
        ss = gs.integers(-max_shift, max_shift + 1, size=(nseg, 2))
        ss[sstill] = 0
        shifts = np.repeat(ss, segment, axis=0)[:n]
    gen = torch.Generator(device=device)
    gen.manual_seed((MASTER_SEED * 17 + cfg * 7919 + cam * 104729 + vid * 131) % (2**63))
    out = torch.empty((n, H, W, 1), dtype=torch.uint8, device=device)
    for i in range(n):
        y, x = int(offs[i, 0]), int(offs[i, 1])
        Ks = torch.roll(Kt, shifts=(int(shifts[i, 0]), int(shifts[i, 1])), dims=(0, 1))
        I = tex[y:y + H, x:x + W] * float(bright[i]) * (1.0 + Ks)
        I = I + noise_std * torch.randn((H, W), generator=gen, device=device)
        out[i, :, :, 0] = torch.round(I).clamp_(0, 255).to(torch.uint8)
    return out, K, shifts
