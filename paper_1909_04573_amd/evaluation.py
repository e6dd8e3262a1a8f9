"""Decision statistics of the attribution protocol (Sec. IV): a pair is
declared "same camera" when its PCE exceeds a threshold (60).  Host-side
summaries of PCE values the library computed; no method arithmetic.

* tpr(matched, thr): fraction of same-camera PCEs above thr;
* fpr(unmatched, thr): fraction of different-camera PCEs above thr;
* roc(matched, unmatched): (FPR, TPR) at every distinct threshold, from
  (0, 0) to (1, 1);
* auc(matched, unmatched): area under that curve, equal to the probability
  that a same-camera PCE exceeds a different-camera one (ties count 1/2).

Fingerprint equivalence and the variance model (Sec. III-B, Sec. IV-B):

* equal_variance_images(n, s1_sq, s2_sq, d): the image count m whose SDA-d
  fingerprint has the error variance of a conventional one of n images;
* variance_components(W, prnu_term): the noise (s1^2) and scene (s2^2)
  variances of the residual model from R residuals of one scene;
* equivalent_images(conv, sda): per conventional image count, the fewest
  images an SDA fingerprint needs to reach at least its TPR.

Stabilised video (Sec. V-E), orchestration of library calls:

* segment_shifts(W, I, K_ref): per SDA frame, the translation of a reference
  fingerprint with the largest fixed-peak PCE;
* aligned_fingerprint(means, shifts, A, B): MLE over the SDA frames
  translated back by their shifts;
* segment_poses(W, I, K_ref, angles): the same search over rotations about
  the frame centre (one warped reference per angle, the translation from the
  argmax of one correlation plane per angle);
* aligned_fingerprint_affine(means, poses, A, B): MLE over the SDA frames
  rotated and translated back by their poses.
"""
from __future__ import annotations

import numpy as np

THRESHOLD = 60.0


def tpr(matched, thr: float = THRESHOLD) -> float:
    m = np.asarray(matched, dtype=np.float64).ravel()
    return float(np.mean(m > thr)) if m.size else float("nan")


def fpr(unmatched, thr: float = THRESHOLD) -> float:
    u = np.asarray(unmatched, dtype=np.float64).ravel()
    return float(np.mean(u > thr)) if u.size else float("nan")


def roc(matched, unmatched):
    """(fpr, tpr) arrays at thresholds just below every distinct value, in
    increasing FPR; the first point is (0, 0) and the last (1, 1)."""
    m = np.asarray(matched, dtype=np.float64).ravel()
    u = np.asarray(unmatched, dtype=np.float64).ravel()
    thr = np.unique(np.concatenate([m, u]))[::-1]  # descending
    ms, us = np.sort(m), np.sort(u)
    # counts of values >= t for each threshold t
    tp = m.size - np.searchsorted(ms, thr, side="left")
    fp = u.size - np.searchsorted(us, thr, side="left")
    f = np.concatenate([[0.0], fp / max(u.size, 1)])
    t = np.concatenate([[0.0], tp / max(m.size, 1)])
    return f, t


def auc(matched, unmatched) -> float:
    """P(matched > unmatched) + P(equal) / 2 over all pairs (rank statistic)."""
    m = np.asarray(matched, dtype=np.float64).ravel()
    u = np.asarray(unmatched, dtype=np.float64).ravel()
    if not m.size or not u.size:
        return float("nan")
    us = np.sort(u)
    below = np.searchsorted(us, m, side="left")
    equal = np.searchsorted(us, m, side="right") - below
    return float((below.sum() + 0.5 * equal.sum()) / (m.size * u.size))


# ---------------------------------------------------------------- equivalence and variance model
def equal_variance_images(n: float, s1_sq: float, s2_sq: float, d: int) -> float:
    """Sec. III-B: with the residual of a frame modelled as I K + psi + xi,
    psi the noise term (variance s1^2, averaged down by d in an SDA frame)
    and xi the scene term (variance s2^2, not averaged), n conventional
    images and m = n (s1^2 + d s2^2) / (s1^2 + s2^2) images in SDA-d frames
    give fingerprints of equal error variance.  s2^2 = 0 gives m = n."""
    if s1_sq < 0 or s2_sq < 0 or s1_sq + s2_sq <= 0 or d < 1:
        raise ValueError("variances must be >= 0, not both 0, and d >= 1")
    return float(n) * (s1_sq + d * s2_sq) / (s1_sq + s2_sq)


def variance_components(W, prnu_term):
    """(s1^2, s2^2) of the residual model from R >= 2 residuals W[r] of one
    scene that share the scene and the PRNU term and differ only in their
    noise: s1^2 is the unbiased variance across the R residuals, averaged
    over pixels; the mean residual minus the PRNU term then holds the scene
    term plus the noise averaged over R, so s2^2 = mean((mean_r W - prnu)^2)
    - s1^2 / R, clipped at 0."""
    W = np.asarray(W, dtype=np.float64)
    P = np.asarray(prnu_term, dtype=np.float64)
    R = W.shape[0]
    if R < 2 or W.shape[1:] != P.shape:
        raise ValueError("need R >= 2 residuals of the PRNU term's shape")
    mean = W.mean(axis=0)
    s1 = float(((W - mean) ** 2).sum(axis=0).mean() / (R - 1))
    s2 = max(float(((mean - P) ** 2).mean()) - s1 / R, 0.0)
    return s1, s2


def equivalent_images(conv: dict, sda: dict) -> dict:
    """{n: m}: for each conventional image count n (TPR conv[n]) the smallest
    m among sda's image counts whose TPR sda[m] is at least conv[n]; None if
    none reaches it (Sec. IV-B, Fig. 5: the fingerprint-equivalence search)."""
    ms = sorted(sda)
    return {n: next((m for m in ms if sda[m] >= t), None) for n, t in sorted(conv.items())}


# ---------------------------------------------------------------- stabilised video (Sec. V-E)
def smooth_floor(n: int) -> int:
    """Largest m <= n with no prime factor above 5 (a size the DFT Wiener
    step of the fingerprint post-processing accepts)."""
    for m in range(int(n), 0, -1):
        r = m
        for q in (2, 3, 5):
            while r % q == 0:
                r //= q
        if r == 1:
            return m
    raise ValueError("n must be >= 1")


def aligned_window(H: int, W: int, M: int):
    """Size (h, w) of aligned fingerprints of H x W frames whose shifts are
    within M: the largest 5-smooth sizes inside [M, H - M) x [M, W - M)."""
    return smooth_floor(H - 2 * M), smooth_floor(W - 2 * M)


def segment_shifts(W, I, K_ref, max_shift: int = 8, margin: int = 60, origin: int = 0,
                   pce_min: float | None = None):
    """Per-segment alignment search for stabilised video (Sec. V-E): the
    sensor pattern of SDA frame j (residual W[j], intensity I[j], planes
    [g][H][W] float32 on the GPU) is compared with every integer translation
    (dy, dx), |dy|, |dx| <= max_shift, of the reference fingerprint K_ref,
    whose pixel (0, 0) sits at frame pixel (origin, origin):
    candidate(y, x) = K_ref(y - origin + dy, x - origin + dx), cut out by
    prnu_resample_bilinear at scale 1, and the fixed-peak PCE of W[j] against
    I[j] * candidate picks the translation.  A `margin` is left out of the
    correlations (the denoiser's boundary pattern) and must cover the search:
    margin >= origin + max_shift.  With pce_min, a frame whose best PCE stays
    below it keeps the zero shift: a frame of another camera would otherwise
    take the translation that best matches the reference's noise, and those
    choices add up in the aligned fingerprint's PCE against the reference
    (pce_min = 25 is a 5-sigma peak; the chance that one of (2 max_shift +
    1)^2 noise candidates reaches it is about 1e-4 per frame at max_shift 8).
    Every step runs in the library (the cut-outs and one pce_match call); the
    argmax is on the host.  Returns
    (shifts int [g][2], pce float64 [g][(2 max_shift + 1)^2]) with candidate
    k = (dy, dx) = divmod(k, 2 max_shift + 1) - max_shift."""
    import torch

    from . import prnu

    g, H, Wd = (int(v) for v in W.shape)
    n = 2 * max_shift + 1
    h, w = H - 2 * margin, Wd - 2 * margin
    o = margin - origin
    if o - max_shift < 0 or o + max_shift + h > K_ref.shape[-2] or o + max_shift + w > K_ref.shape[-1]:
        raise ValueError("the search window leaves the reference fingerprint")
    cands = torch.empty((n * n, h, w), dtype=torch.float32, device=W.device)
    for k in range(n * n):
        dy, dx = k // n - max_shift, k % n - max_shift
        cands[k] = prnu.resample_bilinear(K_ref, 1.0, h, w, o + dy, o + dx)
    Wc = W[:, margin:H - margin, margin:Wd - margin].contiguous()
    Ic = I[:, margin:H - margin, margin:Wd - margin].contiguous()
    P, _, _ = prnu.pce_match(Wc, cands, Ic, peak_mode=prnu.PEAK_FIXED_00, want_ncc=False, want_peak=False)
    P = P.cpu().numpy()
    best = np.argmax(P, axis=1)
    shifts = np.stack([best // n - max_shift, best % n - max_shift], axis=1).astype(np.int64)
    if pce_min is not None:
        shifts[P[np.arange(g), best] < pce_min] = 0
    return shifts, P


def signed_lag(i: int, n: int) -> int:
    """Lag of index i of a circular correlation of length n, in
    (-n/2, n/2]: i for i <= n // 2, else i - n."""
    return i - n if i > n // 2 else i


def segment_shifts_plane(W, I, K_ref, max_shift: int = 8, margin: int = 60, origin: int = 0,
                         pce_min: float | None = None):
    """The search of segment_shifts from one correlation plane per SDA frame.
    With the reference cut to the frame's window as the query and the frame's
    intensity as the modulation of its residual, the plane is
    C(s) = sum_t K_ref(t + s) I[j](t) W[j](t) (circular over the window),
    which is the candidate sum of segment_shifts at (dy, dx) = s, so one
    pce_match call with the argmax peak per frame replaces the
    (2 max_shift + 1)^2 candidates.  The peak is the largest C over the whole
    plane; a frame keeps the zero shift where that peak lies outside
    |dy|, |dx| <= max_shift or (with pce_min) its PCE stays below pce_min.
    The window wraps at its edges (max_shift of its rows and columns).
    Returns (shifts int [g][2], pce float64 [g] at the peak)."""
    from . import prnu

    g, H, Wd = (int(v) for v in W.shape)
    h, w = H - 2 * margin, Wd - 2 * margin
    o = margin - origin
    if o < 0 or o + h > K_ref.shape[-2] or o + w > K_ref.shape[-1]:
        raise ValueError("the search window leaves the reference fingerprint")
    Kc = K_ref[None, o:o + h, o:o + w].contiguous()
    Wc = W[:, margin:H - margin, margin:Wd - margin].contiguous()
    Ic = I[:, margin:H - margin, margin:Wd - margin].contiguous()
    shifts = np.zeros((g, 2), dtype=np.int64)
    pce = np.zeros(g)
    for j in range(g):
        P, _, pk = prnu.pce_match(Kc, Wc[j:j + 1], Ic[j:j + 1], peak_mode=prnu.PEAK_ARGMAX, want_ncc=False)
        r, c = (int(v) for v in pk.cpu()[0, 0])
        dy, dx = signed_lag(r, h), signed_lag(c, w)
        pce[j] = float(P.cpu()[0, 0])
        if max(abs(dy), abs(dx)) <= max_shift and (pce_min is None or pce[j] >= pce_min):
            shifts[j] = (dy, dx)
    return shifts, pce


def aligned_fingerprint(means, shifts, A, B, M: int, params=None, ws=None):
    """MLE over SDA frames after alignment: SDA frame j (means [g][H][W]
    float32) is translated back by its segment's shift (dy, dx), |dy|, |dx|
    <= M, and cut to a window of h x w frame pixels starting at (M, M):
    aligned(y, x) = mean(y + M - dy, x + M - dx), so its sensor pattern lines
    up with the reference pose; the windows are accumulated as frames of
    depth 1 into A, B of [1][h][w] (updated in place; h <= H - 2M,
    w <= W - 2M, normally aligned_window(H, W, M))."""
    import torch

    from . import prnu

    g, H, Wd = (int(v) for v in means.shape)
    if np.abs(np.asarray(shifts)).max(initial=0) > M:
        raise ValueError("a shift exceeds the window margin M")
    h, w = (int(v) for v in A.shape[-2:])
    if h > H - 2 * M or w > Wd - 2 * M:
        raise ValueError("the accumulators exceed the window inside the margin M")
    al = torch.empty((g, h, w, 1), dtype=torch.float32, device=means.device)
    for j in range(g):
        dy, dx = int(shifts[j, 0]), int(shifts[j, 1])
        al[j, :, :, 0] = prnu.resample_bilinear(means[j], 1.0, h, w, M - dy, M - dx)
    prnu.fingerprint_accumulate(al, 1, A, B, params, ws=ws)
    return A, B


# ---------------------------------------------------------------- rotations (stabilised video, Sec. II-B / V-E)
def reference_pose_matrix(theta: float, H: int, W: int, margin: int, origin: int = 0):
    """Affine matrix (prnu_warp_affine layout) of the reference cut-out for
    rotation theta: window pixel q of an H x W frame (frame pixel q + margin)
    samples the reference fingerprint at c + R(theta) (q + margin - c) - origin,
    c the frame centre; R rotates (column, row) coordinates."""
    ca, sa = np.cos(theta), np.sin(theta)
    cx, cy = (W - 1) / 2.0, (H - 1) / 2.0
    return [ca, -sa, ca * (margin - cx) - sa * (margin - cy) + cx - origin,
            sa, ca, sa * (margin - cx) + ca * (margin - cy) + cy - origin]


def alignment_matrix(theta: float, dy: float, dx: float, H: int, W: int, M: int):
    """Affine matrix that brings an H x W frame of pose (theta, dy, dx) (its
    pattern at frame pixel p is the reference at c + R(theta) (p - c) + d) to
    the reference pose: window pixel q samples the frame at
    c + R(-theta) (q + M - d - c).  theta = 0 is the translation of
    aligned_fingerprint."""
    ca, sa = np.cos(theta), np.sin(theta)
    cx, cy = (W - 1) / 2.0, (H - 1) / 2.0
    ax, ay = M - dx - cx, M - dy - cy
    return [ca, sa, cx + ca * ax + sa * ay, -sa, ca, cy - sa * ax + ca * ay]


def segment_poses(W, I, K_ref, angles, max_shift: int = 8, margin: int = 60, origin: int = 0,
                  pce_min: float | None = None):
    """Per-segment pose search for stabilised video whose stabiliser also
    rotates frames (Sec. II-B): for every candidate angle the reference
    fingerprint is warped onto the frames' window (reference_pose_matrix,
    one prnu_warp_affine call for all angles), and each SDA frame j runs one
    pce_match call with the argmax peak against all of them: the plane of
    angle a is C_a(s) = sum_t ref_a(t + s) I[j](t) W[j](t), whose peak gives
    the translation for that angle (as in segment_shifts_plane).  The frame
    takes the angle with the largest PCE; it keeps the zero pose where that
    peak lies outside |dy|, |dx| <= max_shift or (with pce_min) its PCE stays
    below pce_min.  The margin must cover the rotated window inside the
    reference, and the window (H - 2 margin) x (W - 2 margin) must be a size
    the PCE's DFT takes (prime factors up to 5).  Returns (poses float64 [g][3] = (theta, dy, dx),
    pce float64 [g][len(angles)] at each angle's peak)."""
    import torch

    from . import prnu

    g, H, Wd = (int(v) for v in W.shape)
    h, w = H - 2 * margin, Wd - 2 * margin
    mats = np.array([reference_pose_matrix(a, H, Wd, margin, origin) for a in angles])
    refs = prnu.warp_affine(K_ref, mats, h, w)
    Wc = W[:, margin:H - margin, margin:Wd - margin].contiguous()
    Ic = I[:, margin:H - margin, margin:Wd - margin].contiguous()
    na = len(angles)
    poses = np.zeros((g, 3))
    pce = np.zeros((g, na))
    for j in range(g):
        mod = Ic[j:j + 1].expand(na, h, w).contiguous()
        P, _, pk = prnu.pce_match(refs, Wc[j:j + 1], mod, peak_mode=prnu.PEAK_ARGMAX, want_ncc=False)
        P, pk = P.cpu().numpy()[:, 0], pk.cpu().numpy()[:, 0]
        pce[j] = P
        a = int(np.argmax(P))
        dy, dx = signed_lag(int(pk[a, 0]), h), signed_lag(int(pk[a, 1]), w)
        if max(abs(dy), abs(dx)) <= max_shift and (pce_min is None or P[a] >= pce_min):
            poses[j] = (angles[a], dy, dx)
    return poses, pce


def aligned_fingerprint_affine(means, poses, A, B, M: int, params=None, ws=None):
    """MLE over SDA frames brought to the reference pose: frame j (means
    [g][H][W] float32) is warped by alignment_matrix(pose j) onto the window
    of h x w frame pixels from (M, M) (prnu_warp_affine, one call for all
    frames) and the windows are accumulated as frames of depth 1 into A, B of
    [1][h][w]."""
    from . import prnu

    g, H, Wd = (int(v) for v in means.shape)
    h, w = (int(v) for v in A.shape[-2:])
    if h > H - 2 * M or w > Wd - 2 * M:
        raise ValueError("the accumulators exceed the window inside the margin M")
    mats = np.array([alignment_matrix(float(t), float(dy), float(dx), H, Wd, M) for t, dy, dx in poses])
    al = prnu.warp_affine(means.contiguous(), mats, h, w)
    prnu.fingerprint_accumulate(al.unsqueeze(-1).contiguous(), 1, A, B, params, ws=ws)
    return A, B
