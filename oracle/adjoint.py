"""FP64 adjoint of the differentiable fingerprint chain (test infrastructure only).

The chain, for denoiser parameters theta = (sigma0, lambda_1..lambda_4):

  per camera j:  SDA frames I_ji (Sec. III-B) -> residuals W_ji = I - F(I)
                 -> K_j = sum_i W_ji I_ji / sum_i I_ji^2 (Sec. III-B MLE)
                 -> zero-mean
  per query q:   residual W_q -> zero-mean -> x_q
  per pair:      PCE(x_q, I_q * K_j) with the peak at (0,0)
  loss:          mean PCE over matched pairs - mean PCE over unmatched pairs

theta enters only through the shrinkage.  With s_l = lambda_l sigma0^2 and,
per detail coefficient c, the smallest window mean m of c^2 (independent of
theta), the residual coefficient is r = c s_l / max(s_l, m): r = c when
m <= s_l and r = c s_l / m otherwise, so dr/ds_l = [m > s_l] c / m.  The
residual is a linear synthesis of the r's (crop of the periodised inverse
DWT), whose adjoint is the periodised DWT of the zero-embedded gradient, so

  dL/ds_l = sum over level-l detail coefficients of g_r [m > s_l] c / m,

with g_r the detail coefficients of the DWT of dL/dW.  dL/dsigma0 =
sum_l dL/ds_l 2 lambda_l sigma0 and dL/dlambda_l = dL/ds_l sigma0^2.
"""
from __future__ import annotations

import numpy as np

from . import correlate, dwt, pipeline, sda, wiener


def _min_window_mean(c):
    """m = smallest centred-window mean of c^2 over the 3/5/7/9 windows."""
    m = None
    for w in wiener.WINDOWS:
        mw = wiener.box_sum(c * c, w) / (w * w)
        m = mw if m is None else np.minimum(m, mw)
    return m


def residual_with_sensitivity(img, sigma0=3.0, level_weight=(1, 1, 1, 1), taps=16, levels=4,
                              want_masks=False):
    """W = I - F(I) and, per level, the factors [m > s] c / m of its three
    detail bands (the checkpoint the adjoint needs); optionally the [m > s]
    masks themselves."""
    img = np.asarray(img, dtype=np.float64)
    H, W = img.shape
    x = pipeline.pad_symmetric(img, 16)
    ll, det = dwt.wavedec2(x, taps, levels)
    rdet, sens, masks = [], [], []
    for lvl, d in enumerate(det):
        s2 = float(level_weight[lvl]) * sigma0 * sigma0
        rb, sb, mb = {}, {}, {}
        for k, c in d.items():
            m = _min_window_mean(c)
            act = m > s2
            rb[k] = np.where(act, c * s2 / np.where(act, m, 1.0), c)
            sb[k] = np.where(act, c / np.where(act, m, 1.0), 0.0)
            mb[k] = act
        rdet.append(rb)
        sens.append(sb)
        masks.append(mb)
    out = dwt.waverec2(np.zeros_like(ll), rdet, taps)
    (t, _), (l, _) = pipeline.pad_amounts(H, 16), pipeline.pad_amounts(W, 16)
    if want_masks:
        return out[t:t + H, l:l + W], sens, masks
    return out[t:t + H, l:l + W], sens


def residual_vjp_ds(gW, sens, taps=16, want_abs=False):
    """dL/ds_l (one value per level) from dL/dW of one plane and its checkpoint;
    with want_abs also the sums of the terms' magnitudes (the scale of the
    rounding error of any finite-precision evaluation of the same sums)."""
    gW = np.asarray(gW, dtype=np.float64)
    H, W = gW.shape
    (t, b), (l, r) = pipeline.pad_amounts(H, 16), pipeline.pad_amounts(W, 16)
    gp = np.zeros((H + t + b, W + l + r))
    gp[t:t + H, l:l + W] = gW  # adjoint of the crop
    _, gdet = dwt.wavedec2(gp, taps, len(sens))  # adjoint of the synthesis
    ds = np.array([sum(float(np.sum(gdet[lvl][k] * sens[lvl][k])) for k in sens[lvl])
                   for lvl in range(len(sens))])
    if not want_abs:
        return ds
    mag = np.array([sum(float(np.sum(np.abs(gdet[lvl][k] * sens[lvl][k]))) for k in sens[lvl])
                    for lvl in range(len(sens))])
    return ds, mag


def kink_margin(img, sigma0=3.0, level_weight=(1, 1, 1, 1), taps=16, levels=4):
    """Smallest |m - s_l| / s_l over every detail coefficient of the plane."""
    x = pipeline.pad_symmetric(np.asarray(img, dtype=np.float64), 16)
    _, det = dwt.wavedec2(x, taps, levels)
    out = np.inf
    for lvl, d in enumerate(det):
        s2 = float(level_weight[lvl]) * sigma0 * sigma0
        for c in d.values():
            out = min(out, float(np.min(np.abs(_min_window_mean(c) - s2))) / s2)
    return out


def pce_vjp(x, y, nbhd=11):
    """Fixed-peak PCE of (x, y) and its gradients with respect to x and y."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    h, w = x.shape
    N = h * w
    xc, yc = x - x.mean(), y - y.mean()
    C = correlate.xcorr_fft(xc, yc)
    r = nbhd // 2
    Ct = C.copy()
    rows = [dy % h for dy in range(-r, r + 1)]
    cols = [dx % w for dx in range(-r, r + 1)]
    Ct[np.ix_(rows, cols)] = 0.0
    denom = N - nbhd * nbhd
    E = float(np.sum(Ct * Ct)) / denom
    c0 = float(C[0, 0])
    val = np.sign(c0) * c0 * c0 / E
    # dPCE/dC(s)
    gC = (-np.sign(c0) * c0 * c0 / (E * E)) * 2.0 * Ct / denom
    gC[0, 0] += 2.0 * abs(c0) / E
    # C(s) = sum_t xc(t+s) yc(t):  dC/dyc(t) = xc(t+s),  dC/dxc(u) = yc(u-s)
    gy = np.real(np.fft.ifft2(np.conj(np.fft.fft2(gC)) * np.fft.fft2(xc)))
    gx = np.real(np.fft.ifft2(np.fft.fft2(gC) * np.fft.fft2(yc)))
    return float(val), gx - gx.mean(), gy - gy.mean()


def gap_loss(theta, cam_frames, queries, query_cam, d=8, taps=16, nbhd=11, want_grad=True, want_mag=False):
    """Matched-minus-unmatched mean PCE and its gradient w.r.t. theta.

    cam_frames: list over cameras of [m][H][W] float arrays (fingerprint
    patches); queries: [nq][H][W]; query_cam[q] is the camera of query q.
    Fingerprints use SDA depth d and zero-mean; queries use zero-mean; the
    matched statistic modulates the fingerprint by the query intensity.
    With want_mag a fourth value holds, per gradient component, the sum of
    the magnitudes of the per-coefficient terms it adds up (the scale of the
    rounding error of any finite-precision evaluation of the same sums).
    """
    theta = np.asarray(theta, dtype=np.float64)
    sigma0, lam = float(theta[0]), tuple(float(v) for v in theta[1:5])
    kw = dict(sigma0=sigma0, level_weight=lam, taps=taps)
    fp = []
    for fr in cam_frames:
        means = sda.sda_means(np.asarray(fr)[..., None], d)[:, 0]
        Ws, sens = zip(*[residual_with_sensitivity(I, **kw) for I in means])
        A, B = pipeline.mle_accumulate(Ws, means)
        Kz = pipeline.zero_mean(pipeline.mle_ratio(A, B))
        fp.append((means, B, Kz, sens))
    qs = []
    for Iq in queries:
        Wq, sq = residual_with_sensitivity(Iq, **kw)
        qs.append((np.asarray(Iq, dtype=np.float64), pipeline.zero_mean(Wq), sq))
    nq, nc = len(qs), len(fp)
    matched = np.array([[query_cam[q] == j for j in range(nc)] for q in range(nq)])
    wgt = np.where(matched, 1.0 / matched.sum(), -1.0 / (~matched).sum())
    P = np.zeros((nq, nc))
    gK = [np.zeros_like(f[2]) for f in fp]
    gx = [np.zeros_like(q[1]) for q in qs]
    for q, (Iq, xq, _) in enumerate(qs):
        for j, (_, _, Kz, _) in enumerate(fp):
            val, g_x, g_y = pce_vjp(xq, Iq * Kz, nbhd)
            P[q, j] = val
            gx[q] += wgt[q, j] * g_x
            gK[j] += wgt[q, j] * Iq * g_y
    L = float(np.sum(wgt * P))
    if not want_grad:
        return L, None, P
    dLds, mag = np.zeros(4), np.zeros(4)
    for j, (means, B, _, sens) in enumerate(fp):
        gKraw = pipeline.zero_mean(gK[j])  # zero-mean is self-adjoint
        for i, I in enumerate(means):
            gWi = np.where(B > 0, gKraw * I / np.where(B > 0, B, 1.0), 0.0)
            v, a = residual_vjp_ds(gWi, sens[i], taps, want_abs=True)
            dLds[:len(sens[i])] += v
            mag[:len(sens[i])] += a
    for q, (_, _, sq) in enumerate(qs):
        v, a = residual_vjp_ds(pipeline.zero_mean(gx[q]), sq, taps, want_abs=True)
        dLds[:len(sq)] += v
        mag[:len(sq)] += a
    grad = np.zeros(5)
    grad[0] = float(np.sum(dLds * 2.0 * np.array(lam) * sigma0))
    grad[1:5] = dLds * sigma0 * sigma0
    if not want_mag:
        return L, grad, P
    gmag = np.zeros(5)
    gmag[0] = float(np.sum(mag * 2.0 * np.abs(np.array(lam)) * abs(sigma0)))
    gmag[1:5] = mag * sigma0 * sigma0
    return L, grad, P, gmag


def kink_masks(theta, cam_frames, queries, d=8, taps=16):
    """The [m > s_l] masks of every detail coefficient of every plane at theta
    (to check that a finite-difference step crosses no kink)."""
    theta = np.asarray(theta, dtype=np.float64)
    kw = dict(sigma0=float(theta[0]), level_weight=tuple(theta[1:5]), taps=taps)
    out = []
    planes = [I for fr in cam_frames for I in sda.sda_means(np.asarray(fr)[..., None], d)[:, 0]] + list(queries)
    for I in planes:
        _, _, mk = residual_with_sensitivity(I, want_masks=True, **kw)
        out.append(np.concatenate([mk[l][k].ravel() for l in range(len(mk)) for k in mk[l]]))
    return np.concatenate(out)
