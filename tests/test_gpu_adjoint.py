"""GPU adjoint against the FP64 oracle adjoint: the residual's sensitivity to
the shrinkage variances, the fixed-peak PCE gradient, and the full
matched-minus-unmatched PCE gap gradient (tiny and differentiation-workload
sizes), plus a few ascent steps on that gap."""
import numpy as np
import pytest

import synth
from oracle import adjoint
from parity import assert_scaled

torch = pytest.importorskip("torch")
from paper_1909_04573_amd import autograd, prnu  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    prnu.lib()
    return torch.device("cuda:0")


def up(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


@pytest.mark.parametrize("H,W,lw", [(96, 128, (1, 1, 1, 1)), (72, 104, (0.5, 1.5, 2.0, 0.8))])
def test_denoise_vjp_matches_oracle(dev, H, W, lw):
    """dL/ds_l against the oracle.  The FP32 path's error scales with the sum
    of the magnitudes of the terms (white-noise gradients cancel heavily), so
    the bound is 1e-4 of that sum per level; the level weights are nudged until
    no coefficient lies within 1e-5 of the shrinkage kink m = s, where FP32 and
    FP64 may take the branch differently."""
    print(f"denoise vjp {H}x{W}", flush=True)
    g = synth.rng(synth.CFG_TEST, 7000 + H)
    img = np.stack([synth.patch_camera(k, 1, H, W)[0][0] for k in range(3)]).astype(np.float32)
    lw = np.array(lw, dtype=np.float64)
    for _ in range(20):
        if min(adjoint.kink_margin(img[k].astype(np.float64), 3.0, lw) for k in range(3)) > 1e-5:
            break
        lw = lw * (1.0 + 1e-3)
    lw = tuple(float(v) for v in lw)
    gW = g.normal(0, 1, size=(3, H, W)).astype(np.float32)
    mul = g.uniform(50, 200, size=(3, H, W)).astype(np.float32)
    div = g.uniform(1e4, 4e4, size=(H, W)).astype(np.float32)
    p = prnu.denoise_params(3.0, 4, 16, lw)
    Wg, ck = prnu.denoise_residual_ckpt(up(img, dev), p)
    d_plain = prnu.denoise_residual_vjp(up(gW, dev), ck, p).cpu().numpy()
    d_scaled = prnu.denoise_residual_vjp(up(gW[0], dev), ck, p, mul=up(mul, dev), div=up(div, dev)).cpu().numpy()
    ref_plain, ref_scaled = np.zeros(4), np.zeros(4)
    mag_plain, mag_scaled = np.zeros(4), np.zeros(4)
    for k in range(3):
        Wr, sens = adjoint.residual_with_sensitivity(img[k].astype(np.float64), 3.0, lw)
        assert_scaled(Wg[k].cpu().numpy(), Wr, what="W")
        a, b = adjoint.residual_vjp_ds(gW[k].astype(np.float64), sens, want_abs=True)
        ref_plain += a
        mag_plain += b
        a, b = adjoint.residual_vjp_ds(gW[0].astype(np.float64) * mul[k] / div, sens, want_abs=True)
        ref_scaled += a
        mag_scaled += b
    assert np.all(np.abs(d_plain - ref_plain) <= 1e-4 * mag_plain), (d_plain, ref_plain, mag_plain)
    assert np.all(np.abs(d_scaled - ref_scaled) <= 1e-4 * mag_scaled), (d_scaled, ref_scaled, mag_scaled)


@pytest.mark.parametrize("h,w,modulated", [(64, 80, True), (60, 48, False)])
def test_pce_vjp_matches_oracle(dev, h, w, modulated):
    print(f"pce vjp {h}x{w}", flush=True)
    g = synth.rng(synth.CFG_TEST, 7100 + h)
    nx, ny = 2, 3
    X = g.normal(0, 1, size=(nx, h, w)).astype(np.float32)
    Y = g.normal(0, 1, size=(ny, h, w)).astype(np.float32)
    Y[0] = (0.3 * X[0] + g.normal(0, 1, size=(h, w))).astype(np.float32)
    mod = g.uniform(50, 200, size=(nx, h, w)).astype(np.float32) if modulated else None
    wts = g.normal(0, 1, size=(nx, ny))
    pce, gX, gY = prnu.pce_vjp(up(X, dev), up(Y, dev), up(wts, dev), up(mod, dev) if modulated else None)
    rX, rY = np.zeros((nx, h, w)), np.zeros((ny, h, w))
    rp = np.zeros((nx, ny))
    for q in range(nx):
        for j in range(ny):
            m = mod[q].astype(np.float64) if modulated else 1.0
            v, gx, gy = adjoint.pce_vjp(X[q].astype(np.float64), Y[j].astype(np.float64) * m)
            rp[q, j] = v
            rX[q] += wts[q, j] * gx
            rY[j] += wts[q, j] * gy * m
    np.testing.assert_allclose(pce.cpu().numpy(), rp, rtol=1e-4, atol=1e-4)
    assert_scaled(gX.cpu().numpy(), rX, what="gX")
    assert_scaled(gY.cpu().numpy(), rY, what="gY")


def _problem(ncam, nfp, nq, H, W):
    cams, qs, qc = [], [], []
    for c in range(ncam):
        p, _ = synth.patch_camera(c, nfp + nq, H, W)
        cams.append(p[:nfp])
        qs.extend(p[nfp:])
        qc.extend([c] * nq)
    return np.stack(cams), np.stack(qs), qc


@pytest.mark.parametrize("ncam,nfp,nq,H,W,d", [(2, 8, 2, 64, 64, 4), (8, 24, 8, 512, 512, 8)])
def test_gap_gradient_matches_oracle(dev, ncam, nfp, nq, H, W, d):
    """The last case is the differentiation workload: 8 cameras x 32 patches of
    512 x 512 (24 at SDA depth 8 for the fingerprint, 8 single-frame queries),
    64 matched and 448 unmatched pairs."""
    print(f"gap gradient {ncam} cams {H}x{W}", flush=True)
    cams, qs, qc = _problem(ncam, nfp, nq, H, W)
    theta = torch.tensor([3.0, 1.0, 1.0, 1.0, 1.0], dtype=torch.float64, requires_grad=True)
    L = autograd.pce_gap(theta, up(cams.astype(np.float32), dev), up(qs.astype(np.float32), dev), qc, d=d)
    L.backward()
    L = float(L.detach())
    g = theta.grad.numpy()
    cams32 = [c.astype(np.float32).astype(np.float64) for c in cams]
    qs32 = qs.astype(np.float32).astype(np.float64)
    Lr, gr, _ = adjoint.gap_loss(theta.detach().numpy(), cams32, qs32, qc, d=d)
    print(f"loss gpu {L:.6f} oracle {Lr:.6f}; grad gpu {g} oracle {gr}", flush=True)
    assert abs(L - Lr) <= 1e-4 * abs(Lr)
    assert_scaled(g, gr, what="dL/dtheta")


def test_fit_increases_the_gap(dev):
    """A few normalised gradient-ascent steps on (sigma0, lambda) increase the
    matched-minus-unmatched PCE gap."""
    cams, qs, qc = _problem(2, 8, 2, 64, 64)
    cams_t, qs_t = up(cams.astype(np.float32), dev), up(qs.astype(np.float32), dev)
    theta = torch.tensor([3.0, 1.0, 1.0, 1.0, 1.0], dtype=torch.float64)
    losses = []
    for _ in range(4):
        th = theta.clone().requires_grad_(True)
        L = autograd.pce_gap(th, cams_t, qs_t, qc, d=4)
        L.backward()
        losses.append(float(L.detach()))
        step = th.grad / th.grad.norm()
        theta = (theta + 0.05 * step).clamp(min=0.05)
    print("gap along the ascent:", losses, flush=True)
    assert losses[-1] > losses[0]
