"""Differentiable matched-vs-unmatched PCE gap (torch.autograd.Function).

The forward pass runs the fingerprint path through the C ABI: SDA frames
(Sec. III-B), residuals with their shrinkage sensitivities checkpointed per
level, the MLE fingerprint (Sec. III-B) with zero-mean, zero-mean query
residuals, and the fixed-peak PCE (Sec. IV) of every query against every
fingerprint, the query intensity modulating the fingerprint.  The loss is the
mean PCE over matched pairs minus the mean over unmatched pairs.  The backward
pass is the hand-written adjoint in the library (prnu_pce_vjp, zero-mean,
prnu_denoise_residual_vjp); the only parameters are theta = (sigma0,
lambda_1..lambda_4) with per-level noise variance s_l = lambda_l sigma0^2.
"""
from __future__ import annotations

import torch

from . import prnu


def _weights(query_cam, ncam, device):
    qc = torch.as_tensor(query_cam, device=device)
    matched = qc[:, None] == torch.arange(ncam, device=device)[None, :]
    nm, nu = int(matched.sum()), int((~matched).sum())
    w = torch.where(matched, torch.tensor(1.0 / nm, dtype=torch.float64, device=device),
                    torch.tensor(-1.0 / max(nu, 1), dtype=torch.float64, device=device))
    return w.contiguous()


class PceGapLoss(torch.autograd.Function):
    """loss = PceGapLoss.apply(theta, cam_frames, queries, query_cam, d, nbhd, taps)

    theta: float64 CPU tensor (5,); cam_frames: float32 device tensor
    [ncam][m][H][W]; queries: float32 device tensor [nq][H][W]; query_cam:
    camera index of every query.  Returns the loss as a float64 CPU scalar.
    """

    @staticmethod
    def forward(ctx, theta, cam_frames, queries, query_cam, d=8, nbhd=11, taps=16):
        th = [float(v) for v in theta.detach().cpu().tolist()]
        p = prnu.denoise_params(th[0], 4, taps, th[1:5])
        dev = queries.device
        ncam, m, H, W = cam_frames.shape
        Ks, ckpts, means_l, Bs = [], [], [], []
        for c in range(ncam):
            fr = cam_frames[c].contiguous()
            _, means = prnu.sda_average(fr, d, want_sums=False)
            means = means[:, 0].contiguous()
            _, ck = prnu.denoise_residual_ckpt(means, p)
            A, B = prnu.new_accumulators(1, H, W, device=dev)
            prnu.fingerprint_accumulate(fr, d, A, B, p)
            Ks.append(prnu.fingerprint_finalize(A, B, flags=prnu.ZM))
            ckpts.append(ck)
            means_l.append(means)
            Bs.append(B[0].float().contiguous())
        K = torch.stack(Ks).contiguous()
        Wq, ckq = prnu.denoise_residual_ckpt(queries.contiguous(), p)
        xq = prnu.postprocess(Wq, 1, prnu.ZM)
        wts = _weights(query_cam, ncam, dev)
        pce, gX, gY = prnu.pce_vjp(xq, K, wts, modulate=queries.contiguous(), nbhd=nbhd)
        loss = (pce * wts).sum()
        ctx.p = p
        ctx.theta = th
        ctx.saved = (ckpts, means_l, Bs, ckq, gX, gY)
        ctx.pce = pce
        return loss.detach().cpu()

    @staticmethod
    def backward(ctx, gL):
        ckpts, means_l, Bs, ckq, gX, gY = ctx.saved
        p = ctx.p
        sigma0, lam = ctx.theta[0], ctx.theta[1:5]
        dev = gX.device
        dLds = torch.zeros(4, dtype=torch.float64, device=dev)
        gK = prnu.postprocess(gY.contiguous(), 1, prnu.ZM)  # zero-mean is self-adjoint
        for c, ck in enumerate(ckpts):
            prnu.denoise_residual_vjp(gK[c].contiguous(), ck, p, mul=means_l[c], div=Bs[c], dLds=dLds)
        gWq = prnu.postprocess(gX.contiguous(), 1, prnu.ZM)
        prnu.denoise_residual_vjp(gWq, ckq, p, dLds=dLds)
        ds = dLds.cpu()
        g = torch.zeros(5, dtype=torch.float64)
        g[0] = float(torch.sum(ds * 2.0 * torch.tensor(lam, dtype=torch.float64) * sigma0))
        g[1:5] = ds * sigma0 * sigma0
        return g * float(gL), None, None, None, None, None, None


def pce_gap(theta, cam_frames, queries, query_cam, d=8, nbhd=11, taps=16):
    return PceGapLoss.apply(theta, cam_frames, queries, query_cam, d, nbhd, taps)
