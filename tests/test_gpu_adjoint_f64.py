"""FP64 mode of the differentiated chain (prnu_pce_gap_f64) against the FP64
oracle adjoint, and against its own central finite differences: the
matched-minus-unmatched PCE gap and its gradient with respect to
(sigma0, lambda_1..4), at a small size and at the differentiation workload
(8 cameras x 32 patches of 512 x 512)."""
import numpy as np
import pytest

import synth
from oracle import adjoint, sda

torch = pytest.importorskip("torch")
from paper_1909_04573_amd import prnu  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    prnu.lib()
    return torch.device("cuda:0")


def up(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)


def _problem(ncam, nfp, nq, H, W):
    cams, qs, qc = [], [], []
    for c in range(ncam):
        p, _ = synth.patch_camera(c, nfp + nq, H, W)
        cams.append(p[:nfp])
        qs.extend(p[nfp:])
        qc.extend([c] * nq)
    return np.stack(cams).astype(np.float32), np.stack(qs).astype(np.float32), qc


def _kink_free(cams, qs, d, theta, margin):
    """theta nudged until no detail coefficient of any plane lies within
    `margin` (relative) of its level's shrinkage kink."""
    theta = np.asarray(theta, dtype=np.float64)
    planes = [I for fr in cams for I in sda.sda_means(np.asarray(fr, np.float64)[..., None], d)[:, 0]]
    planes += list(np.asarray(qs, np.float64))
    step = np.array([1.0, 1.0013, 1.0017, 1.0019, 1.0023])
    for _ in range(60):
        if min(adjoint.kink_margin(I, theta[0], tuple(theta[1:])) for I in planes) > margin:
            return theta
        theta = theta * step
    raise AssertionError("no kink-free theta found")


def test_f64_gap_matches_oracle_small(dev):
    """2 cameras x 10 patches of 64 x 64 (8 at SDA depth 4, 2 queries each):
    loss and every PCE within 1e-10 relative, every gradient component within
    1e-9 of its own value (FP64 on both sides; only the summation order
    differs)."""
    cams, qs, qc = _problem(2, 8, 2, 64, 64)
    theta = _kink_free(cams, qs, 4, [3.0, 1.0, 1.0, 1.0, 1.0], 1e-6)
    L, g, P = prnu.pce_gap_f64(theta, up(cams, dev), up(qs, dev), qc, d=4)
    Lr, gr, Pr = adjoint.gap_loss(theta, [c.astype(np.float64) for c in cams], qs.astype(np.float64), qc, d=4)
    print(f"f64 gap small: loss {L!r} oracle {Lr!r}; grad {g} oracle {gr}", flush=True)
    assert abs(L - Lr) <= 1e-10 * abs(Lr)
    np.testing.assert_allclose(P, Pr, rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(g, gr, rtol=1e-9, atol=0)


def test_f64_gap_finite_differences(dev):
    """Central differences of the FP64 GPU loss (step 1e-6 relative per
    component) against its FP64 gradient, within 1e-5 relative, at a theta
    where no coefficient lies within 1e-4 of a kink (the steps cross none)."""
    cams, qs, qc = _problem(2, 8, 2, 64, 64)
    ct, qt = up(cams, dev), up(qs, dev)
    theta = _kink_free(cams, qs, 4, [3.0, 1.0, 1.0, 1.0, 1.0], 1e-4)
    _, g, _ = prnu.pce_gap_f64(theta, ct, qt, qc, d=4)
    fd = np.zeros(5)
    for k in range(5):
        h = 1e-6 * theta[k]
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd[k] = (prnu.pce_gap_f64(tp, ct, qt, qc, d=4)[0] - prnu.pce_gap_f64(tm, ct, qt, qc, d=4)[0]) / (2 * h)
    print(f"f64 gap FD: grad {g} central differences {fd}", flush=True)
    np.testing.assert_allclose(g, fd, rtol=1e-5, atol=0)


def test_f64_gap_differentiation_workload(dev):
    """The differentiation workload: 8 cameras x 32 patches of 512 x 512 (24 at
    SDA depth 8, 8 single-frame queries each; 64 matched and 448 unmatched
    pairs) at theta = (3, 1, 1, 1, 1): every gradient component within 1e-5 of
    its own value, the loss within 1e-10."""
    print("f64 gap 8 cams 512x512", flush=True)
    cams, qs, qc = _problem(8, 24, 8, 512, 512)
    theta = np.array([3.0, 1.0, 1.0, 1.0, 1.0])
    L, g, P = prnu.pce_gap_f64(theta, up(cams, dev), up(qs, dev), qc, d=8)
    Lr, gr, Pr = adjoint.gap_loss(theta, [c.astype(np.float64) for c in cams], qs.astype(np.float64), qc, d=8)
    rel = np.abs(g - gr) / np.abs(gr)
    print(f"f64 gap workload: loss {L!r} oracle {Lr!r}; grad {g} oracle {gr}; err/|own| {rel}", flush=True)
    assert abs(L - Lr) <= 1e-10 * abs(Lr)
    np.testing.assert_allclose(P, Pr, rtol=1e-9, atol=1e-9)
    assert np.all(rel <= 1e-5), rel
