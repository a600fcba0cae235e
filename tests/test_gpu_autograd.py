"""The autograd wrappers and the recomputing squaring adjoint.

``loss.backward()`` through ExpSVF -> Warp3d -> Dissimilarity (+ Diffusion)
must give the gradient the FP64 oracle computes for the same subject loss
(itself pinned by finite differences), on 8^3 crops and on volumes spanning
several tiles; recomputing the squarings in the backward pass must give the
same gradient as keeping them.
"""

import numpy as np
import pytest
import torch

from oracle import darc_oracle as O
from paper_2508_10743_amd import autograd as AG
from paper_2508_10743_amd import darc as D
from synthetic.cohorts import WORKLOADS, make_cohort, random_velocity, random_volume

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    D.lib()
    return torch.device("cuda", 0)


def g(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def rel_l2(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("dims,amp", [((19, 21, 70), 3.0), ((20, 21, 70), 0.3)])
def test_recompute_equals_checkpointed_adjoint(dev, dims, amp):
    v = random_velocity(201, 2, dims, amp, corr_len=3.0)
    gu = random_volume(202, v.shape, -1.0, 1.0)
    vd, gud = g(v, dev), g(gu, dev)
    _, ck = D.exp_svf(vd, 7)
    a = D.exp_svf_bwd(vd, ck, gud, 7).cpu().numpy()
    b = D.exp_svf_bwd(vd, None, gud, 7).cpu().numpy()
    assert rel_l2(b, a) <= 1e-6
    for i in range(2):
        _, steps = O.exp_svf(v[i].astype(np.float64))
        assert rel_l2(b[i], O.exp_svf_bwd(steps, gu[i].astype(np.float64))) <= 1e-4


@pytest.mark.parametrize("metric,lam,win", [("mse", 0.01, 9), ("lncc", 0.01, 5), ("lncc", 0.0, 9)])
@pytest.mark.parametrize("dims", [(8, 8, 8), (12, 10, 40)])
@pytest.mark.parametrize("checkpoint", [True, False])
def test_autograd_gradient_matches_oracle(dev, metric, lam, win, dims, checkpoint):
    imgs = make_cohort(WORKLOADS["blobs-4x32^3-mse"], n=3, dims=dims, seed=203)
    atlas = imgs[2]
    v = random_velocity(204, 2, dims, 1.5, corr_len=2.5)
    vd = g(v, dev).requires_grad_(True)
    loss = AG.subject_loss(g(imgs[:2], dev), vd, g(atlas, dev), metric=metric, lam=lam, win=win,
                           checkpoint=checkpoint)
    loss.sum().backward()
    grad = vd.grad.cpu().numpy()
    p = O.SweepParams(metric=metric, win=win, lam=lam)
    for i in range(2):
        rl, rg = O.subject_loss_grad(imgs[i].astype(np.float64), v[i].astype(np.float64),
                                     atlas.astype(np.float64), p)
        assert abs(loss[i].item() - rl) <= 1e-5 * abs(rl)
        assert rel_l2(grad[i], rg) <= 1e-4


def test_autograd_directional_finite_difference(dev):
    """A loose FP32 check of the whole chain on the GPU alone."""
    dims = (8, 8, 8)
    imgs = g(make_cohort(WORKLOADS["blobs-4x32^3-mse"], n=2, dims=dims, seed=205), dev)
    v = g(random_velocity(206, 1, dims, 1.0, corr_len=2.5), dev)
    d = g(random_volume(207, (1, 3) + dims, -1.0, 1.0), dev)
    vd = v.clone().requires_grad_(True)
    loss = AG.subject_loss(imgs[:1], vd, imgs[1], metric="mse", lam=0.01)
    loss.sum().backward()
    lhs = float((vd.grad * d).sum())
    h = 1e-2
    with torch.no_grad():
        lp = AG.subject_loss(imgs[:1], (v + h * d).contiguous(), imgs[1], metric="mse", lam=0.01)
        lm = AG.subject_loss(imgs[:1], (v - h * d).contiguous(), imgs[1], metric="mse", lam=0.01)
    fd = float((lp - lm).sum()) / (2 * h)
    assert abs(lhs - fd) <= 2e-2 * abs(fd)
