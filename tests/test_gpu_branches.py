"""GPU parity of the method's other branches against the FP64 oracle: the L1
metric and its median atlas, the minibatch stochastic atlas for NCC, label
propagation and one-shot segmentation with Dice counts, factor-2
resampling, sweeps using them, and a two-level coarse-to-fine run.

Tolerances as for the main path: atlas and resampled values rel-L-inf <=
1e-5, velocities rel-L2 <= 1e-4, losses rel <= 1e-6 (in a second sweep
1e-5, the FP32 state having drifted);
labels and counts exact.  One-shot segmentation against the oracle's own
FP64 Exp(-v) may differ only at voxels whose position lies within 1e-4 voxel
of a rounding boundary; given the same FP32 displacement it is exact.
"""

import numpy as np
import pytest
import torch

from oracle import darc_oracle as O
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


def h(t):
    return t.detach().cpu().numpy()


def rel_linf(a, b):
    return float(np.abs(np.asarray(a, np.float64) - b).max() / max(np.abs(b).max(), 1e-300))


def rel_l2(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def blobs(n, dims, seed):
    return make_cohort(WORKLOADS["blobs-4x32^3-mse"], n=n, dims=dims, seed=seed)


# --------------------------------------------------------------------- L1


@pytest.mark.parametrize("dims", [(8, 8, 8), (17, 9, 70)])
def test_l1_loss_and_gradient(dev, dims):
    W = blobs(4, dims, 401)
    A = (W.mean(0) + 0.003).astype(np.float32)
    loss, gw = D.sim_grad(g(W, dev), g(A, dev), "l1")
    for i in range(4):
        rl, rg = O.l1(W[i], A)
        assert abs(loss[i].item() - rl) <= 1e-6 * abs(rl)
        assert rel_l2(h(gw[i]), rg) <= 1e-6


@pytest.mark.parametrize("n", [1, 2, 3, 4, 7, 16])
def test_median_atlas(dev, n):
    dims = (19, 12, 40)
    imgs = blobs(n, dims, 402 + n)
    u = random_velocity(403, n, dims, 2.0, corr_len=3.0)
    mean = u.mean(0).astype(np.float32)
    A = D.atlas_median(g(imgs, dev), g(u, dev), g(mean, dev))
    ref = O.atlas_median(imgs, u.astype(np.float64) - mean[None])
    assert rel_linf(h(A), ref) <= 1e-5
    A0 = D.atlas_median(g(imgs, dev), g(np.zeros_like(u), dev))
    assert np.array_equal(h(A0), np.median(imgs, axis=0).astype(np.float32)) or \
        rel_linf(h(A0), np.median(imgs.astype(np.float64), axis=0)) <= 1e-7


def test_median_atlas_many_subjects(dev):
    """n = 300 takes the 32-thread layout (n * 64 floats would not fit)."""
    imgs = random_volume(404, (300, 4, 6, 10), 0.0, 1.0)
    A = D.atlas_median(g(imgs, dev), g(np.zeros((300, 3, 4, 6, 10), np.float32), dev))
    assert rel_linf(h(A), np.median(imgs.astype(np.float64), axis=0)) <= 1e-7


# -------------------------------------------------------- stochastic atlas


@pytest.mark.parametrize("n,batch,epochs,win", [(5, 2, 3, 5), (4, 4, 2, 9), (3, 1, 2, 3)])
def test_sgd_atlas(dev, n, batch, epochs, win):
    dims = (12, 10, 40)
    W = blobs(n, dims, 405)
    A0 = (W.mean(0) * 0.8 + 0.05).astype(np.float32)
    A = g(A0, dev)
    losses = D.atlas_sgd(g(W, dev), A, epochs=epochs, batch=batch, win=win)
    rA, rls = O.atlas_sgd(W.astype(np.float64), A0.astype(np.float64), epochs, batch, win)
    assert rel_linf(h(A), rA) <= 1e-5
    assert np.abs(h(losses) - rls).max() <= 1e-6 * np.abs(rls).max()


# ------------------------------------------------------------ segmentation


def test_label_warp_is_exact(dev):
    dims = (11, 13, 37)
    L = np.random.default_rng(406).integers(0, 7, size=dims).astype(np.uint8)
    # half-integer displacements land exactly on rounding boundaries
    u = (np.round(random_velocity(407, 3, dims, 3.0, corr_len=3.0) * 2) / 2).astype(np.float32)
    u[0, 0, :2] = np.nan  # NaN positions get the background label
    out = h(D.warp_labels(g(L, dev), g(u, dev)))
    for i in range(3):
        assert np.array_equal(out[i], O.warp_labels_nearest(L, u[i]))


def test_one_shot_segmentation(dev):
    dims = (16, 14, 40)
    L = np.zeros(dims, np.uint8)
    L[3:12, 2:11, 5:35] = 1
    L[6:9, 5:8, 10:30] = 2
    v = random_velocity(408, 3, dims, 2.5, corr_len=4.0)
    out = h(D.segment(g(L, dev), g(v, dev)))
    u_neg, _ = D.exp_svf(g(-v, dev), 7)
    u_neg = h(u_neg)
    V = int(np.prod(dims))
    for i in range(3):
        # the fused path equals label propagation along the GPU's own Exp(-v)
        assert np.array_equal(out[i], O.warp_labels_nearest(L, u_neg[i]))
        # against the oracle's FP64 Exp(-v): only near-boundary voxels may differ
        ref = O.segment_one_shot(L, v[i].astype(np.float64))
        u_ref, _ = O.exp_svf(-v[i].astype(np.float64))
        p = O.identity_grid(dims) + u_ref
        near = (np.abs(p - np.floor(p) - 0.5) < 1e-4).any(axis=0)
        assert np.all(near[out[i] != ref])
        assert np.count_nonzero(out[i] != ref) <= 1e-3 * V


def test_dice_counts(dev):
    rng = np.random.default_rng(409)
    a = rng.integers(0, 6, size=(3, 7, 9, 31)).astype(np.uint8)
    b = np.where(rng.uniform(size=a.shape) < 0.6, a, rng.integers(0, 6, size=a.shape)).astype(np.uint8)
    c = h(D.dice_counts(g(a, dev), g(b, dev), 5))  # label 5 is not counted
    for i in range(3):
        assert np.array_equal(c[i], O.dice_counts(a[i], b[i], 5))


# -------------------------------------------------------------- resampling


def test_down2_up2(dev):
    f = random_volume(410, (2, 3, 10, 12, 38), -1.0, 1.0)
    d = D.down2(g(f, dev))
    assert rel_linf(h(d), O.down2(f)) <= 1e-6
    u = D.up2(d, 2.0)
    ref = np.stack([O.up2(h(d)[i].astype(np.float64), 2.0) for i in range(2)])
    assert rel_linf(h(u), ref) <= 1e-6
    imgs = blobs(3, (16, 12, 20), 411)
    assert rel_linf(h(D.down2(g(imgs, dev))), O.down2(imgs)) <= 1e-6


# ------------------------------------------------------------------ sweeps


def _run_pair(dev, imgs, p_gpu, p_or, sweeps, atlas_tol=1e-5, group_tol_first=1e-6,
              level_start=False):
    """Sweeps on the GPU and in the oracle from the same start.  Losses rel
    1e-6 in the first sweep (the state is the oracle's up to FP32 storage),
    1e-5 after; ``group_tol_first`` loosens the first group loss where the
    atlas tolerance is looser.  ``level_start``: both start from the atlas of
    the unwarped subjects under the sweep's own atlas mode."""
    coh = D.Cohort(g(imgs, dev), p_gpu)
    n = len(imgs)
    v = np.zeros((n, 3) + imgs.shape[1:])
    m, s, step, A = v.copy(), v.copy(), 0, O.initial_atlas(imgs.astype(np.float64))
    if level_start:
        coh.level_start()
        v, A = O.level_start(imgs.astype(np.float64), v, p_or)
        assert rel_linf(h(coh.atlas), A) <= 1e-6
    for k in range(sweeps):
        lg = h(coh.sweep())
        r = O.sweep(imgs.astype(np.float64), v, m, s, step, A, p_or)
        v, m, s, step, A = r["v"], r["m"], r["s"], r["step"], r["atlas"]
        tol = 1e-6 if k == 0 else 1e-5
        if p_or.k2:
            inner = r["inner_losses"].ravel()
            assert np.abs(lg[:-1] - inner).max() <= tol * np.abs(inner).max(), k
        gtol = max(tol, group_tol_first) if k == 0 else tol
        assert abs(lg[-1] - r["group_loss"]) <= gtol * abs(r["group_loss"]), k
        assert rel_l2(h(coh.v), v) <= 1e-4
        assert rel_linf(h(coh.atlas), A) <= atlas_tol
    return coh


def test_l1_sweep_with_median_atlas(dev):
    """The L1 subgradient sign(Iw - A) jumps where a warped subject meets the
    atlas; where |Iw - A| is below the FP32 rounding of the warp (the faint
    tails of the blobs) the sign, and with it the whole trajectory, is decided
    by rounding.  Distinct intensity offsets per subject keep every subject
    away from the median, so the comparison is well conditioned; the
    gradient itself is checked near ties by test_l1_loss_and_gradient."""
    imgs = blobs(4, (12, 10, 40), 412) + (0.25 * np.arange(4, dtype=np.float32))[:, None, None, None]
    _run_pair(dev, imgs, D.SweepParams(metric="l1", k2=3), O.SweepParams(metric="l1", k2=3), 2)


def test_l1_sweep_through_exact_ties(dev):
    """An odd cohort against its median atlas: at every voxel one subject is
    the median, so Iw - A = 0 exactly there for a fifth of all subject-voxels.
    With one inner step from v = 0 these ties are exact on both sides
    (Iw = I_i, A one of the I_i) and the subgradient there is 0 (sign(0) = 0,
    the difference formed in FP64 from the FP32 operands), so the whole sweep
    matches the oracle at the usual tolerances."""
    imgs = blobs(5, (12, 10, 40), 418)
    n, V = 5, imgs[0].size
    A = np.median(imgs.astype(np.float64), axis=0)
    ties = sum(int((imgs[i] == A).sum()) for i in range(n))
    assert ties >= V  # every voxel has its median subject
    kw = dict(metric="l1", k2=1, atlas_mode="median")
    _run_pair(dev, imgs, D.SweepParams(**kw), O.SweepParams(**kw), 1, level_start=True)


def test_l1_inner_steps_accept_either_sign_at_near_ties(dev):
    """Three inner steps of every subject of an odd cohort against its median
    atlas, driven through the separate entry points so that the GPU's L1
    subgradient dD/dIw is seen at each step.  After the first step most ties
    are no longer exact: where the oracle's |Iw - A| (FP64, at the oracle's
    state) exceeds FP32 rounding, tau = 2^-20 max(|Iw|, |A|), the GPU's
    subgradient must have the sign of Iw - A (0 at exact ties); below tau but
    not zero either sign or 0 is accepted, the decision being the rounding's.
    The oracle then continues from the GPU's decisions at those voxels, so
    both take the same path: losses rel 1e-6 and velocities rel-L2 1e-4 after
    every step.  No regulariser (lambda = 0): the ties are the data term's."""
    dims = (12, 10, 40)
    imgs = blobs(5, dims, 420)
    n, V = 5, imgs[0].size
    p = O.SweepParams(metric="l1", k2=3, atlas_mode="median", lam=0.0)
    x = imgs.astype(np.float64)
    v, A = O.level_start(x, np.zeros((n, 3) + dims), p)
    m, s = np.zeros_like(v), np.zeros_like(v)
    Ig, Ag = g(imgs, dev), g(A.astype(np.float32), dev)
    assert np.array_equal(A.astype(np.float32), A)  # a median of FP32 values
    vg = torch.zeros((n, 3) + dims, dtype=torch.float32, device=dev)
    mg, sg = torch.zeros_like(vg), torch.zeros_like(vg)
    exact_total = near_total = 0
    for k in range(p.k2):
        ug, ck = D.exp_svf(vg, p.n_sq)
        wg = D.warp3d(Ig, ug)
        lossg, gwg = D.sim_grad(wg, Ag, "l1")
        gug = D.warp3d_bwd(Ig, ug, gwg)
        gvg = D.exp_svf_bwd(vg, ck, gug, p.n_sq)
        D.adam_step(vg, mg, sg, gvg, k + 1, p.lr, p.beta1, p.beta2, p.adam_eps)
        lossg, gw_all = h(lossg), h(gwg)
        for i in range(n):
            u, steps = O.exp_svf(v[i], p.n_sq)
            Iw = O.warp3d(x[i], u)
            d = Iw - A
            rl = float(np.abs(d).mean())
            assert abs(lossg[i] - rl) <= 1e-6 * rl, (k, i)
            near = (d != 0) & (np.abs(d) <= 2.0 ** -20 * np.maximum(np.abs(Iw), np.abs(A)))
            sg_gpu = np.sign(gw_all[i])
            assert np.array_equal(sg_gpu[~near], np.sign(d)[~near]), (k, i)
            assert np.allclose(np.abs(gw_all[i])[sg_gpu != 0], 1.0 / V, rtol=1e-6)
            exact_total += int((d == 0).sum())
            near_total += int(near.sum())
            w = np.sign(d) / V
            w[near] = sg_gpu[near] / V
            gv = O.exp_svf_bwd(steps, O.warp3d_bwd(x[i], u, w))
            v[i], m[i], s[i] = O.adam_step(v[i], m[i], s[i], gv, k + 1, p.lr, p.beta1, p.beta2,
                                           p.adam_eps)
        assert rel_l2(h(vg), v) <= 1e-4, k
    # both kinds of tie occurred: exact ones (a fifth of the subject-voxels at
    # the first step) and ones decided by rounding
    assert exact_total >= V and near_total > 0, (exact_total, near_total)


def test_lncc_sweep_with_sgd_atlas(dev):
    """Atlas tolerance 1e-4: where the minibatch gradient g is near Adam's
    eps (1e-8) the step lr g / (|g| + eps) passes an absolute error of g on
    amplified by lr / eps, and in flat background the four terms of the LNCC
    adjoint cancel to that size; over the 2 x 9 atlas steps of two sweeps this
    reaches a few 1e-5 of the atlas range, while the warped inputs already
    carry the velocities' ~1e-5.  The group loss at that atlas: 1e-5."""
    imgs = blobs(5, (12, 10, 40), 413)
    kw = dict(metric="lncc", win=5, k2=2, atlas_mode="sgd", k3=3, atlas_batch=2)
    _run_pair(dev, imgs, D.SweepParams(batch=2, **kw), O.SweepParams(**kw), 2, atlas_tol=1e-4,
              group_tol_first=1e-5)


def test_lncc_sweep_with_sgd_atlas_literal_start(dev):
    """Algorithm 1's ``A = initialize()`` read literally: every stochastic
    update restarts from A^0 (the mean of the unwarped subjects).  Tolerance
    as in the warm-started case."""
    imgs = blobs(5, (12, 10, 40), 417)
    kw = dict(metric="lncc", win=5, k2=2, atlas_mode="sgd", k3=3, atlas_batch=2,
              sgd_init="initial")
    _run_pair(dev, imgs, D.SweepParams(batch=2, **kw), O.SweepParams(**kw), 2, atlas_tol=1e-4,
              group_tol_first=1e-5)


def test_atlas_update_without_displacements_is_the_mean(dev):
    """u = NULL: A^0, the FP64 mean of the unwarped subjects rounded once."""
    imgs = blobs(7, (9, 14, 33), 418)
    A = D.atlas_update(g(imgs, dev), None)
    ref = imgs.astype(np.float64).mean(axis=0).astype(np.float32)
    assert np.array_equal(h(A), ref)


def test_level_start_is_steps_two_and_three(dev):
    imgs = blobs(3, (12, 10, 40), 414)
    v = random_velocity(415, 3, (12, 10, 40), 1.0, corr_len=3.0)
    for mode, metric in (("mean", "mse"), ("median", "l1"), ("sgd", "lncc")):
        p = D.SweepParams(metric=metric, win=5, atlas_mode=mode, k3=2, atlas_batch=2)
        coh = D.Cohort(g(imgs, dev), p, v0=g(v, dev))
        F = h(coh.level_start())[0]
        po = O.SweepParams(metric=metric, win=5, atlas_mode=mode, k3=2, atlas_batch=2)
        _, A = O.level_start(imgs.astype(np.float64), v.astype(np.float64), po)
        assert rel_linf(h(coh.atlas), A) <= 1e-5, mode
        assert np.isfinite(F)


def test_two_level_pyramid_matches_oracle(dev):
    """Each stage against the oracle from the same inputs: the coarse level
    from v = 0, the carried velocities, and the fine level from the GPU's
    carried velocities.  (Compounded over levels, the fresh Adam moments of
    the fine level take lr * sign(g) steps, so a velocity difference of 1e-5
    at the carry flips the steps of the few entries where g crosses zero:
    the end states then agree in the loss, not entrywise.)"""
    imgs = blobs(3, (12, 16, 20), 416)
    p, po = D.SweepParams(k2=2), O.SweepParams(k2=2)
    pyr = D.Pyramid(g(imgs, dev), p, levels=2)
    coarse = O.down2(imgs)
    assert rel_linf(h(pyr.images[0]), coarse) <= 1e-6
    pyr.sweep()
    z = np.zeros((3, 3) + coarse.shape[1:])
    r0 = O.sweep(h(pyr.images[0]).astype(np.float64), z, z, z, 0,
                 O.initial_atlas(h(pyr.images[0]).astype(np.float64)), po)
    assert rel_l2(h(pyr.cohort.v), r0["v"]) <= 1e-4
    v_coarse = h(pyr.cohort.v).astype(np.float64)
    pyr.next_level()
    v_up = h(pyr.cohort.v).astype(np.float64)
    assert rel_linf(v_up, np.stack([O.up2(v_coarse[i], 2.0) for i in range(3)])) <= 1e-6
    _, A1 = O.level_start(imgs.astype(np.float64), v_up, po)
    assert rel_linf(h(pyr.cohort.atlas), A1) <= 1e-5
    pyr.sweep()
    z = np.zeros_like(v_up)
    r1 = O.sweep(imgs.astype(np.float64), v_up, z, z, 0, A1, po)
    assert rel_l2(h(pyr.cohort.v), r1["v"]) <= 1e-4
    assert rel_linf(h(pyr.cohort.atlas), r1["atlas"]) <= 1e-5
    assert abs(pyr.cohort.group_loss() - r1["group_loss"]) <= 1e-5 * abs(r1["group_loss"])
    ref = O.pyramid(imgs.astype(np.float64), 2, [1, 1], po)
    assert abs(pyr.cohort.group_loss() - ref["group_loss"]) <= 1e-3 * abs(ref["group_loss"])
