"""Pins of the oracle's other branches of the method: the L1 metric and its
median atlas, the minibatch stochastic atlas update for NCC, one-shot label
propagation and its Dice score, and the factor-2 resampling of a
coarse-to-fine schedule.  Each is tied to a closed form, a brute-force
definition, an optimality property or finite differences.  CPU only."""

import numpy as np
import pytest

from oracle import darc_oracle as O
from synthetic.cohorts import WORKLOADS, make_cohort, random_velocity


def rel_l2(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# ------------------------------------------------------------------------- L1


def test_l1_closed_forms():
    rng = np.random.default_rng(1)
    A = rng.uniform(size=(4, 5, 6))
    for delta in (0.25, -0.5):
        loss, g = O.l1(A + delta, A)
        assert loss == pytest.approx(abs(delta), abs=1e-15)
        assert np.allclose(g, np.sign(delta) / A.size, atol=0)
    loss, g = O.l1(A, A)
    assert loss == 0.0 and not g.any()


def test_l1_gradient_by_finite_differences():
    rng = np.random.default_rng(2)
    A = rng.uniform(size=(4, 4, 5))
    I = A + rng.choice([-1.0, 1.0], size=A.shape) * rng.uniform(0.1, 0.5, size=A.shape)
    _, g = O.l1(I, A)
    h = 1e-6
    for _ in range(20):
        k = tuple(rng.integers(0, s) for s in A.shape)
        Ip, Im = I.copy(), I.copy()
        Ip[k] += h
        Im[k] -= h
        fd = (O.l1(Ip, A)[0] - O.l1(Im, A)[0]) / (2 * h)
        assert fd == pytest.approx(g[k], rel=1e-7)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 7])
def test_median_atlas_is_the_order_statistic_and_minimises_l1(n):
    rng = np.random.default_rng(10 + n)
    dims = (3, 4, 5)
    imgs = rng.uniform(size=(n,) + dims)
    u = np.zeros((n, 3) + dims)
    A = O.atlas_median(imgs, u)
    # brute force: sort each voxel's n values
    for k in np.ndindex(dims):
        vals = sorted(imgs[(slice(None),) + k])
        ref = vals[n // 2] if n % 2 else 0.5 * (vals[n // 2 - 1] + vals[n // 2])
        assert A[k] == ref
    # optimality: sum_i |I_i - A| does not decrease at any perturbed atlas
    cost = np.abs(imgs - A[None]).sum(axis=0)
    for d in (1e-3, -1e-3, 0.1, -0.1):
        assert np.all(np.abs(imgs - (A + d)[None]).sum(axis=0) >= cost - 1e-12)


def test_median_atlas_uses_the_warped_subjects():
    imgs = make_cohort(WORKLOADS["blobs-4x32^3-mse"], n=3, dims=(8, 8, 10), seed=3)
    u = np.zeros((3, 3, 8, 8, 10))
    u[:, 2] = 1.0  # integer shift along axis 2: I(x + 1), zero past the end
    shifted = np.concatenate([imgs[..., 1:], np.zeros(imgs.shape[:-1] + (1,))], axis=-1)
    assert np.array_equal(O.atlas_median(imgs, u), np.median(shifted, axis=0))


# ------------------------------------------------------------ NCC SGD atlas


def test_lncc_is_symmetric_and_atlas_gradient_matches_finite_differences():
    rng = np.random.default_rng(4)
    I = rng.uniform(size=(6, 7, 8))
    A = 0.5 * I + rng.uniform(size=I.shape) * 0.5
    l1_, _ = O.lncc(I, A, 5)
    l2_, _ = O.lncc(A, I, 5)
    assert l1_ == pytest.approx(l2_, rel=1e-13)
    loss, gA = O.lncc_atlas_grad(I, A, 5)
    assert loss == pytest.approx(l1_, rel=1e-13)
    h = 1e-6
    for _ in range(12):
        k = tuple(rng.integers(0, s) for s in A.shape)
        Ap, Am = A.copy(), A.copy()
        Ap[k] += h
        Am[k] -= h
        fd = (O.lncc(I, Ap, 5)[0] - O.lncc(I, Am, 5)[0]) / (2 * h)
        assert fd == pytest.approx(gA[k], rel=1e-5, abs=1e-12)


def test_sgd_atlas_first_step_and_descent():
    rng = np.random.default_rng(5)
    W = make_cohort(WORKLOADS["blobs-4x32^3-mse"], n=4, dims=(10, 10, 12), seed=6).astype(np.float64)
    A0 = rng.uniform(size=W.shape[1:])
    # one epoch, one minibatch holding everything: Adam's first step moves each
    # voxel by lr * g / (|g| + eps) against the mean gradient
    A1, losses = O.atlas_sgd(W, A0, epochs=1, batch=4, win=5, lr=1e-2)
    g = np.mean([O.lncc(A0, W[i], 5)[1] for i in range(4)], axis=0)
    assert np.allclose(A1, A0 - 1e-2 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-12)
    assert losses[0] == pytest.approx(np.mean([O.lncc(W[i], A0, 5)[0] for i in range(4)]))
    # minibatches of 2: two steps per epoch, and the loss goes down over epochs
    A, losses = O.atlas_sgd(W, A0, epochs=15, batch=2, win=5, lr=2e-2)
    assert len(losses) == 30
    assert np.mean(losses[-2:]) < np.mean(losses[:2]) - 0.05


def test_sweep_with_sgd_atlas_and_l1_runs_and_descends():
    imgs = make_cohort(WORKLOADS["blobs-4x32^3-mse"], n=3, dims=(8, 8, 10), seed=7).astype(np.float64)
    for p in (O.SweepParams(metric="l1", k2=3, lam=0.01),
              O.SweepParams(metric="lncc", win=5, k2=2, atlas_mode="sgd", k3=2, atlas_batch=2)):
        n = len(imgs)
        v = np.zeros((n, 3) + imgs.shape[1:])
        r = O.sweep(imgs, v, v, v, 0, O.initial_atlas(imgs), p)
        if p.metric == "l1":
            assert np.array_equal(r["atlas"], O.atlas_median(imgs, r["u_hat"]))
        else:
            W = np.stack([O.warp3d(imgs[i], r["u_hat"][i]) for i in range(n)])
            ref, _ = O.atlas_sgd(W, O.initial_atlas(imgs), 2, 2, 5)
            assert np.array_equal(r["atlas"], ref)
        assert r["inner_losses"][:, -1].mean() < r["inner_losses"][:, 0].mean()


# ------------------------------------------------------------- segmentation


def test_label_warp_rounds_to_the_nearest_voxel():
    rng = np.random.default_rng(8)
    L = rng.integers(0, 5, size=(6, 7, 8)).astype(np.uint8)
    u = np.zeros((3, 6, 7, 8), np.float32)
    assert np.array_equal(O.warp_labels_nearest(L, u), L)
    u[:] = 0.49
    assert np.array_equal(O.warp_labels_nearest(L, u), L)
    for c in (0.5, 0.51, 1.2):  # a half rounds up; all shift by one voxel
        u[:] = 0.0
        u[1] = c
        ref = np.zeros_like(L)
        ref[:, :-1] = L[:, 1:]
        assert np.array_equal(O.warp_labels_nearest(L, u), ref)
    u[:] = 0.0
    u[2] = -2.0
    ref = np.zeros_like(L)
    ref[:, :, 2:] = L[:, :, :-2]
    assert np.array_equal(O.warp_labels_nearest(L, u), ref)


def test_one_shot_segmentation_inverts_a_translation():
    rng = np.random.default_rng(9)
    L = rng.integers(0, 4, size=(6, 7, 9)).astype(np.uint8)
    v = np.zeros((3, 6, 7, 9))
    v[2] = 2.0  # Exp(v) translates by +2, Exp(-v) by -2 (border sampling keeps it exact)
    ref = np.zeros_like(L)
    ref[:, :, 2:] = L[:, :, :-2]
    assert np.array_equal(O.segment_one_shot(L, v), ref)


def test_dice_counts_by_brute_force():
    rng = np.random.default_rng(10)
    a = rng.integers(0, 4, size=200)
    b = np.where(rng.uniform(size=200) < 0.7, a, rng.integers(0, 4, size=200))
    c = O.dice_counts(a, b, 5)
    for lab in range(5):
        inter = sum(1 for x, y in zip(a, b) if x == lab and y == lab)
        assert tuple(c[lab]) == (inter, int((a == lab).sum()), int((b == lab).sum()))
    assert np.array_equal(O.dice_counts(a, a, 4)[:, 0], O.dice_counts(a, a, 4)[:, 1])


# --------------------------------------------------------------- resampling


def test_down2_and_up2_on_constant_and_linear_fields():
    dims = (6, 8, 10)
    x = O.identity_grid(dims)
    coef = np.array([0.3, -0.7, 1.1])
    lin = np.tensordot(coef, x, axes=1) + 2.0
    d = O.down2(lin)
    k = O.identity_grid(d.shape)
    assert np.allclose(d, np.tensordot(coef, 2 * k + 0.5, axes=1) + 2.0, atol=1e-13)
    assert np.allclose(O.down2(np.full(dims, 3.5)), 3.5, atol=0)
    f = np.stack([d, -d, 0.5 * d])
    up = O.up2(f, scale=2.0)
    assert up.shape == (3,) + dims
    inner = (slice(None), slice(1, -1), slice(1, -1), slice(1, -1))
    assert np.allclose(up[inner], (2.0 * np.stack([lin, -lin, 0.5 * lin]))[inner], atol=1e-12)
    assert np.allclose(O.up2(np.full((3, 3, 4, 5), 1.25), 2.0), 2.5, atol=0)


def test_one_level_pyramid_is_a_plain_run():
    imgs = make_cohort(WORKLOADS["blobs-4x32^3-mse"], n=2, dims=(8, 8, 8), seed=11).astype(np.float64)
    p = O.SweepParams(k2=2)
    out = O.pyramid(imgs, 1, [2], p)
    v = np.zeros((2, 3, 8, 8, 8))
    r = O.sweep(imgs, v, v, v, 0, O.initial_atlas(imgs), p)
    r = O.sweep(imgs, r["v"], r["m"], r["s"], r["step"], r["atlas"], p)
    assert np.array_equal(out["v"], r["v"]) and np.array_equal(out["atlas"], r["atlas"])
    out2 = O.pyramid(imgs, 2, [1, 1], p)
    assert out2["v"].shape == (2, 3, 8, 8, 8) and np.isfinite(out2["group_loss"])
