"""Pins of the oracle's sweep-level functions: the group objective, the start
of a level, the coarse-to-fine schedule, the restart of the velocities and the
Jacobian determinant.

Each value is rebuilt here from a closed form or from SciPy/NumPy routines
that the oracle does not use for it (``map_coordinates`` for the warp,
``uniform_filter`` for the window sums, ``np.diff`` for the regulariser), so
that evaluating the objective at the old atlas, dropping the regulariser, or
skipping the centring fails.  CPU only.
"""

import numpy as np
import pytest
from scipy import ndimage

from oracle import darc_oracle as O
from synthetic.cohorts import WORKLOADS, make_cohort, random_velocity


def _warp_scipy(img, u):
    """I(x + u(x)), trilinear, zero outside: SciPy's grid-constant mode."""
    pos = O.identity_grid(img.shape) + u
    return ndimage.map_coordinates(np.asarray(img, np.float64), pos.reshape(3, -1), order=1,
                                   mode="grid-constant", cval=0.0).reshape(img.shape)


def _diffusion_by_hand(u):
    """(1/3) sum_d mean over components and voxels with a forward neighbour
    along d of the squared forward difference."""
    return sum(float((np.diff(u, axis=d + 1) ** 2).mean()) for d in range(3)) / 3.0


def _lncc_by_hand(a, b, win, eps):
    """-mean cc with zero-padded window sums from SciPy's uniform filter."""
    N = float(win ** 3)

    def box(f):
        return ndimage.uniform_filter(f, size=win, mode="constant", cval=0.0) * N

    sa, sb = box(a), box(b)
    cross = box(a * b) - sa * sb / N
    va = box(a * a) - sa * sa / N
    vb = box(b * b) - sb * sb / N
    return -float((cross * cross / (va * vb + eps)).mean())


def _cohort(n=3, dims=(10, 9, 11), seed=21):
    w = WORKLOADS["blobs-4x32^3-mse"]
    return make_cohort(w, n=n, dims=dims, seed=seed).astype(np.float64)


# ------------------------------------------------------------- group objective


@pytest.mark.parametrize("metric", ["mse", "lncc", "l1"])
def test_group_loss_at_zero_displacement(metric):
    """Eq. (2) divided by n at u = 0: the mean over subjects of D(I_i, A)."""
    imgs = _cohort()
    rng = np.random.default_rng(5)
    A = rng.uniform(0.0, 1.0, size=imgs.shape[1:])
    p = O.SweepParams(metric=metric, win=5, lam=0.7)
    F = O.group_loss(imgs, np.zeros((len(imgs), 3) + imgs.shape[1:]), A, p)
    if metric == "mse":
        ref = np.mean([((I - A) ** 2).mean() for I in imgs])
    elif metric == "l1":
        ref = np.mean([np.abs(I - A).mean() for I in imgs])
    else:
        ref = np.mean([_lncc_by_hand(I, A, 5, p.ncc_eps) for I in imgs])
    assert F == pytest.approx(ref, rel=1e-12, abs=1e-15)


def test_group_loss_with_affine_displacements_closed_form():
    """Affine images under contracting affine displacements: the warped image
    is affine in closed form (trilinear interpolation reproduces affine
    functions and every sample stays inside the volume), and the diffusion
    regulariser of u = B (x - c) is ||B||_F^2 / 9."""
    dims = (9, 10, 8)
    rng = np.random.default_rng(6)
    x = O.identity_grid(dims)
    c = (np.asarray(dims, np.float64) - 1.0) / 2.0
    n, lam = 3, 0.4
    imgs, us, refs = [], [], []
    A = rng.uniform(0.0, 1.0, size=dims)
    for i in range(n):
        a = rng.normal(size=3)
        b0 = rng.normal()
        B = -0.1 * np.eye(3) + 0.03 * rng.normal(size=(3, 3))
        u = np.einsum("cd,d...->c...", B, x - c[:, None, None, None])
        p = x + u
        assert p.min() > 0.0 and all(p[d].max() < dims[d] - 1 for d in range(3))
        imgs.append(np.tensordot(a, x, axes=1) + b0)
        us.append(u)
        warped = np.tensordot(a, p, axes=1) + b0
        refs.append(((warped - A) ** 2).mean() + lam * (B ** 2).sum() / 9.0)
    F = O.group_loss(np.stack(imgs), np.stack(us), A, O.SweepParams(metric="mse", lam=lam))
    assert F == pytest.approx(np.mean(refs), rel=1e-12)


@pytest.mark.parametrize("metric", ["mse", "lncc"])
def test_sweep_reports_the_objective_at_the_new_atlas(metric):
    """The sweep's F is Eq. (2) / n at the centred displacements and the
    updated atlas A^{k+1}, regulariser included; the old atlas or a dropped
    regulariser gives a different value."""
    imgs = _cohort(n=3, dims=(10, 9, 11))
    n = len(imgs)
    z = np.zeros((n, 3) + imgs.shape[1:])
    p = O.SweepParams(metric=metric, win=5, lam=0.5, k2=2)
    A0 = O.initial_atlas(imgs)
    out = O.sweep(imgs, z, z, z, 0, A0, p)
    uh, A1 = out["u_hat"], out["atlas"]
    assert np.abs(uh.sum(axis=0)).max() < 1e-13

    def hand(atlas, lam):
        tot = 0.0
        for i in range(n):
            w = _warp_scipy(imgs[i], uh[i])
            if metric == "mse":
                d = ((w - atlas) ** 2).mean()
            else:
                d = _lncc_by_hand(w, atlas, 5, p.ncc_eps)
            tot += d + lam * _diffusion_by_hand(uh[i])
        return tot / n

    F = out["group_loss"]
    assert F == pytest.approx(hand(A1, p.lam), rel=1e-11)
    assert abs(F - hand(A0, p.lam)) > 1e-6 * abs(F)
    assert abs(F - hand(A1, 0.0)) > 1e-6 * abs(F)


# ---------------------------------------------------------------- level start


def test_level_start_at_zero_velocity_gives_the_unwarped_atlases():
    """v = 0: the mean (MSE), the median (L1) and, for the stochastic update,
    the minibatch descent from the mean of the unwarped subjects."""
    imgs = _cohort(n=4, dims=(8, 9, 10))
    v = np.zeros((4, 3) + imgs.shape[1:])
    v_out, A = O.level_start(imgs, v, O.SweepParams(metric="mse"))
    assert np.array_equal(v_out, v)
    assert np.abs(A - imgs.mean(axis=0)).max() < 1e-15
    _, A = O.level_start(imgs, v, O.SweepParams(metric="l1"))
    srt = np.sort(imgs, axis=0)
    assert np.abs(A - 0.5 * (srt[1] + srt[2])).max() < 1e-15
    p = O.SweepParams(metric="lncc", win=3, atlas_mode="sgd", k3=2, atlas_batch=2)
    _, A = O.level_start(imgs, v, p)
    ref, _ = O.atlas_sgd(imgs, imgs.mean(axis=0), 2, 2, win=3)
    assert np.abs(A - ref).max() < 1e-14


@pytest.mark.parametrize("center_mode", ["displacement", "velocity"])
def test_level_start_with_integer_translations(center_mode):
    """Constant integer velocities are exact translations; after centring,
    subject i moves by c_i - mean_j c_j and the atlas is the mean of the
    shifted subjects with zero fill, built here by slicing."""
    imgs = _cohort(n=2, dims=(9, 8, 10))
    shifts = np.array([[1, 0, -2], [3, 2, 0]], dtype=np.float64)
    v = np.stack([np.broadcast_to(s[:, None, None, None], (3,) + imgs.shape[1:])
                  for s in shifts]).copy()
    _, A = O.level_start(imgs, v, O.SweepParams(metric="mse", center_mode=center_mode))
    centred = (shifts - shifts.mean(axis=0)).astype(int)
    ref = np.zeros(imgs.shape[1:])
    for i, s in enumerate(centred):
        shifted = np.zeros(imgs.shape[1:])
        src = tuple(slice(max(0, k), min(D, D + k)) for k, D in zip(s, imgs.shape[1:]))
        dst = tuple(slice(max(0, -k), min(D, D - k)) for k, D in zip(s, imgs.shape[1:]))
        shifted[dst] = imgs[i][src]          # shifted(x) = I(x + s)
        ref += shifted / len(imgs)
    assert np.abs(A - ref).max() < 1e-14


def test_two_level_pyramid_is_the_explicit_composition():
    """down2 -> sweeps from v = 0 and A^0 -> up2(v, 2) -> level start ->
    sweeps with fresh moments, spelt out step by step."""
    imgs = _cohort(n=2, dims=(8, 8, 12))
    p = O.SweepParams(metric="mse", lam=0.02, k2=2)
    got = O.pyramid(imgs, 2, [2, 1], p)

    coarse = imgs.reshape(2, 4, 2, 4, 2, 6, 2).mean(axis=(2, 4, 6))
    z = np.zeros((2, 3) + coarse.shape[1:])
    st = dict(v=z, m=z, s=z, step=0, atlas=coarse.mean(axis=0))
    for _ in range(2):
        st = O.sweep(coarse, st["v"], st["m"], st["s"], st["step"], st["atlas"], p)
    vf = np.stack([O.up2(st["v"][i], 2.0) for i in range(2)])
    vf, A = O.level_start(imgs, vf, p)
    zf = np.zeros_like(vf)
    ref = O.sweep(imgs, vf, zf, zf, 0, A, p)
    for key in ("v", "m", "s", "atlas", "u_hat", "inner_losses"):
        assert np.array_equal(got[key], ref[key]), key
    assert got["group_loss"] == ref["group_loss"]
    assert got["step"] == p.k2


def test_up2_carries_a_constant_coarse_velocity_as_twice_the_constant():
    """A coarse voxel is two fine voxels: a constant coarse displacement c is
    2c at the finer level, exactly (border sampling keeps constants)."""
    c = np.array([0.3, -1.25, 0.5])
    f = np.broadcast_to(c[:, None, None, None], (3, 4, 5, 3)).copy()
    up = O.up2(f, 2.0)
    assert up.shape == (3, 8, 10, 6)
    assert np.abs(up - 2.0 * c[:, None, None, None]).max() == 0.0


# ------------------------------------------------------- restart of velocities


def test_reinit_v_sweep_equals_a_sweep_from_the_zero_state():
    """Algorithm 1's literal ``v = initialize()`` inside the per-subject
    registration: from any state, the sweep equals one from v = m = s = 0 and
    step 0."""
    imgs = _cohort(n=3, dims=(8, 10, 9))
    shape = (3, 3) + imgs.shape[1:]
    rng = np.random.default_rng(8)
    v = random_velocity(9, 3, imgs.shape[1:], 1.5).astype(np.float64)
    m = rng.normal(size=shape) * 1e-2
    s = rng.uniform(0.0, 1e-3, size=shape)
    A = O.initial_atlas(imgs) + 0.01
    p = O.SweepParams(metric="mse", lam=0.05, k2=2, reinit_v=True)
    got = O.sweep(imgs, v, m, s, 17, A, p)
    z = np.zeros(shape)
    ref = O.sweep(imgs, z, z, z, 0, A, O.SweepParams(metric="mse", lam=0.05, k2=2))
    for key in ("v", "m", "s", "atlas", "u_hat", "inner_losses"):
        assert np.array_equal(got[key], ref[key]), key
    assert got["step"] == ref["step"] == 2
    # the restart matters: without it the same state gives another sweep
    keep = O.sweep(imgs, v, m, s, 17, A, O.SweepParams(metric="mse", lam=0.05, k2=2))
    assert not np.allclose(keep["v"], ref["v"])


# ------------------------------------------------------ stochastic atlas start


def test_sgd_atlas_literal_initialisation():
    """``sgd_init = "initial"``: the stochastic update restarts from A^0 (the
    mean of the unwarped subjects), so the atlas passed in does not matter;
    ``"warm"`` starts from it."""
    imgs = _cohort(n=3, dims=(8, 8, 9))
    uh = O.center(random_velocity(3, 3, imgs.shape[1:], 1.0).astype(np.float64))[0]
    warped = np.stack([_warp_scipy(imgs[i], uh[i]) for i in range(3)])
    p = O.SweepParams(metric="lncc", win=3, atlas_mode="sgd", k3=2, atlas_batch=2,
                      sgd_init="initial")
    A_a = O.atlas_update(imgs, uh, np.zeros(imgs.shape[1:]), p)
    A_b = O.atlas_update(imgs, uh, np.ones(imgs.shape[1:]), p)
    assert np.array_equal(A_a, A_b)
    ref, _ = O.atlas_sgd(warped, imgs.mean(axis=0), 2, 2, win=3)
    assert np.abs(A_a - ref).max() < 1e-13
    pw = O.SweepParams(metric="lncc", win=3, atlas_mode="sgd", k3=2, atlas_batch=2)
    start = 0.8 * imgs[0] + 0.1      # a non-constant start (a constant one has zero variance)
    ref_w, _ = O.atlas_sgd(warped, start, 2, 2, win=3)
    assert np.abs(O.atlas_update(imgs, uh, start, pw) - ref_w).max() < 1e-13


# ------------------------------------------------------- Jacobian determinant


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_jacobian_det_of_an_affine_field(seed):
    """u = B x + b: det(I + grad u) = det(I + B) at every voxel (central and
    one-sided differences are exact on linear functions); a folding B gives a
    negative determinant."""
    rng = np.random.default_rng(seed)
    dims = (6, 7, 5)
    x = O.identity_grid(dims)
    B = 0.4 * rng.normal(size=(3, 3))
    if seed == 2:
        B = np.diag([-1.6, 0.2, 0.1]) + 0.05 * rng.normal(size=(3, 3))
    b = rng.normal(size=3)
    u = np.einsum("cd,d...->c...", B, x) + b[:, None, None, None]
    det = O.jacobian_det(u)
    ref = np.linalg.det(np.eye(3) + B)
    assert np.abs(det - ref).max() < 1e-12 * max(1.0, abs(ref))
    if seed == 2:
        assert ref < 0 and (det < 0).all()


# --------------------------------------------- the squaring adjoint at v = 0


def test_exp_adjoint_at_zero_velocity_is_the_identity():
    """At v = 0 every u_t is 0: the position derivative vanishes and each
    sample sits on its own voxel with weight 1 (the last voxel of an axis at
    fraction 1 of the last cell), so each adjoint step doubles g and
    dL/dv = 2^N g / 2^N = dL/du exactly."""
    rng = np.random.default_rng(12)
    dims = (5, 7, 6)
    g = rng.normal(size=(3,) + dims)
    _, steps = O.exp_svf(np.zeros((3,) + dims), 7)
    assert np.array_equal(O.exp_svf_bwd(steps, g), g)
