"""Pins of the FP64 oracle against facts fixed outside the oracle itself.

Each test ties one oracle function to a closed form, a library special case,
a brute-force definition, an exact identity (adjoint, translation, constant
preservation) or finite differences, chosen so that a dropped term, a sign or
index slip, or a transposed operand fails.  CPU only.
"""

import numpy as np
import pytest
from scipy import ndimage
from scipy.linalg import expm

from oracle import darc_oracle as O
from synthetic.cohorts import WORKLOADS, make_cohort, random_velocity


def rel_l2(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _positions(rng, dims, n, lo=-1.5, hi_pad=1.5):
    return np.stack([rng.uniform(lo, d - 1 + hi_pad, size=n) for d in dims])


# --------------------------------------------------------------------- sampler


def test_sampler_integer_positions_reproduce_samples():
    rng = np.random.default_rng(0)
    img = rng.normal(size=(5, 6, 7))
    x = O.identity_grid(img.shape)
    val, _ = O.sample_zero(img, x)
    assert np.array_equal(val, img)
    f = rng.normal(size=(3, 5, 6, 7))
    vb, _ = O.sample_border(f, x)
    # the last index sits at fraction 1 of the last cell: a + 1*(b - a) == b up to rounding
    assert np.array_equal(vb[:, :-1, :-1, :-1], f[:, :-1, :-1, :-1])
    assert np.abs(vb - f).max() < 1e-14


def test_sampler_matches_scipy_map_coordinates():
    """Zero padding == mode 'grid-constant'; border clamping == mode 'nearest'."""
    rng = np.random.default_rng(1)
    img = rng.normal(size=(6, 7, 9))
    pos = _positions(rng, img.shape, 4000)
    val, _ = O.sample_zero(img, pos)
    ref = ndimage.map_coordinates(img, pos, order=1, mode="grid-constant", cval=0.0)
    assert np.abs(val - ref).max() < 1e-12
    f = rng.normal(size=(3,) + img.shape)
    vb, _ = O.sample_border(f, pos)
    for c in range(3):
        refb = ndimage.map_coordinates(f[c], pos, order=1, mode="nearest")
        assert np.abs(vb[c] - refb).max() < 1e-12


def test_sampler_reproduces_affine_and_its_gradient():
    rng = np.random.default_rng(2)
    dims = (7, 8, 9)
    a = rng.normal(size=3)
    b = rng.normal()
    x = O.identity_grid(dims)
    img = np.tensordot(a, x, axes=1) + b
    pos = np.stack([rng.uniform(0, d - 1, size=500) for d in dims])
    val, grad = O.sample_zero(img, pos)
    assert np.abs(val - (np.tensordot(a, pos, axes=1) + b)).max() < 1e-12
    assert np.abs(grad - a[:, None]).max() < 1e-12


def test_sampler_position_derivative_matches_central_differences():
    rng = np.random.default_rng(3)
    img = rng.normal(size=(6, 6, 6))
    f = rng.normal(size=(3, 6, 6, 6))
    pos = np.stack([rng.uniform(-0.8, 5.8, size=300) for _ in range(3)])
    # keep samples away from cell faces and the clamp boundaries
    frac = pos - np.floor(pos)
    keep = np.all((frac > 0.05) & (frac < 0.95), axis=0)
    pos = pos[:, keep]
    h = 1e-6
    _, grad = O.sample_zero(img, pos)
    _, jac = O.sample_border(f, pos)
    for d in range(3):
        e = np.zeros((3, 1))
        e[d] = h
        fd = (O.sample_zero(img, pos + e)[0] - O.sample_zero(img, pos - e)[0]) / (2 * h)
        assert np.abs(fd - grad[d]).max() < 1e-7
        fdb = (O.sample_border(f, pos + e)[0] - O.sample_border(f, pos - e)[0]) / (2 * h)
        assert np.abs(fdb - jac[:, d]).max() < 1e-7


def test_scatter_is_the_adjoint_of_border_sampling():
    rng = np.random.default_rng(4)
    dims = (5, 6, 7)
    f = rng.normal(size=(3,) + dims)
    pos = _positions(rng, dims, 700)
    g = rng.normal(size=(3, 700))
    lhs = float((O.sample_border(f, pos)[0] * g).sum())
    rhs = float((f * O.scatter_border(pos, g, dims)).sum())
    assert abs(lhs - rhs) < 1e-11 * max(1.0, abs(lhs))


# ------------------------------------------------------------------------- Exp


def test_exp_zero_velocity_is_identity():
    u, steps = O.exp_svf(np.zeros((3, 6, 7, 8)))
    assert np.array_equal(u, np.zeros_like(u)) and len(steps) == 7


def test_exp_constant_velocity_is_exact_translation():
    c = np.array([1.75, -2.5, 0.375])
    v = np.broadcast_to(c[:, None, None, None], (3, 6, 7, 8)).copy()
    u, _ = O.exp_svf(v)
    assert np.array_equal(u, v)


@pytest.mark.parametrize("n_sq", [3, 7])
def test_exp_affine_velocity_matches_matrix_power(n_sq):
    """Affine v: every sample is exact, so phi_N = (x -> M x)^(2^N)."""
    rng = np.random.default_rng(5)
    dims = (32, 32, 32)
    B = 0.04 * rng.normal(size=(3, 3))
    b = 0.2 * rng.normal(size=3)
    x0 = np.array([15.5, 15.5, 15.5])
    x = O.identity_grid(dims)
    v = np.einsum("cd,d...->c...", B, x - x0[:, None, None, None]) + b[:, None, None, None]
    u, _ = O.exp_svf(v, n_sq)
    M = np.eye(4)
    M[:3, :3] += B / 2 ** n_sq
    M[:3, 3] = (b - B @ x0) / 2 ** n_sq
    P = np.linalg.matrix_power(M, 2 ** n_sq)
    sl = (slice(None),) + (slice(10, 22),) * 3
    xi = x[sl].reshape(3, -1)
    ref = (P[:3, :3] - np.eye(3)) @ xi + P[:3, 3:4]
    assert np.abs(u[sl].reshape(3, -1) - ref).max() < 1e-12
    # as N grows the closed form tends to the matrix exponential of the generator
    G = np.zeros((4, 4))
    G[:3, :3] = B
    G[:3, 3] = b - B @ x0
    E = expm(G)
    ref_exp = (E[:3, :3] - np.eye(3)) @ xi + E[:3, 3:4]
    assert np.abs(ref - ref_exp).max() < 4.0 / 2 ** n_sq


def test_exp_of_minus_v_inverts_exp_of_v():
    """Exp(-v) is the inverse of Exp(v) (Section 4, one-shot segmentation)."""
    v = random_velocity(7, 1, (32, 32, 32), 3.0)[0].astype(np.float64)
    up, _ = O.exp_svf(v)
    um, _ = O.exp_svf(-v)
    x = O.identity_grid(v.shape[1:])
    # phi_+(phi_-(x)) - x = u_-(x) + u_+(x + u_-(x)), on the interior
    s, _ = O.sample_border(up, x + um)
    res = np.sqrt(((um + s) ** 2).sum(axis=0))[4:-4, 4:-4, 4:-4]
    # calibrated on seeded fields of max norm 3 voxels: the discrete inverse
    # error is ~1% of the displacement and grows with its square
    assert res.mean() < 0.03 and res.max() < 0.1


def test_exp_is_diffeomorphic_on_workload_fields():
    v = random_velocity(8, 2, (32, 32, 32), 3.0).astype(np.float64)
    for i in range(2):
        u, _ = O.exp_svf(v[i])
        assert O.jacobian_det(u).min() > 0.0


def _fd_dot(fun, x, direction, h=1e-6):
    return (fun(x + h * direction) - fun(x - h * direction)) / (2 * h)


def test_squaring_step_adjoint_matches_finite_differences():
    rng = np.random.default_rng(9)
    u = random_velocity(9, 1, (8, 8, 8), 1.2, corr_len=2.0)[0].astype(np.float64)
    g = rng.normal(size=u.shape)
    du = rng.normal(size=u.shape)
    lhs = float((O.squaring_step_bwd(u, g) * du).sum())
    fd = _fd_dot(lambda w: float((O.squaring_step(w) * g).sum()), u, du)
    assert abs(lhs - fd) < 1e-6 * abs(fd)


def test_pointwise_adjoint_equals_full_adjoint():
    """The per-voxel evaluation used for large volumes sums the same terms as
    the whole-volume adjoint (checked against it, including clamped borders)."""
    rng = np.random.default_rng(22)
    dims = (9, 11, 10)
    u = random_velocity(23, 1, dims, 4.0, corr_len=2.0)[0].astype(np.float64)
    g = rng.normal(size=u.shape)
    full = O.squaring_step_bwd(u, g)
    pts = np.stack([rng.integers(0, d, size=60) for d in dims])
    pts[:, :4] = [[0, 8, 0, 8], [0, 10, 10, 0], [0, 9, 0, 9]]  # corners
    at = O.squaring_step_bwd_at(u, g, pts)
    assert np.abs(at - full[:, pts[0], pts[1], pts[2]]).max() < 1e-12 * np.abs(full).max()


# ------------------------------------------------------------------------ warp


def test_warp_integer_translation_shifts_with_zero_fill():
    rng = np.random.default_rng(10)
    img = rng.normal(size=(6, 7, 8))
    s = np.array([2, -1, 3])
    u = np.broadcast_to(s[:, None, None, None].astype(np.float64), (3,) + img.shape)
    w = O.warp3d(img, u)
    ref = np.zeros_like(img)
    src = [slice(max(k, 0), d + min(k, 0)) for k, d in zip(s, img.shape)]
    dst = [slice(max(-k, 0), d + min(-k, 0)) for k, d in zip(s, img.shape)]
    ref[tuple(dst)] = img[tuple(src)]
    assert np.array_equal(w, ref)


def test_warp_backward_matches_finite_differences():
    rng = np.random.default_rng(11)
    img = rng.uniform(size=(8, 8, 8))
    u = random_velocity(11, 1, (8, 8, 8), 1.5, corr_len=2.0)[0].astype(np.float64)
    g = rng.normal(size=img.shape)
    du = rng.normal(size=u.shape)
    lhs = float((O.warp3d_bwd(img, u, g) * du).sum())
    fd = _fd_dot(lambda w: float((O.warp3d(img, w) * g).sum()), u, du)
    assert abs(lhs - fd) < 1e-6 * abs(fd)


# ------------------------------------------------------------ dissimilarities


def test_mse_closed_forms():
    rng = np.random.default_rng(12)
    A = rng.uniform(size=(5, 6, 7))
    loss, g = O.mse(A, A)
    assert loss == 0.0 and not g.any()
    loss, g = O.mse(A + 0.25, A)
    assert abs(loss - 0.0625) < 1e-15
    assert np.allclose(g, 2 * 0.25 / A.size, rtol=0, atol=1e-16)


def _brute_box(f, win):
    r = win // 2
    D0, D1, D2 = f.shape
    out = np.zeros_like(f)
    for i in range(D0):
        for j in range(D1):
            for k in range(D2):
                out[i, j, k] = f[max(i - r, 0):i + r + 1, max(j - r, 0):j + r + 1,
                                 max(k - r, 0):k + r + 1].sum()
    return out


@pytest.mark.parametrize("win", [3, 5, 9])
def test_box_sum_matches_brute_force_and_scipy(win):
    rng = np.random.default_rng(13)
    f = rng.normal(size=(6, 7, 8))
    b = O.box_sum(f, win)
    assert np.abs(b - _brute_box(f, win)).max() < 1e-12
    ref = ndimage.uniform_filter(f, size=win, mode="constant", cval=0.0) * win ** 3
    assert np.abs(b - ref).max() < 1e-11


def test_lncc_matches_brute_force_window_loops():
    rng = np.random.default_rng(14)
    I = rng.uniform(size=(6, 7, 6))
    J = rng.uniform(size=(6, 7, 6))
    win, eps = 5, 1e-5
    N = win ** 3
    r = win // 2
    cc = np.zeros(I.shape)
    for x in np.ndindex(I.shape):
        sl = tuple(slice(max(c - r, 0), c + r + 1) for c in x)
        a, b = I[sl].ravel(), J[sl].ravel()
        # zero padding: the missing entries are zeros in an N-sample window
        a = np.concatenate([a, np.zeros(N - a.size)])
        b = np.concatenate([b, np.zeros(N - b.size)])
        cross = ((a - a.mean()) * (b - b.mean())).sum()
        va = ((a - a.mean()) ** 2).sum()
        vb = ((b - b.mean()) ** 2).sum()
        cc[x] = cross ** 2 / (va * vb + eps)
    loss, _ = O.lncc(I, J, win, eps)
    assert abs(loss - (-cc.mean())) < 1e-12


def test_lncc_identical_and_constant_images():
    rng = np.random.default_rng(15)
    I = rng.uniform(size=(7, 7, 7))
    win, eps = 5, 1e-5
    loss, g = O.lncc(I, I, win, eps)
    S_I, S_II = O.box_sum(I, win), O.box_sum(I * I, win)
    var = S_II - S_I ** 2 / win ** 3
    assert abs(loss - (-(var ** 2 / (var ** 2 + eps)).mean())) < 1e-12
    # an all-zero warped image has S_I = S_II = S_IJ = 0, so cross = 0 in every
    # window (zero padding included): the loss and its gradient vanish
    loss_z, g_z = O.lncc(np.zeros(I.shape), I, win, eps)
    assert loss_z == 0.0 and not g_z.any()
    # with eps = 0 the squared NCC is invariant to scaling either image
    J = rng.uniform(size=I.shape)
    l1, _ = O.lncc(I, J, win, 0.0)
    l2, _ = O.lncc(3.5 * I, 0.25 * J, win, 0.0)
    assert abs(l1 - l2) < 1e-12
    # cc lies in [0, 1] (Cauchy-Schwarz on centred windows)
    assert -1.0 - 1e-12 <= l1 <= 0.0


@pytest.mark.parametrize("metric", ["mse", "lncc"])
def test_dissimilarity_gradient_matches_finite_differences(metric):
    rng = np.random.default_rng(16)
    I = rng.uniform(size=(7, 8, 6))
    J = rng.uniform(size=(7, 8, 6))
    p = O.SweepParams(metric=metric, win=5)
    _, g = O.dissimilarity(I, J, p)
    d = rng.normal(size=I.shape)
    fd = _fd_dot(lambda w: O.dissimilarity(w, J, p)[0], I, d)
    assert abs(float((g * d).sum()) - fd) < 1e-6 * abs(fd)


# ----------------------------------------------------------------- regulariser


def test_diffusion_reg_closed_forms():
    dims = (5, 6, 7)
    R, g = O.diffusion_reg(np.full((3,) + dims, 1.7))
    assert R == 0.0 and not g.any()
    A = np.arange(9.0).reshape(3, 3) / 7.0
    x = O.identity_grid(dims)
    u = np.einsum("cd,d...->c...", A, x)
    R, _ = O.diffusion_reg(u)
    assert abs(R - (A ** 2).sum() / 9.0) < 1e-13


def test_diffusion_reg_gradient_matches_finite_differences():
    rng = np.random.default_rng(17)
    u = rng.normal(size=(3, 5, 6, 4))
    d = rng.normal(size=u.shape)
    _, g = O.diffusion_reg(u)
    fd = _fd_dot(lambda w: O.diffusion_reg(w)[0], u, d)
    assert abs(float((g * d).sum()) - fd) < 1e-7 * abs(fd)


def test_gauss_smooth_matches_scipy_and_keeps_constants():
    rng = np.random.default_rng(18)
    f = rng.normal(size=(3, 9, 10, 11))
    out = O.gauss_smooth(f, 1.5)
    assert len(O.gaussian_weights(1.5)) == 11
    for c in range(3):
        ref = ndimage.gaussian_filter(f[c], 1.5, mode="nearest", truncate=3.0)
        assert np.abs(out[c] - ref).max() < 1e-13
    const = np.full((3, 6, 6, 6), 0.7)
    assert np.abs(O.gauss_smooth(const, 1.5) - 0.7).max() < 1e-15


# ------------------------------------------------------------ Adam, centring


def test_adam_first_step_moves_by_lr_times_sign():
    rng = np.random.default_rng(19)
    v = rng.normal(size=100)
    g = rng.normal(size=100)
    v1, m1, s1 = O.adam_step(v, np.zeros(100), np.zeros(100), g, 1, lr=1e-2, eps=1e-8)
    assert np.abs(v1 - (v - 1e-2 * g / (np.abs(g) + 1e-8))).max() < 1e-15
    assert np.allclose(m1, 0.1 * g, rtol=1e-15) and np.allclose(s1, 0.001 * g * g, rtol=1e-15)


def test_center_is_exactly_centred_and_idempotent():
    rng = np.random.default_rng(20)
    u = rng.normal(size=(5, 3, 4, 5, 6))
    uh, mean = O.center(u)
    assert np.abs(uh.sum(axis=0)).max() < 5 * 1e-15 * np.abs(u).max() * 5
    uh2, mean2 = O.center(uh)
    assert np.abs(uh2 - uh).max() < 1e-15 and np.abs(mean2).max() < 1e-15
    assert O.centrality_error(uh) < 1e-15


def test_atlas_is_the_mean_of_warped_subjects():
    rng = np.random.default_rng(21)
    img = rng.uniform(size=(6, 6, 6))
    images = np.stack([img] * 4)
    A = O.atlas_mean(images, np.zeros((4, 3, 6, 6, 6)))
    assert np.array_equal(A, img)
    # with deformations: the mean minimises sum_i ||I_i o phi_i - A||^2
    imgs = rng.uniform(size=(3, 6, 6, 6))
    uh = 0.5 * rng.normal(size=(3, 3, 6, 6, 6))
    A = O.atlas_mean(imgs, uh)
    grad_A = sum(-2 * (O.warp3d(imgs[i], uh[i]) - A) for i in range(3))
    assert np.abs(grad_A).max() < 1e-14


# ------------------------------------------------------ whole-chain gradients


@pytest.mark.parametrize("metric,lam", [("mse", 0.01), ("lncc", 0.01), ("lncc", 0.0)])
def test_subject_gradient_matches_finite_differences(metric, lam):
    """Whole chain v -> Exp -> warp -> dissimilarity + lam R on 8^3 volumes."""
    w = WORKLOADS["blobs-4x32^3-mse"]
    imgs = make_cohort(w, n=2, dims=(8, 8, 8), seed=33).astype(np.float64)
    v = random_velocity(34, 1, (8, 8, 8), 1.5, corr_len=2.0)[0].astype(np.float64)
    p = O.SweepParams(metric=metric, win=5, lam=lam)
    _, g = O.subject_loss_grad(imgs[0], v, imgs[1], p)
    d = np.random.default_rng(35).normal(size=v.shape)
    fd = _fd_dot(lambda x: O.subject_loss_grad(imgs[0], x, imgs[1], p)[0], v, d)
    assert abs(float((g * d).sum()) - fd) < 1e-6 * abs(fd)


# ----------------------------------------------------------------------- sweep


def _c1_state(n=4, dims=(16, 16, 16)):
    w = WORKLOADS["blobs-4x32^3-mse"]
    imgs = make_cohort(w, n=n, dims=dims, seed=40).astype(np.float64)
    z = np.zeros((n, 3) + dims)
    return imgs, z


def test_sweep_subject_order_does_not_matter():
    """Subjects are uncoupled within a sweep (Section 3, after Eq. (3))."""
    imgs, z = _c1_state()
    p = O.SweepParams(k2=2)
    A0 = O.initial_atlas(imgs)
    r1 = O.sweep(imgs, z, z, z, 0, A0, p)
    perm = [2, 0, 3, 1]
    r2 = O.sweep(imgs[perm], z, z, z, 0, A0, p)
    assert np.array_equal(r1["v"][perm], r2["v"])
    assert np.abs(r1["atlas"] - r2["atlas"]).max() < 1e-15


def test_sweep_centres_and_lowers_group_loss():
    imgs, z = _c1_state()
    p = O.SweepParams(k2=3)
    A = O.initial_atlas(imgs)
    F0 = O.group_loss(imgs, z, A, p)
    state = (z, z, z, 0, A)
    for _ in range(2):
        r = O.sweep(imgs, *state, p)
        state = (r["v"], r["m"], r["s"], r["step"], r["atlas"])
        assert np.abs(r["u_hat"].sum(axis=0)).max() < 1e-12
    assert r["group_loss"] < F0


def test_sweep_velocity_centring_mode():
    imgs, z = _c1_state()
    p = O.SweepParams(k2=2, center_mode="velocity")
    r = O.sweep(imgs, z, z, z, 0, O.initial_atlas(imgs), p)
    assert np.abs(r["v"].sum(axis=0)).max() < 1e-14
