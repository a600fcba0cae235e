"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Inputs are seeded FP32 arrays from ``synthetic``; the oracle receives the
same values promoted to FP64.  Volumes are sized to span several 32 x 8
tiles with ragged tails on every axis.  Tolerances (derived from FP32
storage of fields and images between kernels):
  warped intensities / fields / atlas: rel-Linf <= 1e-5
  gradients and optimiser state: rel-L2 <= 1e-4
  losses: rel <= 1e-6
"""

import numpy as np
import pytest
import torch

from oracle import darc_oracle as O
from paper_2508_10743_amd import darc as D
from paper_2508_10743_amd._lib import DarcError
from synthetic.cohorts import WORKLOADS, make_cohort, random_velocity, random_volume

pytestmark = pytest.mark.gpu

TOL_WARP = 1e-5
TOL_GRAD = 1e-4
TOL_LOSS = 1e-6

DIMS = (19, 21, 70)  # 3 tiles along d2 (32-wide), 3 along d1 (8-high), all ragged


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    D.lib()
    return torch.device("cuda", 0)


@pytest.fixture(autouse=True, params=["march", "planes"])
def squaring_shape(request, dev):
    """Every test of this module runs with the marching squaring kernels and
    with the plane-parallel ones (one plane of a tile per block, the tiled
    adjoint for every subject)."""
    D.set_launch_shape("squaring", None, 0, 1 if request.param == "march" else -1)
    yield request.param
    D.autotune_clear()


def g(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def h(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_linf(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def rel_l2(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def blobs(n, dims, seed):
    return make_cohort(WORKLOADS["blobs-4x32^3-mse"], n=n, dims=dims, seed=seed)


# ------------------------------------------------------------------- Exp


@pytest.mark.parametrize("n_sq", [7, 1, 2, 0])
def test_exp_svf_and_checkpoints(dev, n_sq):
    v = random_velocity(101, 2, DIMS, 3.0, corr_len=3.0)
    u, ck = D.exp_svf(g(v, dev), n_sq)
    u = h(u)
    ck = None if ck is None else h(ck)
    for i in range(2):
        ref, steps = O.exp_svf(v[i].astype(np.float64), n_sq)
        assert rel_linf(u[i], ref) <= TOL_WARP
        if ck is not None:
            for t in range(1, n_sq):
                assert rel_linf(ck[t - 1, i], steps[t]) <= TOL_WARP


def test_exp_without_checkpoints_matches(dev):
    v = g(random_velocity(102, 2, DIMS, 3.0), dev)
    u1, _ = D.exp_svf(v, 7, checkpoints=True)
    u2, _ = D.exp_svf(v, 7, checkpoints=False)
    assert torch.equal(u1, u2)


def test_exp_constant_velocity_is_exact_translation(dev):
    c = np.array([1.75, -2.5, 0.375], np.float32)
    v = np.broadcast_to(c[None, :, None, None, None], (1, 3) + DIMS).copy()
    u, _ = D.exp_svf(g(v, dev), 7)
    assert np.array_equal(h(u), v)


def test_exp_zero_is_identity_and_minimum_dims(dev):
    v = np.zeros((1, 3, 2, 2, 2), np.float32)
    u, _ = D.exp_svf(g(v, dev), 7)
    assert not h(u).any()
    v = random_velocity(103, 1, (2, 3, 2), 0.7, corr_len=1.0)
    u, _ = D.exp_svf(g(v, dev), 7)
    assert rel_linf(h(u)[0], O.exp_svf(v[0].astype(np.float64))[0]) <= TOL_WARP


@pytest.mark.parametrize("n_sq", [7, 2, 1])
def test_exp_svf_bwd(dev, n_sq):
    v = random_velocity(104, 2, DIMS, 3.0, corr_len=3.0)
    gu = random_volume(105, v.shape, -1.0, 1.0)
    vd = g(v, dev)
    _, ck = D.exp_svf(vd, n_sq)
    gv = h(D.exp_svf_bwd(vd, ck, g(gu, dev), n_sq))
    for i in range(2):
        _, steps = O.exp_svf(v[i].astype(np.float64), n_sq)
        assert rel_l2(gv[i], O.exp_svf_bwd(steps, gu[i].astype(np.float64))) <= TOL_GRAD


@pytest.mark.parametrize("dims,amp,corr", [((20, 30, 70), 12.0, 6.0), ((11, 9, 40), 40.0, 2.0),
                                            ((40, 26, 33), 6.0, 3.0)])
def test_exp_large_displacements(dev, dims, amp, corr):
    """Displacements reaching across several 32 x 8 x 8 tiles, and (amp 40 on
    a small volume) positions clamped at the border.

    The adjoint is always compared with the oracle's adjoint of the squaring
    steps the GPU computed (its checkpoints).  Where Exp(v) is a
    diffeomorphism it is also compared end to end; the amp-40 field folds
    (det J down to about -700, |grad u| about 26), and there the FP32 rounding
    of the forward steps moves sample points across cell faces, which the
    gradient of a piecewise-linear interpolant cannot be stable against.
    """
    v = random_velocity(130, 2, dims, amp, corr_len=corr)
    gu = random_volume(131, v.shape, -1.0, 1.0)
    vd = g(v, dev)
    u, ck = D.exp_svf(vd, 7)
    gv = h(D.exp_svf_bwd(vd, ck, g(gu, dev), 7))
    u, ck = h(u), h(ck)
    for i in range(2):
        ref, steps = O.exp_svf(v[i].astype(np.float64))
        assert rel_linf(u[i], ref) <= TOL_WARP
        own = [v[i].astype(np.float64) / 2 ** 7] + [ck[t, i].astype(np.float64) for t in range(6)]
        assert rel_l2(gv[i], O.exp_svf_bwd(own, gu[i].astype(np.float64))) <= TOL_GRAD
        if O.jacobian_det(ref).min() > 0:
            assert rel_l2(gv[i], O.exp_svf_bwd(steps, gu[i].astype(np.float64))) <= TOL_GRAD


@pytest.mark.parametrize("dims,amp", [((20, 21, 70), 0.3), ((9, 17, 33), 0.8)])
def test_exp_small_displacements(dev, dims, amp):
    """Every cell offset in [-1, 0] (the marching adjoint's case)."""
    v = random_velocity(140, 2, dims, amp, corr_len=3.0)
    gu = random_volume(141, v.shape, -1.0, 1.0)
    vd = g(v, dev)
    u, ck = D.exp_svf(vd, 7)
    gv = h(D.exp_svf_bwd(vd, ck, g(gu, dev), 7))
    u = h(u)
    for i in range(2):
        ref, steps = O.exp_svf(v[i].astype(np.float64))
        assert rel_linf(u[i], ref) <= TOL_WARP
        assert rel_l2(gv[i], O.exp_svf_bwd(steps, gu[i].astype(np.float64))) <= TOL_GRAD


def cell_offsets(u):
    """Per axis, the border cell of x + u (floor clamped to [0, D - 2]) minus x."""
    dims = u.shape[1:]
    out = []
    for d in range(3):
        x = np.arange(dims[d]).reshape([-1 if k == d else 1 for k in range(3)])
        out.append(np.clip(np.floor(x + u[d]), 0, dims[d] - 2) - x)
    return out


@pytest.mark.parametrize("dims,amp,corr", [((24, 20, 70), 3.5, 4.0), ((13, 37, 41), 3.0, 3.0)])
def test_exp_adjoint_reach_two(dev, dims, amp, corr):
    """Squaring steps whose cell offsets span [-2, 1] on some axis, the case of
    the reach-2 marching adjoint (the others run on the reach-1 marching or
    the tiled kernel): the adjoint against the oracle's adjoint of the GPU's
    own squaring steps, and at least one step of the case is checked to be in
    that regime."""
    v = random_velocity(150, 2, dims, amp, corr_len=corr)
    gu = random_volume(151, v.shape, -1.0, 1.0)
    vd = g(v, dev)
    u, ck = D.exp_svf(vd, 7)
    gv = h(D.exp_svf_bwd(vd, ck, g(gu, dev), 7))
    ck = h(ck)
    reach2 = 0
    for i in range(2):
        own = [v[i].astype(np.float64) / 2 ** 7] + [ck[t, i].astype(np.float64) for t in range(6)]
        for ut in own:
            offs = cell_offsets(ut)
            lo, hi = min(o.min() for o in offs), max(o.max() for o in offs)
            reach2 += int(lo >= -2 and hi <= 1 and (lo < -1 or hi > 0))
        assert rel_l2(gv[i], O.exp_svf_bwd(own, gu[i].astype(np.float64))) <= TOL_GRAD
    assert reach2 >= 1


def test_exp_adjoint_mixed_reach_in_one_launch(dev):
    """Three subjects in one launch whose last squaring step has reach 1, 2
    and beyond 2: each step runs the three adjoint kernels side by side, each
    taking its own subjects (chosen on the device from the recorded reach)."""
    dims = (22, 19, 45)
    v = np.concatenate([random_velocity(160 + k, 1, dims, amp, corr_len=4.0)
                        for k, amp in enumerate((0.6, 3.5, 10.0))])
    gu = random_volume(163, v.shape, -1.0, 1.0)
    vd = g(v, dev)
    u, ck = D.exp_svf(vd, 7)
    gv = h(D.exp_svf_bwd(vd, ck, g(gu, dev), 7))
    ck = h(ck)
    reaches = []
    for i in range(3):
        own = [v[i].astype(np.float64) / 2 ** 7] + [ck[t, i].astype(np.float64) for t in range(6)]
        offs = cell_offsets(own[-1])
        lo, hi = min(o.min() for o in offs), max(o.max() for o in offs)
        reaches.append(int(max(-lo, hi + 1)))
        assert rel_l2(gv[i], O.exp_svf_bwd(own, gu[i].astype(np.float64))) <= TOL_GRAD
    assert reaches[0] == 1 and reaches[1] == 2 and reaches[2] > 2, reaches


# ------------------------------------------------------------------- warp


def test_warp_and_adjoint(dev):
    imgs = blobs(2, DIMS, 106)
    u = random_velocity(107, 2, DIMS, 4.0, corr_len=3.0)
    gout = random_volume(108, imgs.shape, -1.0, 1.0)
    gu0 = random_volume(109, u.shape, -1.0, 1.0)
    w = h(D.warp3d(g(imgs, dev), g(u, dev)))
    gu = h(D.warp3d_bwd(g(imgs, dev), g(u, dev), g(gout, dev), g(gu0, dev)))
    for i in range(2):
        assert rel_linf(w[i], O.warp3d(imgs[i], u[i])) <= TOL_WARP
        ref = gu0[i] + O.warp3d_bwd(imgs[i], u[i], gout[i])
        assert rel_l2(gu[i], ref) <= TOL_GRAD


def test_warp_far_outside_is_zero(dev):
    imgs = blobs(1, DIMS, 110)
    u = np.full((1, 3) + DIMS, 500.0, np.float32)
    u[0, 1] = np.nan  # non-finite displacements sample outside, never fault
    assert not h(D.warp3d(g(imgs, dev), g(u, dev))).any()


def test_warp_integer_translation(dev):
    imgs = blobs(1, DIMS, 111)
    s = np.array([2, -1, 3], np.float32)
    u = np.broadcast_to(s[None, :, None, None, None], (1, 3) + DIMS).copy()
    assert np.array_equal(h(D.warp3d(g(imgs, dev), g(u, dev)))[0],
                          O.warp3d(imgs[0], u[0]).astype(np.float32))


# ---------------------------------------------------------- dissimilarity


@pytest.mark.parametrize("metric,win", [("mse", 9), ("lncc", 3), ("lncc", 5), ("lncc", 7),
                                        ("lncc", 9), ("lncc", 11)])
def test_sim_grad(dev, metric, win):
    imgs = blobs(3, DIMS, 112)
    atlas = blobs(1, DIMS, 113)[0]
    loss, gw = D.sim_grad(g(imgs, dev), g(atlas, dev), metric, win, 1e-5)
    loss, gw = h(loss), h(gw)
    for i in range(3):
        rl, rg = O.dissimilarity(imgs[i], atlas, O.SweepParams(metric=metric, win=win))
        assert abs(loss[i] - rl) <= TOL_LOSS * abs(rl)
        assert rel_l2(gw[i], rg) <= TOL_GRAD


def test_sim_identical_images(dev):
    imgs = blobs(2, DIMS, 114)
    loss, gw = D.sim_grad(g(imgs, dev), g(imgs[0], dev), "mse")
    loss, gw = h(loss), h(gw)
    assert loss[0] == 0.0 and not gw[0].any()
    loss_n, _ = D.sim_grad(g(imgs[:1], dev), g(imgs[0], dev), "lncc", 9)
    ref, _ = O.lncc(imgs[0], imgs[0], 9)
    assert abs(h(loss_n)[0] - ref) <= TOL_LOSS * abs(ref)


# -------------------------------------------------------------- smoothing


@pytest.mark.parametrize("sigma", [0.5, 1.5, 2.5])
@pytest.mark.parametrize("dims", [DIMS, (11, 70, 45), (5, 33, 3)], ids=["base", "tall", "thin"])
def test_gauss_smooth(dev, sigma, dims):
    """The smoother's blocks own 32 x 32 tiles of a plane: the extra shapes
    give several tiles along d1 with a ragged tail, and a plane narrower
    than the radius."""
    x = random_volume(115, (2, 3) + dims, -1.0, 1.0)
    out = h(D.gauss_smooth(g(x, dev), sigma))
    for i in range(2):
        assert rel_linf(out[i], O.gauss_smooth(x[i], sigma)) <= TOL_WARP


def _guarded(n_elem, dtype, dev, guard=4096, sentinel=7.25):
    """A buffer of n_elem elements between two guard bands holding a sentinel."""
    buf = torch.full((guard + n_elem + guard,), sentinel, dtype=dtype, device=dev)
    return buf, buf[guard:guard + n_elem], guard


def _guards_intact(buf, guard, sentinel=7.25):
    b = h(buf)
    return bool((b[:guard] == sentinel).all() and (b[-guard:] == sentinel).all())


@pytest.mark.parametrize("win", [3, 9, 11])
def test_range_checked_stores_stay_in_their_arrays(dev, win):
    """The smoother and the LNCC statistics write through buffer stores whose
    masked lanes are dropped by the range check: with the output arrays (and
    the workspace holding the factor fields) placed between guard bands, the
    guards keep their sentinel and the outputs equal those of ordinary
    allocations bit for bit.  Ragged shapes give lanes outside the volume in
    every tile, chunks whose plane count is not a multiple of the window, and
    padding planes."""
    dims = (11, 70, 45)
    n, V = 2, 11 * 70 * 45
    x = g(random_volume(171, (n, 3) + dims, -1.0, 1.0), dev)
    ref = D.gauss_smooth(x, 1.5)
    buf, out, guard = _guarded(n * 3 * V, torch.float32, dev)
    D._call("darc_smooth3d", D._p(x), D._p(out), n, 3, *dims, D.L.DARC_GAUSS, 1.5, None, None, 0,
            D._stream())
    assert _guards_intact(buf, guard)
    assert torch.equal(out.view(ref.shape), ref)

    imgs, atlas = g(blobs(n, dims, 172), dev), g(blobs(1, dims, 173)[0], dev)
    loss_ref, gw_ref = D.sim_grad(imgs, atlas, "lncc", win, 1e-5)
    m = D.METRICS["lncc"]
    ws_bytes = D.lib().darc_sim_grad_ws_bytes(m, n, *dims)
    wbuf, ws, wguard = _guarded(ws_bytes, torch.uint8, dev, sentinel=0x5A)
    gbuf, gw, gguard = _guarded(n * V, torch.float32, dev)
    loss = torch.zeros(n, dtype=torch.float64, device=dev)
    D._call("darc_sim_grad", D._p(imgs), D._p(atlas), m, win, 1e-5, D._p(loss), D._p(gw), n,
            *dims, D._p(ws), ws_bytes, D._stream())
    assert _guards_intact(wbuf, wguard, sentinel=0x5A)
    assert _guards_intact(gbuf, gguard)
    assert torch.equal(gw.view(gw_ref.shape), gw_ref)
    # the loss is summed by FP64 atomics, in an order that varies by run
    assert torch.allclose(loss, loss_ref, rtol=1e-12, atol=0.0)


def test_diffusion_regulariser(dev):
    x = random_volume(116, (2, 3) + DIMS, -1.0, 1.0)
    out, loss = D.diffusion(g(x, dev), 0.3)
    out, loss = h(out), h(loss)
    for i in range(2):
        R, gR = O.diffusion_reg(x[i])
        assert abs(loss[i] - 0.3 * R) <= TOL_LOSS * 0.3 * R
        assert rel_l2(out[i], 0.3 * gR) <= TOL_GRAD


# ------------------------------------------------- Adam, centring, atlas


def test_adam_step(dev):
    shape = (2, 3) + DIMS
    v, m = random_volume(117, shape, -1, 1), random_volume(118, shape, -0.1, 0.1)
    s, gr = random_volume(119, shape, 0.0, 0.01), random_volume(120, shape, -1, 1)
    rv, rm, rs = O.adam_step(v, m, s, gr, 4)
    vd, md, sd = g(v, dev), g(m, dev), g(s, dev)
    D.adam_step(vd, md, sd, g(gr, dev), 4)
    assert rel_linf(h(vd), rv) <= 1e-6
    assert rel_linf(h(md), rm) <= 1e-6
    assert rel_linf(h(sd), rs) <= 1e-6


@pytest.mark.parametrize("offset", [0, 1, 3])
def test_adam_step_alignment_and_tail(dev, offset):
    """The Adam step on arrays at any element offset (not 16-byte aligned)
    and of odd length; elements outside the given range stay untouched."""
    n = 4099
    v, m = random_volume(131, (n + 3,), -1, 1), random_volume(132, (n + 3,), -0.1, 0.1)
    s, gr = random_volume(133, (n + 3,), 0.0, 0.01), random_volume(134, (n + 3,), -1, 1)
    sl = slice(offset, offset + n)
    rv, rm, rs = O.adam_step(v[sl], m[sl], s[sl], gr[sl], 3)
    vd, md, sd, gd = g(v, dev), g(m, dev), g(s, dev), g(gr, dev)
    D.adam_step(vd[sl], md[sl], sd[sl], gd[sl], 3)
    assert rel_linf(h(vd)[sl], rv) <= 1e-6
    assert rel_linf(h(md)[sl], rm) <= 1e-6
    assert rel_linf(h(sd)[sl], rs) <= 1e-6
    # elements outside the slice are untouched
    assert np.array_equal(h(vd)[:offset], v[:offset]) and np.array_equal(h(vd)[offset + n:], v[offset + n:])


def test_center_and_atlas(dev):
    u = random_velocity(121, 5, DIMS, 2.0)
    ud = g(u, dev)
    mean = h(D.center(ud))
    uh, rmean = O.center(u)
    assert rel_linf(h(ud), uh) <= 1e-6 and rel_linf(mean, rmean) <= 1e-6
    # centrality holds up to FP32 rounding of each centred field
    assert np.abs(h(ud).astype(np.float64).sum(0)).max() <= 5 * 5 * np.abs(u).max() * 2 ** -24
    imgs = blobs(5, DIMS, 122)
    A = h(D.atlas_update(g(imgs, dev), g(u, dev)))
    assert rel_linf(A, O.atlas_mean(imgs, u)) <= TOL_WARP
    A2 = h(D.atlas_update(g(imgs, dev), g(u, dev), g(rmean.astype(np.float32), dev)))
    ref = O.atlas_mean(imgs, u.astype(np.float64) - rmean.astype(np.float32)[None])
    assert rel_linf(A2, ref) <= TOL_WARP


@pytest.mark.parametrize("n", [1, 16, 17])
def test_center_register_and_loop_paths(dev, n):
    """Centring holds up to 16 subjects in registers between the mean and the
    update and loops over larger cohorts: both sides of that boundary, and
    one subject (its mean is the field itself, so the centred field is
    exactly zero), against the oracle."""
    dims = (5, 9, 33)
    u = random_velocity(123 + n, n, dims, 2.0)
    ud = g(u, dev)
    mean = h(D.center(ud))
    uh, rmean = O.center(u)
    assert rel_linf(mean, rmean) <= 1e-6
    if n == 1:
        assert np.array_equal(mean, u[0]) and not h(ud).any()
    else:
        assert rel_linf(h(ud), uh) <= 1e-6


# ------------------------------------------------------------------ errors


def test_errors_surface_as_exceptions(dev):
    v = g(random_velocity(123, 1, DIMS, 1.0), dev)
    with pytest.raises(DarcError):
        D.sim_grad(g(blobs(1, DIMS, 1), dev), g(blobs(1, DIMS, 2)[0], dev), "lncc", 13)
    with pytest.raises(ValueError):
        D.exp_svf(v.cpu(), 7)
    with pytest.raises(DarcError):
        D.gauss_smooth(v, 4.0)


# ------------------------------------------------------------------- sweeps


def _oracle_run(imgs, p, sweeps):
    n = len(imgs)
    shape = (n, 3) + imgs.shape[1:]
    v, m, s, step = np.zeros(shape), np.zeros(shape), np.zeros(shape), 0
    A = O.initial_atlas(imgs)
    out = []
    for _ in range(sweeps):
        r = O.sweep(imgs.astype(np.float64), v, m, s, step, A, p)
        v, m, s, step, A = r["v"], r["m"], r["s"], r["step"], r["atlas"]
        out.append(r)
    return out


def _check_run(imgs, p_o, p_d, sweeps, dev):
    ref = _oracle_run(imgs, p_o, sweeps)
    c = D.Cohort(g(imgs, dev), p_d)
    assert rel_linf(h(c.atlas), imgs.astype(np.float64).mean(0)) <= TOL_WARP
    for k in range(sweeps):
        losses = h(c.sweep())
        r = ref[k]
        inner = r["inner_losses"].ravel()
        assert np.abs(losses[:-1] - inner).max() <= TOL_LOSS * np.abs(inner).max()
        assert abs(losses[-1] - r["group_loss"]) <= TOL_LOSS * abs(r["group_loss"])
        assert rel_l2(h(c.v), r["v"]) <= TOL_GRAD
        assert rel_l2(h(c.u_hat), r["u_hat"]) <= TOL_GRAD
        assert rel_linf(h(c.atlas), r["atlas"]) <= TOL_WARP
        assert c.step == r["step"]


@pytest.mark.parametrize("metric,sigma,lam,center,batch", [
    ("mse", 0.0, 0.01, "displacement", 0),
    ("mse", 0.0, 0.01, "velocity", 2),
    ("lncc", 1.0, 0.0, "displacement", 1),
    ("lncc", 0.0, 0.01, "displacement", 0),
])
def test_sweep_matches_oracle(dev, metric, sigma, lam, center, batch):
    imgs = blobs(3, (12, 10, 40), 124)
    kw = dict(metric=metric, win=5, lam=lam, smooth_sigma=sigma, k2=2, center_mode=center)
    _check_run(imgs, O.SweepParams(**kw), D.SweepParams(batch=batch, **kw), 2, dev)


@pytest.mark.parametrize("k2,batch", [(3, 2), (1, 0)])
def test_smoothed_sweep_with_odd_inner_steps(dev, k2, batch):
    """Smoothing after each Adam step with an odd number of inner steps, with
    and without subject batching."""
    imgs = blobs(3, (12, 10, 40), 127)
    kw = dict(metric="mse", lam=0.01, smooth_sigma=1.0, k2=k2)
    _check_run(imgs, O.SweepParams(**kw), D.SweepParams(batch=batch, **kw), 2, dev)


@pytest.mark.parametrize("n_sq,amp", [(1, 3.0), (7, 2.5)], ids=["tiled-first-step", "marching"])
def test_smoothed_sweep_from_given_velocities(dev, n_sq, amp):
    """A smoothed sweep from nonzero velocities.  With one squaring step and
    |v| up to 3 voxels the adjoint's reach exceeds one voxel (the tiled
    adjoint); with seven it stays under one (the marching adjoint)."""
    dims = (12, 10, 40)
    imgs = blobs(3, dims, 128)
    v0 = random_velocity(129, 3, dims, amp, corr_len=3.0)
    kw = dict(metric="mse", lam=0.01, smooth_sigma=1.0, k2=2, n_sq=n_sq)
    z = np.zeros(v0.shape)
    r = O.sweep(imgs.astype(np.float64), v0.astype(np.float64), z, z, 0, O.initial_atlas(imgs),
                O.SweepParams(**kw))
    c = D.Cohort(g(imgs, dev), D.SweepParams(batch=2, **kw), v0=g(v0, dev))
    losses = h(c.sweep())
    inner = r["inner_losses"].ravel()
    assert np.abs(losses[:-1] - inner).max() <= TOL_LOSS * np.abs(inner).max()
    assert rel_l2(h(c.v), r["v"]) <= TOL_GRAD
    assert rel_l2(h(c.m), r["m"]) <= TOL_GRAD
    assert rel_l2(h(c.s), r["s"]) <= TOL_GRAD
    assert rel_linf(h(c.atlas), r["atlas"]) <= TOL_WARP


def test_blobs_4x32_mse_two_sweeps(dev):
    """The 4-subject 32^3 MSE workload (lambda 0.01, 7 squarings, K2 = 5)."""
    w = WORKLOADS["blobs-4x32^3-mse"]
    imgs = make_cohort(w)
    kw = dict(metric=w.metric, lam=w.lam, n_sq=w.n_sq, k2=w.k2)
    _check_run(imgs, O.SweepParams(**kw), D.SweepParams(**kw), 2, dev)


def test_batched_equals_per_subject(dev):
    """Subjects are uncoupled within a sweep: one launch per subject and one
    launch for all give the same state."""
    imgs = g(blobs(4, (16, 12, 36), 125), dev)
    a = D.Cohort(imgs, D.SweepParams(k2=3, batch=1))
    b = D.Cohort(imgs, D.SweepParams(k2=3, batch=0))
    for _ in range(2):
        la, lb = h(a.sweep()), h(b.sweep())
    assert np.abs(la - lb).max() <= TOL_LOSS * np.abs(lb).max()
    assert rel_l2(h(a.v), h(b.v)) <= 1e-5


def test_reinit_v_restarts_from_zero(dev):
    imgs = g(blobs(3, (12, 10, 40), 126), dev)
    a = D.Cohort(imgs, D.SweepParams(k2=2))
    a.sweep()
    b = D.Cohort(imgs, D.SweepParams(k2=2, reinit_v=True))
    b.atlas.copy_(a.atlas)
    b.v.fill_(3.0)
    lb = h(b.sweep())
    c = D.Cohort(imgs, D.SweepParams(k2=2))
    c.atlas.copy_(a.atlas)
    lc = h(c.sweep())
    assert np.abs(lb - lc).max() <= TOL_LOSS * np.abs(lc).max()
    assert b.step == 2
