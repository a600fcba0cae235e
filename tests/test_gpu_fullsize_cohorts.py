"""Parity at the full shapes of the two large cohorts, in their launch
configurations.

* 64 subjects of 128^3 (blobs, LNCC 9^3 plus the diffusion regulariser
  lambda = 0.01), all 64 in each launch;
* 200 subjects of 160 x 192 x 224 (compartments, LNCC 9^3, Gaussian sigma 1.5
  on v), 64 subjects per launch as the benchmark runs it, so the last batch
  of the sweep holds 8 subjects.

The oracle cannot afford these volumes step by step, so the checks are:
squaring steps, one adjoint step and the warp at sampled voxels of the first
and last subject of a 64-subject launch; sweeps of one or two inner steps from
v = 0, where the first inner loss is D(I_i, A^0) over the whole volume and the
first velocity gradient equals dL/du at u = 0 exactly (the adjoint of Exp is
the identity at v = 0), so the velocities after the first Adam step (and the
Gaussian) are checked over whole volumes; centrality over all subjects; and
the atlas at sampled voxels from the GPU's centred displacements.  Subjects
0, 63, 64 and 199 cover the batch offsets and the ragged last batch.
"""

import numpy as np
import pytest
import torch

from oracle import darc_oracle as O
from paper_2508_10743_amd import darc as D
from synthetic.cohorts import WORKLOADS, make_cohort, random_velocity, random_volume

pytestmark = pytest.mark.gpu

W3 = WORKLOADS["blobs-64x128^3-lncc9"]
W5 = WORKLOADS["compartments-200x160x192x224-lncc9"]
BATCH5 = 64
WORKERS = 16


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    D.lib()
    return torch.device("cuda", 0)


def samples(seed, dims, k=3000):
    rng = np.random.default_rng(seed)
    pts = np.stack([rng.integers(0, d, size=k) for d in dims])
    corners = np.array([[a, b, c] for a in (0, dims[0] - 1) for b in (0, dims[1] - 1)
                        for c in (0, dims[2] - 1)]).T
    return np.concatenate([corners, pts], axis=1)


def at(field, pts):
    return field[..., pts[0], pts[1], pts[2]]


def params_of(w, k2, batch):
    return D.SweepParams(metric=w.metric, win=w.win, ncc_eps=w.ncc_eps, lam=w.lam,
                         smooth_sigma=w.smooth_sigma, n_sq=w.n_sq, k2=k2, batch=batch)


def first_step_velocity(img, A0, w):
    """v after the first inner step from v = 0 (oracle): dL/dv = dL/du at
    u = 0 (the regulariser's gradient vanishes there), one Adam step, then the
    Gaussian when the workload smooths v."""
    _, gw = O.lncc(img, A0, w.win, w.ncc_eps)
    g = O.warp3d_bwd(img, np.zeros((3,) + img.shape), gw)
    z = np.zeros_like(g)
    v, _, _ = O.adam_step(z, z, z, g, 1, w.lr, w.beta1, w.beta2, w.adam_eps)
    if w.smooth_sigma > 0:
        v = O.gauss_smooth(v, w.smooth_sigma)
    return v


def rel_l2(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def check_sweep_from_zero(dev, w, images, batch, check, k2, second_loss_of=None):
    """One sweep of k2 inner steps from v = 0 in the given launch
    configuration, checked as the module docstring says."""
    print(f"sweep {w.name}: batch {batch}, k2 {k2}, subjects {check}", flush=True)
    imgs = torch.from_numpy(images).to(dev)
    c = D.Cohort(imgs, params_of(w, k2, batch))
    A0 = c.atlas.cpu().numpy()
    assert np.array_equal(A0, np.mean(images, axis=0, dtype=np.float64).astype(np.float32))
    losses = c.sweep().cpu().numpy()
    torch.cuda.synchronize()
    assert np.all(np.isfinite(losses))
    for i in check:
        rl, _ = O.lncc(images[i], A0, w.win, w.ncc_eps)
        assert abs(losses[i * k2] - rl) <= 1e-6 * abs(rl), (i, losses[i * k2], rl)
        if k2 == 1:
            v1 = first_step_velocity(images[i].astype(np.float64), A0.astype(np.float64), w)
            err = rel_l2(c.v[i].cpu().numpy(), v1)
            assert err <= 1e-4, (i, err)
    if second_loss_of is not None:
        i = second_loss_of
        v1 = first_step_velocity(images[i].astype(np.float64), A0.astype(np.float64), w)
        u1, _ = O.exp_svf(v1, w.n_sq)
        rl, _ = O.lncc(O.warp3d(images[i], u1), A0, w.win, w.ncc_eps)
        if w.lam:
            rl += w.lam * O.diffusion_reg(u1)[0]
        assert abs(losses[i * k2 + 1] - rl) <= 1e-5 * abs(rl), (i, losses[i * k2 + 1], rl)
    # centred displacements: the FP64 sum over all subjects vanishes
    uh = c.u_hat
    s = torch.sum(uh, dim=0, dtype=torch.float64).abs().max().item()
    assert s <= w.n * uh.abs().max().item() * 2.0 ** -22, s
    # the atlas is the mean of the warped subjects
    pts = samples(4, w.dims)
    pt = torch.from_numpy(pts).to(dev)
    u_at = uh[:, :, pt[0], pt[1], pt[2]].cpu().numpy().astype(np.float64)
    ref = np.mean([O.sample_zero(images[i], pts.astype(np.float64) + u_at[i])[0]
                   for i in range(w.n)], axis=0)
    A = c.atlas.cpu().numpy()
    assert np.abs(at(A, pts) - ref).max() <= 1e-5 * np.abs(A).max()


# ------------------------------------------------------ 64 subjects of 128^3


@pytest.fixture(scope="module")
def images3():
    return make_cohort(W3, workers=WORKERS)


def test_c3_sweep_at_full_size(dev, images3):
    """All 64 subjects per launch; LNCC with the regulariser fused into its
    adjoint: the second inner loss of the last subject includes lambda R."""
    check_sweep_from_zero(dev, W3, images3, 0, (0, W3.n - 1), 2, second_loss_of=W3.n - 1)


def test_c3_first_step_velocities(dev, images3):
    check_sweep_from_zero(dev, W3, images3, 0, (0, W3.n - 1), 1)


# ------------------------------------- 200 subjects of 160 x 192 x 224, 64/launch


@pytest.fixture(scope="module")
def images5():
    return make_cohort(W5, workers=WORKERS)


@pytest.fixture(scope="module")
def velocity5():
    # 64 fields of the workload's deformation scale (max 10 voxels)
    return random_velocity(2005, BATCH5, W5.dims, W5.max_disp, corr_len=W5.corr_len,
                           workers=WORKERS)


def test_c5_squaring_steps_and_warp_batched(dev, images5, velocity5):
    vd = torch.from_numpy(velocity5).to(dev)
    u, ck = D.exp_svf(vd, W5.n_sq)
    imgs = torch.from_numpy(images5[:BATCH5]).to(dev)
    w = D.warp3d(imgs, u)
    torch.cuda.synchronize()
    pts = samples(1, W5.dims)
    x = pts.astype(np.float64)
    pt = torch.from_numpy(pts).to(dev)
    for i in (0, BATCH5 - 1):
        print(f"c5 squaring steps, subject {i}", flush=True)
        full = [velocity5[i].astype(np.float64) / 2 ** W5.n_sq]
        for t in range(W5.n_sq - 1):
            full.append(ck[t, i].cpu().numpy().astype(np.float64))
        full.append(u[i].cpu().numpy().astype(np.float64))
        for t in range(W5.n_sq):
            ut = full[t]
            ref = at(ut, pts) + O.sample_border(ut, x + at(ut, pts))[0]
            err = np.abs(at(full[t + 1], pts) - ref).max() / np.abs(ref).max()
            assert err <= 1e-6, (i, t, err)
        u_i = u[i][:, pt[0], pt[1], pt[2]].cpu().numpy().astype(np.float64)
        ref = O.sample_zero(images5[i], x + u_i)[0]
        got = w[i][pt[0], pt[1], pt[2]].cpu().numpy()
        assert np.abs(got - ref).max() <= 1e-5 * np.abs(images5[i]).max()


@pytest.mark.parametrize("step", [0, 6])
def test_c5_squaring_adjoint_batched(dev, velocity5, step):
    """One adjoint step on 64 subjects (n_sq = 1 on v = 2 u_t is half the
    adjoint of the squaring step at u_t)."""
    vd = torch.from_numpy(velocity5).to(dev)
    if step == 0:
        ut = vd / 2 ** W5.n_sq
    else:
        _, ck = D.exp_svf(vd, W5.n_sq)
        ut = ck[step - 1].contiguous()
        del ck
    gu = torch.from_numpy(random_volume(2006, velocity5.shape, -1.0, 1.0)).to(dev)
    gv = D.exp_svf_bwd((2.0 * ut).contiguous(), None, gu, 1)
    torch.cuda.synchronize()
    pts = samples(2, W5.dims, k=300)
    for i in (0, BATCH5 - 1):
        print(f"c5 adjoint step {step}, subject {i}", flush=True)
        u_i = ut[i].cpu().numpy().astype(np.float64)
        ref = 0.5 * O.squaring_step_bwd_at(u_i, gu[i].cpu().numpy(), pts)
        got = at(gv[i].cpu().numpy(), pts)
        assert rel_l2(got, ref) <= 1e-5, (i, rel_l2(got, ref))


def test_c5_sweep_batched_with_ragged_last_batch(dev, images5):
    """64 subjects per launch over 200 (batches 64, 64, 64, 8)."""
    check_sweep_from_zero(dev, W5, images5, BATCH5, (0, BATCH5 - 1, BATCH5, W5.n - 1), 1)
