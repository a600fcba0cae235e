"""The fused inner iteration (one persistent launch per iteration) against the
FP64 oracle.

- Sweeps with `fused="on"` match the oracle (MSE and L1, both centring modes,
  subject batches, displacements whose adjoint reaches beyond one voxel).
- Fused and separate launches agree with each other.
- A captured sweep replayed several times matches the oracle's sweeps after
  every replay, on both paths.
- The autotuner's fused-or-separate choice leaves the state alone and the
  tuned sweeps still match the oracle.
- A barrier wait bound of zero makes every wait give up: the sweep finishes
  and reports NaN as its group loss; the default bound restores normal sweeps.

Tolerances as in the main parity tests: inner and group losses rel 1e-6 after
one sweep (1e-5 after more, FP32 state drifts), velocities and centred
displacements rel-L2 1e-4, atlas rel-L-inf 1e-5.
"""

import numpy as np
import pytest
import torch

from oracle import darc_oracle as O
from paper_2508_10743_amd import darc as D
from synthetic.cohorts import WORKLOADS, make_cohort, random_velocity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    D.lib()
    return torch.device("cuda", 0)


def g(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def h(t):
    return t.detach().cpu().numpy().astype(np.float64)


def rel_linf(a, b):
    return float(np.abs(np.asarray(a, np.float64) - b).max() / max(np.abs(b).max(), 1e-300))


def rel_l2(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def blobs(n, dims, seed):
    return make_cohort(WORKLOADS["blobs-4x32^3-mse"], n=n, dims=dims, seed=seed)


def oracle_run(imgs, p, sweeps, v0=None):
    n = len(imgs)
    x = imgs.astype(np.float64)
    v = np.zeros((n, 3) + imgs.shape[1:]) if v0 is None else v0.astype(np.float64)
    m, s = np.zeros_like(v), np.zeros_like(v)
    step, A = 0, O.initial_atlas(x)
    if v0 is not None:
        v, A = O.level_start(x, v, p)
    out = []
    for _ in range(sweeps):
        r = O.sweep(x, v, m, s, step, A, p)
        v, m, s, step, A = r["v"], r["m"], r["s"], r["step"], r["atlas"]
        out.append(r)
    return out


def check_against(c, losses, r, k):
    tol = 1e-6 if k == 0 else 1e-5
    inner = r["inner_losses"].ravel()
    assert np.abs(losses[:-1] - inner).max() <= tol * np.abs(inner).max(), k
    assert abs(losses[-1] - r["group_loss"]) <= tol * abs(r["group_loss"]), k
    assert rel_l2(h(c.v), r["v"]) <= 1e-4, k
    assert rel_l2(h(c.u_hat), r["u_hat"]) <= 1e-4, k
    assert rel_linf(h(c.atlas), r["atlas"]) <= 1e-5, k
    assert c.step == r["step"]


@pytest.mark.parametrize("metric,lam,center,batch,dims", [
    ("mse", 0.01, "displacement", 0, (32, 32, 32)),
    ("mse", 0.01, "velocity", 2, (12, 10, 40)),
    ("mse", 0.0, "displacement", 1, (9, 17, 23)),
    ("l1", 0.01, "displacement", 0, (12, 10, 40)),
])
def test_fused_sweeps_match_oracle(dev, metric, lam, center, batch, dims):
    imgs = blobs(3, dims, 501)
    if metric == "l1":
        # distinct intensity offsets keep every subject off the median, where
        # sign(Iw - A) would be decided by rounding
        imgs = imgs + (0.25 * np.arange(3, dtype=np.float32))[:, None, None, None]
    kw = dict(metric=metric, lam=lam, k2=3, center_mode=center)
    ref = oracle_run(imgs, O.SweepParams(**kw), 2)
    c = D.Cohort(g(imgs, dev), D.SweepParams(batch=batch, fused="on", **kw))
    for k in range(2):
        check_against(c, h(c.sweep()), ref[k], k)


def test_fused_sweep_with_large_displacements(dev):
    """Velocities of up to 3 voxels with seven squarings: the later adjoint
    steps reach beyond one voxel (every step takes the tiled adjoint here)."""
    dims = (20, 16, 36)
    imgs = blobs(3, dims, 502)
    v0 = random_velocity(503, 3, dims, 3.0, corr_len=3.0)
    kw = dict(metric="mse", lam=0.01, k2=2)
    ref = oracle_run(imgs, O.SweepParams(**kw), 1, v0=v0)
    c = D.Cohort(g(imgs, dev), D.SweepParams(fused="on", **kw), v0=g(v0, dev))
    c.level_start()
    check_against(c, h(c.sweep()), ref[0], 0)


def test_fused_and_separate_launches_agree(dev):
    w = WORKLOADS["blobs-4x32^3-mse"]
    imgs = g(make_cohort(w), dev)
    kw = dict(metric="mse", lam=w.lam, k2=w.k2)
    a = D.Cohort(imgs, D.SweepParams(fused="on", **kw))
    b = D.Cohort(imgs, D.SweepParams(fused="off", **kw))
    for k in range(3):
        la, lb = h(a.sweep()), h(b.sweep())
        assert np.abs(la - lb).max() <= 1e-6 * np.abs(lb).max(), k
        assert rel_l2(h(a.v), h(b.v)) <= 1e-5, k
        assert rel_linf(h(a.atlas), h(b.atlas)) <= 1e-6, k


@pytest.mark.parametrize("fused", ["on", "off"])
def test_captured_sweeps_match_oracle(dev, fused):
    """One sweep captured into a HIP graph and replayed three times, with
    unrelated eager work in between: each replay is the oracle's next sweep."""
    imgs = blobs(3, (16, 12, 40), 504)
    kw = dict(metric="mse", lam=0.01, k2=2)
    ref = oracle_run(imgs, O.SweepParams(**kw), 3)
    c = D.Cohort(g(imgs, dev), D.SweepParams(fused=fused, **kw), device_step=True)
    graph = c.capture()
    torch.cuda.synchronize()
    assert float(c.v.abs().max()) == 0.0
    for k in range(3):
        losses = h(graph.replay())
        junk = torch.randn(4096, device=dev)
        junk.mul_(3.0).sum().item()
        torch.cuda.synchronize()
        check_against(c, losses, ref[k], k)


def test_autotune_fused_choice_keeps_results(dev):
    imgs = blobs(4, (32, 32, 32), 505)
    kw = dict(metric="mse", lam=0.01, k2=2)
    ref = oracle_run(imgs, O.SweepParams(**kw), 2)
    c = D.Cohort(g(imgs, dev), D.SweepParams(**kw))
    check_against(c, h(c.sweep()), ref[0], 0)
    v0, m0, a0 = c.v.clone(), c.m.clone(), c.atlas.clone()
    try:
        chosen = c.autotune()
        torch.cuda.synchronize()
        assert chosen[0] in (-1, 8, 16, 32, 64)
        assert chosen[2] in (1, 2)
        assert torch.equal(c.v, v0) and torch.equal(c.m, m0) and torch.equal(c.atlas, a0)
        check_against(c, h(c.sweep()), ref[1], 1)
    finally:
        D.autotune_clear()


def test_barrier_timeout_is_reported(dev):
    imgs = g(blobs(2, (16, 16, 16), 506), dev)
    kw = dict(metric="mse", lam=0.01, k2=1, fused="on")
    try:
        D.fused_barrier_ticks(0)
        c = D.Cohort(imgs, D.SweepParams(**kw))
        losses = h(c.sweep())
        torch.cuda.synchronize()
        assert np.isnan(losses[-1])
    finally:
        D.fused_barrier_ticks(-1)
    c = D.Cohort(imgs, D.SweepParams(**kw))
    assert np.isfinite(h(c.sweep())).all()


def test_fused_on_rejects_lncc_and_smoothing(dev):
    imgs = g(blobs(2, (8, 8, 8), 507), dev)
    for kw in (dict(metric="lncc", win=3), dict(metric="mse", smooth_sigma=1.0)):
        with pytest.raises(D.DarcError):
            D.Cohort(imgs, D.SweepParams(fused="on", **kw))


@pytest.mark.parametrize("metric,sigma,lam,batch", [("mse", 0.0, 0.01, 0), ("lncc", 1.0, 0.0, 2),
                                                   ("mse", 0.0, 0.01, 1)])
def test_plane_parallel_squaring_shape_matches_oracle(dev, metric, sigma, lam, batch):
    """The squaring steps with one plane of a tile per block (no marching) and
    every subject on the tiled adjoint, on separate launches."""
    dims = (20, 12, 40)
    imgs = blobs(3, dims, 508)
    kw = dict(metric=metric, win=5, smooth_sigma=sigma, lam=lam, k2=2)
    ref = oracle_run(imgs, O.SweepParams(**kw), 2)
    c = D.Cohort(g(imgs, dev), D.SweepParams(batch=batch, fused="off", **kw))
    nb = batch or 3
    try:
        D.set_launch_shape("squaring", dims, nb, -1)
        for k in range(2):
            check_against(c, h(c.sweep()), ref[k], k)
    finally:
        D.autotune_clear()


def test_plane_parallel_shape_with_large_displacements(dev):
    dims = (20, 16, 36)
    imgs = blobs(3, dims, 509)
    v0 = random_velocity(510, 3, dims, 3.0, corr_len=3.0)
    kw = dict(metric="mse", lam=0.01, k2=2)
    ref = oracle_run(imgs, O.SweepParams(**kw), 1, v0=v0)
    c = D.Cohort(g(imgs, dev), D.SweepParams(fused="off", **kw), v0=g(v0, dev))
    try:
        D.set_launch_shape("squaring", dims, 3, -1)
        c.level_start()
        check_against(c, h(c.sweep()), ref[0], 0)
    finally:
        D.autotune_clear()
