"""darc_sim_grad_noalloc against darc_sim_grad, through the C ABI.

The entry point that allocates nothing keeps the LNCC factor fields in the
library's per-GPU scratch array.  Two calls in a row, the second on a smaller
volume (the array still holds the first call's fields), must give what
darc_sim_grad gives with a caller workspace: gradients bit for bit (the same
kernels on the same inputs), losses to 1e-12 (FP64 atomics across blocks add
in any order), and both within the oracle's tolerances.  A call that needs
more than the array holds fails before enqueueing anything.
"""

import numpy as np
import pytest
import torch

from oracle import darc_oracle as O
from paper_2508_10743_amd import _lib as L
from paper_2508_10743_amd import darc as D
from synthetic.cohorts import WORKLOADS, make_cohort

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    D.lib()
    return torch.device("cuda", 0)


def _case(n, dims, seed, dev):
    w = WORKLOADS["blobs-4x32^3-mse"]
    imgs = make_cohort(w, n=n + 1, dims=dims, seed=seed)
    warped = torch.from_numpy(imgs[:n].copy()).to(dev)
    atlas = torch.from_numpy(imgs[n].copy()).to(dev)
    return warped, atlas


@pytest.mark.parametrize("metric,win", [("lncc", 9), ("lncc", 5), ("mse", 9), ("l1", 9)])
def test_noalloc_matches_workspace_entry_point(dev, metric, win):
    for n, dims, seed in ((3, (40, 48, 56), 901), (1, (17, 23, 31), 902)):
        print(f"noalloc case: metric={metric} win={win} n={n} dims={dims}", flush=True)
        warped, atlas = _case(n, dims, seed, dev)
        ref_loss, ref_g = D.sim_grad(warped, atlas, metric, win)
        loss = torch.zeros(n, dtype=torch.float64, device=dev)
        g = torch.full_like(warped, float("nan"))
        D.sim_grad_noalloc(warped, atlas, loss, g, metric, win)
        torch.cuda.synchronize()
        assert torch.equal(g, ref_g)
        rl, tl = loss.cpu().numpy(), ref_loss.cpu().numpy()
        assert np.abs(rl - tl).max() <= 1e-12 * np.abs(tl).max()
        # loss only: no scratch needed
        loss2 = torch.zeros(n, dtype=torch.float64, device=dev)
        D.sim_grad_noalloc(warped, atlas, loss2, None, metric, win)
        assert np.abs(loss2.cpu().numpy() - tl).max() <= 1e-12 * np.abs(tl).max()
    # the smaller case against the oracle
    W, A = warped.cpu().numpy()[0], atlas.cpu().numpy()
    if metric == "lncc":
        ol, og = O.lncc(W, A, win)
    elif metric == "mse":
        ol, og = O.mse(W, A)
    else:
        ol, og = O.l1(W, A)
    assert abs(loss[0].item() - ol) <= 1e-6 * abs(ol)
    gg = g[0].cpu().numpy().astype(np.float64)
    assert np.linalg.norm(gg - og) <= 1e-4 * np.linalg.norm(og)


def test_noalloc_rejects_more_than_its_scratch(dev):
    cap = D.lib().darc_sim_grad_noalloc_max_bytes()
    assert cap == 128 << 20
    # 16 bytes per subject-voxel: 2 subjects of 160 x 192 x 224 exceed 128 MiB
    n, dims = 2, (160, 192, 224)
    assert 16 * n * int(np.prod(dims)) > cap
    warped = torch.zeros((n,) + dims, dtype=torch.float32, device=dev)
    atlas = torch.zeros(dims, dtype=torch.float32, device=dev)
    loss = torch.zeros(n, dtype=torch.float64, device=dev)
    g = torch.zeros_like(warped)
    with pytest.raises(D.DarcError) as ei:
        D.sim_grad_noalloc(warped, atlas, loss, g, "lncc", 9)
    assert ei.value.status == L.DARC_EWORKSPACE
    assert "darc_sim_grad_noalloc" in str(ei.value)
    # one such subject fits
    D.sim_grad_noalloc(warped[:1], atlas, loss[:1], g[:1], "lncc", 9)
    torch.cuda.synchronize()
    assert float(loss[0].item()) == 0.0
