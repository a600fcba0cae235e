"""The learned warm start end to end on a small scale: triples produced by
DARC itself, the U-Net trained on them, and on held-out cohorts (i) its
velocities are closer to DARC's than v = 0 is and (ii) DARC started from
them is ahead of DARC started from v = 0 after one sweep."""

import numpy as np
import pytest
import torch

from paper_2508_10743_amd import darc as D
from paper_2508_10743_amd import warmstart as WS
from synthetic.cohorts import WORKLOADS

pytestmark = pytest.mark.gpu


def test_warm_start_learns_and_helps():
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    dev = torch.device("cuda", 0)
    w = WORKLOADS["blobs-4x32^3-mse"]
    targets = D.SweepParams(metric="mse", lam=0.01, k2=20)
    train = WS.make_triples(w, range(4000, 4024), targets, 10, dev)
    net, hist = WS.train(train, epochs=6, lr=1e-3, seed=7)
    assert hist[-1] < 0.5 * hist[0], hist
    test = WS.make_triples(w, range(5000, 5004), targets, 10, dev)
    err = np.mean([float(((net(t.atlas0, t.images) - t.v) ** 2).mean()) for t in test])
    zero = np.mean([float((t.v ** 2).mean()) for t in test])
    assert err < 0.5 * zero, (err, zero)
    res = WS.evaluate(net, [t.images for t in test], D.SweepParams(metric="mse", lam=0.01, k2=5),
                      4)["cohorts"]
    for r in res:
        assert r["warm_first"] < r["plain_first"], r
        assert r["plain_sweeps"] is not None and r["plain_s"] > 0.0, r
        assert r["warm_sweeps"] is not None and r["warm_sweeps"] <= r["plain_sweeps"], r
        assert r["target"] >= r["plain_final"]

