"""Learned warm start of DARC: produce training triples with DARC itself,
train the U-Net on them, and measure how much sooner DARC reaches a given
group loss when it starts from the network's velocities instead of v = 0.

Every step runs in libdarc (sweeps, network forward and training steps);
this module only schedules them.  Cohorts come from ``synthetic.cohorts``
(seeded phantoms), one cohort per seed.
"""

from __future__ import annotations

import dataclasses
import time
from typing import List, Tuple

import numpy as np
import torch

from synthetic.cohorts import Workload, make_cohort

from . import darc as D
from . import unet as N


@dataclasses.dataclass
class Triple:
    """(A^0, images, target velocities) of one cohort on the device."""

    atlas0: torch.Tensor
    images: torch.Tensor
    v: torch.Tensor


def darc_run(images: torch.Tensor, params: D.SweepParams, sweeps: int,
             v0: torch.Tensor = None) -> Tuple[D.Cohort, List[float]]:
    """``sweeps`` sweeps from v = 0, or from ``v0`` (atlas and centring from
    a k2 = 0 sweep first); returns the cohort and the group loss after each
    sweep (the first entry is the starting point)."""
    coh = D.Cohort(images, params, v0=v0)
    losses = [float(coh.level_start()[0].item())]
    for _ in range(sweeps):
        coh.sweep()
        losses.append(coh.group_loss())
    return coh, losses


def make_triples(w: Workload, seeds, params: D.SweepParams, sweeps: int, device) -> List[Triple]:
    """One triple per seed: the cohort, its A^0 and DARC's velocities after
    ``sweeps`` sweeps with ``params``."""
    out = []
    for s in seeds:
        imgs = torch.from_numpy(make_cohort(w, seed=int(s))).to(device)
        coh, _ = darc_run(imgs, params, sweeps)
        out.append(Triple(D.atlas_update(imgs, None), imgs, coh.v.clone()))
    torch.cuda.synchronize()
    return out


def train(triples: List[Triple], epochs: int, lr: float = 1e-3, seed: int = 0,
          net: N.UNet = None) -> Tuple[N.UNet, List[float]]:
    """Adam on the mean squared velocity error, one cohort per step, cohorts
    in a seeded random order every epoch; returns the net and the per-epoch
    mean loss."""
    net = net or N.UNet(seed=seed)
    tr = N.Trainer(net, lr=lr)
    rng = np.random.default_rng(seed)
    hist = []
    for _ in range(epochs):
        losses = [tr.step(t.atlas0, t.images, t.v) for t in
                  (triples[i] for i in rng.permutation(len(triples)))]
        hist.append(float(torch.stack(losses).mean().item()))
    return net, hist


def sweeps_to_reach(losses: List[float], target: float) -> int:
    """First sweep index whose group loss is <= target (len if never)."""
    for k, f in enumerate(losses):
        if f <= target:
            return k
    return len(losses)


def evaluate(net: N.UNet, w: Workload, seeds, params: D.SweepParams, sweeps: int, device,
             tol: float = 1.005) -> dict:
    """Held-out cohorts: DARC from v = 0 and from the network's velocities.
    Time-to-loss: sweeps (and seconds) until F <= tol * F_plain_final."""
    res = {"plain_final": [], "plain_sweeps": [], "warm_sweeps": [], "plain_s": [],
           "warm_s": [], "warm_first": [], "plain_first": []}
    for s in seeds:
        imgs = torch.from_numpy(make_cohort(w, seed=int(s))).to(device)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, lp = darc_run(imgs, params, sweeps)
        t1 = time.perf_counter()
        v0 = net(D.atlas_update(imgs, None), imgs)
        _, lw = darc_run(imgs, params, sweeps, v0=v0)
        t2 = time.perf_counter()
        target = tol * lp[-1]
        kp, kw = sweeps_to_reach(lp, target), sweeps_to_reach(lw, target)
        res["plain_final"].append(lp[-1])
        res["plain_first"].append(lp[1])
        res["warm_first"].append(lw[1])
        res["plain_sweeps"].append(kp)
        res["warm_sweeps"].append(kw)
        res["plain_s"].append((t1 - t0) * kp / sweeps)
        res["warm_s"].append((t2 - t1) * kw / sweeps)
    return {k: float(np.mean(v)) for k, v in res.items()}
