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

from synthetic.cohorts import Workload, make_cohorts

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


def make_triples(w: Workload, seeds, params: D.SweepParams, sweeps: int, device,
                 workers: int = 1, chunk: int = 50, progress=None) -> List[Triple]:
    """One triple per seed: the cohort, its A^0 and DARC's velocities after
    ``sweeps`` sweeps with ``params`` (phantoms generated in ``workers``
    processes, ``chunk`` cohorts at a time; the triples stay on the device).
    ``progress(msg)``, if given, is called after every chunk."""
    seeds = list(seeds)
    out = []
    t0 = time.perf_counter()
    for c0 in range(0, len(seeds), chunk):
        for imgs in make_cohorts(w, seeds[c0:c0 + chunk], workers=workers):
            imgs = torch.from_numpy(imgs).to(device)
            coh, _ = darc_run(imgs, params, sweeps)
            out.append(Triple(D.atlas_update(imgs, None), imgs, coh.v.clone()))
        if progress is not None:
            torch.cuda.synchronize()
            progress(f"triples: {len(out)}/{len(seeds)} cohorts in {time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    return out


def unet_flop(n: int, dims) -> float:
    """Multiply-adds x 2 of one forward pass on n subjects (unpadded channels)."""
    V = float(np.prod(dims))
    levels = (0, 1, 2, 3, 2, 1, 0, 0)  # resolution level of each layer's output
    return sum(2.0 * 27 * cin * cout * n * V / 8 ** lev
               for lev, (cin, cout, _, _) in zip(levels, N.LAYERS))


BF16_PEAK = 2.5e15  # dense BF16 matrix-core FLOP/s of the MI355X


def unet_rates(net: N.UNet, triple: Triple, reps: int = 5) -> dict:
    """Milliseconds and matrix-core rate of the network's forward pass and of
    one training step (forward, input and weight gradients: three times the
    forward's products) on one training cohort, timed with GPU events.  The
    training step runs on a copy of the network's parameters."""
    tr = N.Trainer(N.UNet(seed=12345, device=net.device))

    def timed(fn):
        fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        b.synchronize()
        return a.elapsed_time(b) / reps

    n = triple.images.shape[0]
    flop = unet_flop(n, tuple(triple.images.shape[1:]))
    fwd = timed(lambda: net(triple.atlas0, triple.images))
    step = timed(lambda: tr.step(triple.atlas0, triple.images, triple.v))
    return {"subjects": n, "dims": list(triple.images.shape[1:]),
            "forward_ms": round(fwd, 3), "forward_GFLOP": round(flop / 1e9, 1),
            "forward_TFLOPs": round(flop / fwd / 1e9, 1),
            "forward_frac_bf16_peak": round(flop / (fwd * 1e-3) / BF16_PEAK, 4),
            "train_step_ms": round(step, 3),
            "train_step_TFLOPs": round(3 * flop / step / 1e9, 1),
            "train_step_frac_bf16_peak": round(3 * flop / (step * 1e-3) / BF16_PEAK, 4)}


def train(triples: List[Triple], epochs: int, lr: float = 1e-3, seed: int = 0,
          net: N.UNet = None, progress=None) -> Tuple[N.UNet, List[float]]:
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
        if progress is not None:
            progress(f"training: epoch {len(hist)}/{epochs}, mean loss {hist[-1]:.3e}")
    return net, hist


def loss_target(f_final: float, tol: float = 0.005) -> float:
    """Equal final loss within +-tol: a run has reached F_final once its group
    loss is at most F_final + tol |F_final| (losses fall; LNCC's are negative)."""
    return f_final + tol * abs(f_final)


def first_reach(times: List[float], losses: List[float], target: float):
    """(seconds, sweeps) at the first sweep whose group loss is <= target, or
    (None, None)."""
    for k, (t, f) in enumerate(zip(times, losses)):
        if f <= target:
            return t, k + 1
    return None, None


def timed_run(images: torch.Tensor, params: D.SweepParams, sweeps: int,
              net: N.UNet = None) -> Tuple[List[float], List[float]]:
    """One DARC run, timed on the GPU: from v = 0, or from the network's
    velocities (its inference, the atlas of A^0 it reads and the level start
    inside the timed region).  Returns the seconds from the start to the end
    of each sweep and the group loss after each sweep; the host enqueues the
    sweeps back to back and synchronises once at the end."""
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    start.record()
    v0 = net(D.atlas_update(images, None), images) if net is not None else None
    coh = D.Cohort(images, params, v0=v0)
    if v0 is not None:
        coh.level_start()
    events, fs = [], []
    for _ in range(sweeps):
        losses = coh.sweep()
        fs.append(losses[-1:].clone())
        ev = torch.cuda.Event(enable_timing=True)
        ev.record()
        events.append(ev)
    torch.cuda.synchronize()
    return [start.elapsed_time(e) * 1e-3 for e in events], [float(f.item()) for f in fs]


def evaluate(net: N.UNet, cohorts: List[torch.Tensor], params: D.SweepParams, sweeps: int,
             tol: float = 0.005) -> dict:
    """Time-to-loss on held-out cohorts: plain DARC (one subject per launch,
    from v = 0) runs ``sweeps`` sweeps and sets the target F_plain_final +
    tol |F_plain_final|; the batched, warm-started form (every subject in one
    launch, from the network's velocities) runs until it reaches that target
    or ``sweeps`` sweeps.  Wall-clock seconds are measured, per cohort."""
    plain_p = dataclasses.replace(params, batch=1)
    warm_p = dataclasses.replace(params, batch=0)
    rows = []
    # first calls load code objects and grow the allocator: run both once untimed
    timed_run(cohorts[0], plain_p, 1)
    timed_run(cohorts[0], warm_p, 1, net)
    for imgs in cohorts:
        tp, fp = timed_run(imgs, plain_p, sweeps)
        target = loss_target(fp[-1], tol)
        sp, kp = first_reach(tp, fp, target)
        tw, fw = timed_run(imgs, warm_p, sweeps, net)
        sw, kw = first_reach(tw, fw, target)
        rows.append(dict(plain_final=fp[-1], target=target, plain_s=sp, plain_sweeps=kp,
                         warm_s=sw, warm_sweeps=kw, warm_final=fw[-1], plain_first=fp[0],
                         warm_first=fw[0]))
    return {"cohorts": rows}


def time_to_loss(w: Workload, train_seeds, test_seeds, device, target_sweeps: int = 10,
                 target_k2: int = 10, epochs: int = 10, lr: float = 1e-3,
                 workers: int = 1, progress=None) -> dict:
    """The whole comparison on cohorts of workload ``w``: training triples from
    plain DARC (``target_sweeps`` sweeps of ``target_k2`` steps), the U-Net
    trained on them, then :func:`evaluate` on held-out cohorts with the
    workload's own schedule (K1 sweeps of K2 steps).  Times of each stage in
    seconds; per-cohort results plus their means."""
    params = D.SweepParams(metric=w.metric, win=w.win, ncc_eps=w.ncc_eps, lam=w.lam,
                           smooth_sigma=w.smooth_sigma, n_sq=w.n_sq, k2=w.k2, lr=w.lr,
                           beta1=w.beta1, beta2=w.beta2, adam_eps=w.adam_eps)
    t0 = time.perf_counter()
    triples = make_triples(w, train_seeds, dataclasses.replace(params, k2=target_k2),
                           target_sweeps, device, workers=workers, progress=progress)
    t1 = time.perf_counter()
    net, hist = train(triples, epochs=epochs, lr=lr, progress=progress)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    rates = unet_rates(net, triples[0])
    del triples
    test = [torch.from_numpy(c).to(device) for c in make_cohorts(w, test_seeds, workers=workers)]
    res = evaluate(net, test, params, w.k1)
    rows = res["cohorts"]
    reached = [r for r in rows if r["warm_s"] is not None]
    out = {
        "cohort": w.name,
        "schedule": f"{w.k1} sweeps x {w.k2} steps",
        "target": "F <= F_plain_final + 0.005 |F_plain_final|",
        "plain": "one subject per launch, from v = 0",
        "warm": "all subjects per launch, from the U-Net's velocities (inference timed)",
        "train": {"cohorts": len(train_seeds), "pairs": len(train_seeds) * w.n,
                  "target_run": f"{target_sweeps} sweeps x {target_k2} steps",
                  "epochs": epochs, "triples_s": round(t1 - t0, 2), "train_s": round(t2 - t1, 2),
                  "loss_first_last": [round(hist[0], 6), round(hist[-1], 6)]},
        "unet": rates,
        "test_cohorts": len(rows),
        "warm_reached": len(reached),
        "plain_s": float(np.mean([r["plain_s"] for r in rows])),
        "plain_sweeps": float(np.mean([r["plain_sweeps"] for r in rows])),
        "cohorts_detail": rows,
    }
    if reached:
        out["warm_s"] = float(np.mean([r["warm_s"] for r in reached]))
        out["warm_sweeps"] = float(np.mean([r["warm_sweeps"] for r in reached]))
        out["speedup"] = float(np.mean([r["plain_s"] / r["warm_s"] for r in reached]))
    return out
