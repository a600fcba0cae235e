#!/usr/bin/env python3
"""Throughput of one DARC coordinate-descent sweep on one MI355X.

A step is one sweep of Eq. (3) / Algorithm 1 over the whole cohort: K2 inner
iterations per subject (Exp by scaling and squaring, warp, dissimilarity and
regulariser, adjoint through warp and squarings, Adam, Gaussian smoothing of
v), then Exp, centrality activation, mean atlas and group loss.  Inputs are a
seeded synthetic cohort already resident in GPU memory when timing starts.

Prints one JSON line: subject-voxel-iterations per second (n * V * K2 per
sweep time), the roofline position of the kernel class that takes the most
time, the per-class achieved bandwidth, and the FP64 CPU oracle timed on a
bounded sample of the same workload on one host core.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
BF16_PEAK_FLOPS = 2.5e15  # MI355X dense BF16 matrix-core peak, vendor figure

DEFAULT_WORKLOAD = "brain-16x160x192x160-lncc9"


def algorithmic_bytes(w, batch):
    """Bytes each kernel class must move per sweep (FP32 state, one pass per
    step, gathers served from cache), keyed like the library's timing classes."""
    n, V, k2, N = w.n, w.voxels, w.k2, w.n_sq
    lncc = w.metric == "lncc"
    b = {
        # per squaring step: read u_t (12 B), write u_{t+1} (12 B)
        "exp_fwd_step": N * (k2 + 1) * n * V * 24,
        # per adjoint step: read u_t and g_{t+1}, write g_t (12 B each)
        "exp_bwd_step": N * k2 * n * V * 36,
        # read g, v, m, s; write v, m, s
        "adam": k2 * n * V * 84,
        # read u of every subject, write centred u
        "center": n * V * 24,
        # read u and the image of every subject, write the atlas
        "atlas": n * V * 16 + V * 4,
    }
    if lncc:
        b["warp"] = (k2 + 1) * n * V * 20           # read u, image; write warped
        b["lncc_fwd"] = k2 * n * V * 24 + n * V * 8  # read warped, atlas; write 4 factors
        b["lncc_bwd"] = k2 * n * V * 52              # read 4 factors, warped, atlas, u, image; write g
        if w.lam:
            b["diffusion"] = n * V * 12
    else:
        b["mse"] = k2 * n * V * 32 + n * V * 20      # fused warp + MSE (+ adjoint)
    if w.smooth_sigma > 0:
        b["gauss"] = k2 * n * V * 24
    return b


def source_digest():
    """SHA-256 over the HIP sources, to tell whether counters taken earlier
    still describe the kernels that run now."""
    import hashlib

    h = hashlib.sha256()
    src = os.path.join(ROOT, "paper_2508_10743_amd", "csrc")
    for name in sorted(os.listdir(src)):
        with open(os.path.join(src, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def measured_traffic(workload, kernel_class):
    """HBM bytes per launch of `kernel_class` from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, each scaled by the same counter's
    reading for a plain 1 GiB copy), in GB; None when there is no summary for
    this workload and class or the kernels changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].split(": ", 1)
                fields[k.strip("` ")] = v.strip().strip("`")
    if fields.get("source_sha256") != source_digest() or fields.get("class") != kernel_class:
        return None
    try:
        return float(fields["hbm_GB_per_launch"])
    except (KeyError, ValueError):
        return None


def time_extras(D, cohort, w, reps=3):
    """Time the other branches of the method on the bench cohort (its
    current state): each entry gives ms per call and the achieved rate of its
    algorithmic bytes (FP32 state read or written once, gathers from cache)."""
    import torch

    n, V = w.n, w.voxels
    imgs, u, atlas = cohort.images, cohort.u_hat, cohort.atlas

    def timed(fn):
        fn()
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        start.record()
        for _ in range(reps):
            fn()
        stop.record()
        stop.synchronize()
        return start.elapsed_time(stop) / reps

    warped = D.warp3d(imgs, u)
    labels = (imgs[0] > 0.35).to(torch.uint8) + (imgs[0] > 0.65).to(torch.uint8)
    a_sgd = atlas.clone()
    coarse = D.down2(u)
    batch = 4
    cases = {
        # read n images (gathered) and n displacements, write the atlas
        "atlas_median": (lambda: D.atlas_median(imgs, u), n * V * 16 + V * 4),
        # one epoch: per minibatch LNCC statistics and adjoint of the atlas
        # against each subject (read 2, write 4 factors; read 4 factors and 2,
        # write 1), then Adam on the atlas reading the minibatch gradients
        "atlas_sgd_epoch": (lambda: D.atlas_sgd(warped, a_sgd, epochs=1, batch=batch, win=w.win),
                            n * V * (24 + 28) + ((n + batch - 1) // batch) * V * 24 + n * V * 4),
        # Exp(-v) (7 squaring steps) and the label lookup
        "segment": (lambda: D.segment(labels, cohort.v), n * V * (7 * 24 + 13)),
        # 2x2x2 means of the displacements; trilinear upsampling back
        "down2_fields": (lambda: D.down2(u), n * 3 * V * 4 + n * 3 * V // 2),
        "up2_fields": (lambda: D.up2(coarse, 2.0), n * 3 * V * 4 + n * 3 * V // 2),
    }
    res = {}
    for name, (fn, nbytes) in cases.items():
        ms = timed(fn)
        res[name] = {"ms": round(ms, 3), "algo_GB": round(nbytes / 1e9, 4),
                     "GB/s": round(nbytes / (ms * 1e-3) / 1e9, 1)}
    # the warm-start network on 4 subjects: matrix-core bound, so its rate is
    # given in TFLOP/s against the dense BF16 peak
    from paper_2508_10743_amd import unet as N

    net = N.UNet(seed=0)
    sub = imgs[:4].contiguous()
    flop = 0.0
    for level, (cin, cout, stride, _) in zip((0, 1, 2, 3, 2, 1, 0, 0), N.LAYERS):
        flop += 2.0 * 27 * cin * cout * sub.shape[0] * V / 8 ** level
    ms = timed(lambda: net(atlas, sub))
    res["unet_forward_4"] = {"ms": round(ms, 3), "GFLOP": round(flop / 1e9, 1),
                             "TFLOP/s": round(flop / (ms * 1e-3) / 1e12, 1),
                             "frac_bf16_peak": round(flop / (ms * 1e-3) / BF16_PEAK_FLOPS, 4)}
    # one training step on 2 subjects against their current velocities:
    # forward, input and weight gradients (3x the forward's products)
    tr = N.Trainer(N.UNet(seed=1), lr=1e-4)
    sub2, tgt2 = imgs[:2].contiguous(), cohort.v[:2].contiguous()
    ms = timed(lambda: tr.step(atlas, sub2, tgt2))
    flop2 = 3.0 * flop / 2.0
    res["unet_train_step_2"] = {"ms": round(ms, 3), "GFLOP": round(flop2 / 1e9, 1),
                                "TFLOP/s": round(flop2 / (ms * 1e-3) / 1e12, 1),
                                "frac_bf16_peak": round(flop2 / (ms * 1e-3) / BF16_PEAK_FLOPS, 4)}
    res["warm_start"] = warm_start_trial(dev=imgs.device)
    return res


def warm_start_trial(dev, n_train=64, n_test=8, epochs=10):
    """Time-to-loss of the learned warm start on 4 x 32^3 blob cohorts:
    train the U-Net on DARC's velocities (20 sweeps of 20 steps) for n_train
    cohorts, then on n_test held-out cohorts run the C1 schedule (10 sweeps
    of 5 steps) from v = 0 and from the network's velocities, and count the
    sweeps until the group loss is within 0.5 % of plain DARC's final one."""
    from synthetic.cohorts import WORKLOADS

    from paper_2508_10743_amd import darc as D
    from paper_2508_10743_amd import warmstart as WS

    w = WORKLOADS["blobs-4x32^3-mse"]
    t0 = time.perf_counter()
    train = WS.make_triples(w, range(2000, 2000 + n_train), D.SweepParams(k2=20), 20, dev)
    t1 = time.perf_counter()
    net, hist = WS.train(train, epochs=epochs, lr=1e-3)
    torch_sync = __import__("torch").cuda.synchronize
    torch_sync()
    t2 = time.perf_counter()
    r = WS.evaluate(net, w, range(3000, 3000 + n_test), D.SweepParams(k2=5), 10, dev)
    return {"train_cohorts": n_train, "epochs": epochs, "triples_s": round(t1 - t0, 2),
            "train_s": round(t2 - t1, 2), "train_loss_first_last": [round(hist[0], 5),
                                                                   round(hist[-1], 5)],
            "sweeps_to_plain_final": {"plain": r["plain_sweeps"], "warm": r["warm_sweeps"]},
            "seconds_to_plain_final": {"plain": round(r["plain_s"], 4),
                                       "warm": round(r["warm_s"], 4)},
            "loss_after_1_sweep": {"plain": r["plain_first"], "warm": r["warm_first"]}}


def cpu_baseline(w, seconds_hint=True):
    """The FP64 oracle on one subject's central crop (1/8 of the voxels),
    two inner iterations, one thread."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import darc_oracle as O
    from synthetic.cohorts import make_cohort

    imgs = make_cohort(w, n=2)
    d0, d1, d2 = w.dims
    sl = (slice(d0 // 4, d0 // 4 + d0 // 2), slice(d1 // 4, d1 // 4 + d1 // 2),
          slice(d2 // 4, d2 // 4 + d2 // 2))
    subj = imgs[0][sl].astype(np.float64)
    atlas = imgs[1][sl].astype(np.float64)
    p = O.SweepParams(metric=w.metric, win=w.win, ncc_eps=w.ncc_eps, lam=w.lam,
                      smooth_sigma=w.smooth_sigma, n_sq=w.n_sq, k2=w.k2)
    iters = 2
    with threadpool_limits(limits=1):
        v = np.zeros((3,) + subj.shape)
        m = np.zeros_like(v)
        s = np.zeros_like(v)
        t0 = time.perf_counter()
        for k in range(iters):
            _, g = O.subject_loss_grad(subj, v, atlas, p)
            v, m, s = O.adam_step(v, m, s, g, k + 1)
            if p.smooth_sigma > 0:
                v = O.gauss_smooth(v, p.smooth_sigma)
        dt = time.perf_counter() - t0
    vox = subj.size
    return {
        "value": vox * iters / dt,
        "unit": "subject-voxel-iters/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"1 subject, central {subj.shape[0]}x{subj.shape[1]}x{subj.shape[2]} crop "
                  f"of {w.name}, {iters} inner iterations (Exp, warp, dissimilarity, adjoint, "
                  f"Adam, smoothing), FP64 NumPy, {dt:.1f} s",
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed sweeps")
    ap.add_argument("--warmup", type=int, default=1, help="untimed sweeps before timing")
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--batch", type=int, default=0, help="subjects per launch (0 = all)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="skip the per-kernel event timing")
    ap.add_argument("--graph", action="store_true",
                    help="capture one sweep in a HIP graph and time its replays")
    ap.add_argument("--extras", action="store_true",
                    help="also time the method's other branches (median and stochastic atlas, "
                         "one-shot segmentation, pyramid resampling) on the same cohort")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 1 GiB device-to-device copy first (a known-size kernel for "
                         "calibrating HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU: the DARC path here runs on a single MI355X and has "
              f"no multi-GPU mode (asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)

    from synthetic.cohorts import WORKLOADS, make_cohort

    w = WORKLOADS[args.workload]
    cpu = None if args.no_cpu_baseline else cpu_baseline(w)

    import torch

    from paper_2508_10743_amd import darc as D

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    print(f"# generating {w.name}", file=sys.stderr, flush=True)
    # large cohorts are generated in a process pool (same images), sized to the
    # CPU share of one GPU
    workers = min(16, os.cpu_count() or 1) if w.n >= 32 else 1
    images = torch.from_numpy(make_cohort(w, workers=workers)).to(dev)
    params = D.SweepParams(metric=w.metric, win=w.win, ncc_eps=w.ncc_eps, lam=w.lam,
                           smooth_sigma=w.smooth_sigma, n_sq=w.n_sq, k2=w.k2, lr=w.lr,
                           beta1=w.beta1, beta2=w.beta2, adam_eps=w.adam_eps, batch=args.batch)
    cohort = D.Cohort(images, params, device_step=args.graph)
    torch.cuda.synchronize()
    if args.calib_copy:
        a = torch.full((1 << 28,), 1.0, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)  # reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        del a, b
    for i in range(args.warmup):
        cohort.sweep()
        torch.cuda.synchronize()
        print(f"# warmup sweep {i + 1}/{args.warmup}: F = {cohort.group_loss():.6f}",
              file=sys.stderr, flush=True)

    # per-kernel events cannot be recorded inside a captured graph
    profile = not args.no_profile and not args.graph
    if profile:
        D.profile_reset()
        D.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if args.graph:
        # one sweep captured into a HIP graph, replayed per timed step
        graph = cohort.capture()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            graph.replay()
    else:
        for _ in range(args.steps):
            cohort.sweep()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kernels = {}
    roofline = None
    if profile:
        D.profile_enable(False)
        prof = D.profile_collect()
        algo = algorithmic_bytes(w, args.batch)
        for cls, (cnt, ms) in prof.items():
            if cnt == 0:
                continue
            entry = {"launches": cnt, "ms": round(ms, 4), "avg_us": round(1e3 * ms / cnt, 2)}
            if cls in algo:
                gbs = algo[cls] * args.steps / (ms * 1e-3) / 1e9
                entry["algo_GB_per_launch"] = round(algo[cls] * args.steps / cnt / 1e9, 4)
                entry["GB/s"] = round(gbs, 1)
            kernels[cls] = entry
        dom = max((c for c in kernels if "GB/s" in kernels[c]), key=lambda c: kernels[c]["ms"])
        achieved = kernels[dom]["GB/s"]
        roofline = {
            "kernel": dom,
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(w.name, dom),
            "traffic_unit": "GB per launch (HBM, from counters)",
        }

    extras = time_extras(D, cohort, w) if args.extras else None
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = w.n * w.voxels * w.k2 / (ms_per_step * 1e-3)
    out = {
        "metric": "subject-voxel-iters/s per DARC sweep",
        "value": round(value, 1),
        "unit": "subject-voxel-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": w.name,
            "n_subjects": w.n,
            "dims": list(w.dims),
            "metric": f"{w.metric}{w.win if w.metric == 'lncc' else ''}",
            "k2": w.k2,
            "n_sq": w.n_sq,
            "smooth_sigma": w.smooth_sigma,
            "lam": w.lam,
            "batch": args.batch or w.n,
        },
        "group_loss": cohort.group_loss(),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels": kernels,
    }
    if extras is not None:
        out["extras"] = extras
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
