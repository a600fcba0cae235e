#!/usr/bin/env python3
"""Throughput of one DARC coordinate-descent sweep on one MI355X.

A step is one sweep of Eq. (3) / Algorithm 1 over the whole cohort: K2 inner
iterations per subject (Exp by scaling and squaring, warp, dissimilarity and
regulariser, adjoint through warp and squarings, Adam, Gaussian smoothing of
v), then Exp, centrality activation, mean atlas and group loss.  Inputs are a
seeded synthetic cohort already resident in GPU memory when timing starts.
The default workload is the full-resolution level of the 200-subject cohort
(200 x 160x192x224, LNCC 9^3, Gaussian sigma 1.5 on v), 64 subjects per
launch.

Prints one JSON line: subject-voxel-iterations per second (n * V * K2 per
sweep time), the roofline position of the kernel class that takes the most
time (against the vendor's 8 TB/s and against the copy bandwidth measured
live), the per-class achieved bandwidth, the brain workload
(16 x 160x192x160) as a second line of figures, the measured time-to-loss of
the batched, warm-started form against plain DARC, and the FP64 CPU oracle
timed on a bounded sample of the same workload on one host core.
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

DEFAULT_WORKLOAD = "compartments-200x160x192x224-lncc9"
SECOND_WORKLOAD = "brain-16x160x192x160-lncc9"
TTL_WORKLOAD = "blobs-4x96x112x96-mse"
MAX_BATCH = 64  # subjects per launch for cohorts larger than this


def log(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


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


# sources that define each timed kernel class's kernels and their launches
# (the shared headers and the entry points included)
CLASS_SOURCES = {
    "exp_bwd_step": ("api.hip", "exp_kernels.hip", "darc_common.hpp", "darc_kernels.hpp",
                     "voxel_bodies.hpp"),
}


def source_digest(kernel_class="exp_bwd_step"):
    """SHA-256 over the HIP sources of a kernel class, to tell whether
    counters taken earlier still describe the kernels that run now."""
    import hashlib

    h = hashlib.sha256()
    src = os.path.join(ROOT, "paper_2508_10743_amd", "csrc")
    for name in sorted(CLASS_SOURCES[kernel_class]):
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
    if (kernel_class not in CLASS_SOURCES or fields.get("class") != kernel_class
            or fields.get("source_sha256") != source_digest(kernel_class)):
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
    return res


def attainable_bandwidth(dev, gib=4, reps=5):
    """Copy, read-only and write-only streams of this library's own kernels
    over `gib` GiB buffers: the bandwidth this GPU reaches, in GB/s (best of
    `reps` timed launches after one untimed one)."""
    import ctypes

    import torch

    from paper_2508_10743_amd import darc as D

    lb = D.lib()
    nbytes = gib << 30
    a = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    sink = torch.zeros(1, dtype=torch.float32, device=dev)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    pa, pb, ps = (ctypes.c_void_p(t.data_ptr()) for t in (a, b, sink))
    cases = {
        "copy": (lambda: lb.darc_bw_copy(pa, pb, nbytes, 0, st), 2 * nbytes),
        "read": (lambda: lb.darc_bw_read(pa, nbytes, ps, 0, st), nbytes),
        "write": (lambda: lb.darc_bw_write(pb, nbytes, 0, st), nbytes),
    }
    out = {}
    for name, (fn, moved) in cases.items():
        assert fn() == 0, name
        best = None
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            assert fn() == 0, name
            e1.record()
            e1.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
        out[name] = round(moved / (best * 1e-3) / 1e9, 1)
    torch.cuda.synchronize()
    del a, b, sink
    torch.cuda.empty_cache()
    out["buffer_GiB"] = gib
    return out


def _oracle_sweep_seconds(sub, p):
    """Seconds of one single-threaded oracle sweep of the cropped subjects
    `sub` (a process-pool task of the whole-host figure)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import darc_oracle as O

    z = np.zeros((len(sub), 3) + sub.shape[1:])
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        O.sweep(sub, z, z, z, 0, O.initial_atlas(sub), p)
        return time.perf_counter() - t0


def cpu_baseline(w, max_crop=(40, 96, 112), n_sub=2, host_procs=16):
    """The FP64 oracle on a bounded sample of workload `w`: one whole sweep
    (K2 inner iterations per subject, then Exp, centring, the atlas update
    and the group loss) of `n_sub` subjects cropped to at most `max_crop`
    about the volume centre, on one thread, in subject-voxel-iterations/s;
    `whole_host` runs the same sample in `host_procs` processes at once
    (at most one per core)."""
    import platform

    import numpy as np

    from oracle import darc_oracle as O
    from synthetic.cohorts import make_cohort

    imgs = make_cohort(w, n=n_sub)
    sl = tuple(slice((d - min(d, c)) // 2, (d - min(d, c)) // 2 + min(d, c))
               for d, c in zip(w.dims, max_crop))
    sub = np.stack([im[sl] for im in imgs]).astype(np.float64)
    p = O.SweepParams(metric=w.metric, win=w.win, ncc_eps=w.ncc_eps, lam=w.lam,
                      smooth_sigma=w.smooth_sigma, n_sq=w.n_sq, k2=w.k2)
    dt = _oracle_sweep_seconds(sub, p)
    # whole host: the same sample in one single-threaded process per core
    # (subjects are independent within a sweep), timed by the wall clock
    procs = max(1, min(host_procs, os.cpu_count() or 1))
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(max_workers=procs) as ex:
        t0 = time.perf_counter()
        list(ex.map(_oracle_sweep_seconds, [sub] * procs, [p] * procs))
        wall = time.perf_counter() - t0
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")),
                         "")
    except OSError:
        pass
    return {
        "value": n_sub * sub[0].size * w.k2 / dt,
        "unit": "subject-voxel-iters/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"one oracle sweep of {n_sub} subjects of {w.name} cropped to "
                  f"{'x'.join(str(d) for d in sub.shape[1:])} about the centre: {w.k2} inner "
                  f"iterations each (Exp, warp, dissimilarity, adjoint, Adam, smoothing), then "
                  f"Exp, centring, atlas and group loss; FP64 NumPy on one thread, {dt:.1f} s",
        "host": {"cpu_model": model or platform.processor(), "cpu_count": os.cpu_count()},
        "whole_host": {"value": procs * n_sub * sub[0].size * w.k2 / wall, "processes": procs,
                       "seconds": round(wall, 1),
                       "sample": "the same sample in each of `processes` single-threaded "
                                 "processes at once (the pool's start-up included)"},
    }


def run_workload(D, w, batch, steps, warmup, dev, profile=True, graph=False, keep=False,
                 workers=1, autotune=False):
    """Generate workload `w`, run `warmup` untimed sweeps and `steps` timed
    ones; returns (result dict, cohort or None)."""
    import torch

    from synthetic.cohorts import make_cohort

    t0 = time.perf_counter()
    images = torch.from_numpy(make_cohort(w, workers=workers)).to(dev)
    log(f"generated {w.name} in {time.perf_counter() - t0:.1f} s ({workers} processes)")
    params = D.SweepParams(metric=w.metric, win=w.win, ncc_eps=w.ncc_eps, lam=w.lam,
                           smooth_sigma=w.smooth_sigma, n_sq=w.n_sq, k2=w.k2, lr=w.lr,
                           beta1=w.beta1, beta2=w.beta2, adam_eps=w.adam_eps, batch=batch)
    cohort = D.Cohort(images, params, device_step=graph)
    torch.cuda.synchronize()
    tuned = None
    if autotune:
        t0 = time.perf_counter()
        tuned = cohort.autotune()
        log(f"{w.name}: autotuned launch shapes {tuned} in {time.perf_counter() - t0:.1f} s")
    for i in range(warmup):
        cohort.sweep()
        torch.cuda.synchronize()
        log(f"{w.name}: warmup sweep {i + 1}/{warmup}: F = {cohort.group_loss():.6f}")
    if profile:
        D.profile_reset()
        D.profile_enable(True)
    torch.cuda.synchronize()
    if graph:
        sweep_graph = cohort.capture()
        torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        if graph:
            sweep_graph.replay()
        else:
            cohort.sweep()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    log(f"{w.name}: {steps} timed sweeps in {t1 - t0:.2f} s, F = {cohort.group_loss():.6f}")
    kernels = {}
    if profile:
        D.profile_enable(False)
        prof = D.profile_collect()
        algo = algorithmic_bytes(w, batch)
        for cls, (cnt, ms) in prof.items():
            if cnt == 0:
                continue
            entry = {"launches": cnt, "ms": round(ms, 4), "avg_us": round(1e3 * ms / cnt, 2)}
            if cls in algo:
                entry["algo_GB_per_launch"] = round(algo[cls] * steps / cnt / 1e9, 4)
                entry["GB/s"] = round(algo[cls] * steps / (ms * 1e-3) / 1e9, 1)
            kernels[cls] = entry
    ms_per_step = (t1 - t0) * 1e3 / steps
    res = {
        "workload": w.name,
        "ms_per_step": round(ms_per_step, 3),
        "value": round(w.n * w.voxels * w.k2 / (ms_per_step * 1e-3), 1),
        "group_loss": cohort.group_loss(),
        "kernels": kernels,
    }
    if tuned is not None:
        res["autotuned"] = {"squaring_tz": tuned[0], "window_tz": tuned[1], "fused": tuned[2]}
    if not keep:
        del cohort, images
        torch.cuda.empty_cache()
        cohort = None
    return res, cohort


def roofline_of(w, kernels, attainable):
    """Roofline position of the kernel class that takes the most time."""
    dom = max((c for c in kernels if "GB/s" in kernels[c]), key=lambda c: kernels[c]["ms"])
    achieved = kernels[dom]["GB/s"]
    out = {
        "kernel": dom,
        "bound": "hbm",
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": measured_traffic(w.name, dom),
        "traffic_unit": "GB per launch (HBM, from counters)",
        "algo_GB_per_launch": kernels[dom]["algo_GB_per_launch"],
        "avg_us": kernels[dom]["avg_us"],
    }
    if attainable:
        out["attainable_copy"] = attainable["copy"]
        out["frac_attainable"] = round(achieved / attainable["copy"], 4)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed sweeps")
    ap.add_argument("--warmup", type=int, default=1, help="untimed sweeps before timing")
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--batch", type=int, default=None,
                    help=f"subjects per launch (default: all, at most {MAX_BATCH})")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="skip the per-kernel event timing")
    ap.add_argument("--no-second", action="store_true",
                    help=f"skip the second workload ({SECOND_WORKLOAD})")
    ap.add_argument("--no-time-to-loss", action="store_true",
                    help="skip the warm-start time-to-loss trial")
    ap.add_argument("--no-attainable", action="store_true",
                    help="skip the copy/read/write bandwidth measurement")
    ap.add_argument("--autotune", action="store_true",
                    help="run the library's autotuner on the cohort before timing")
    ap.add_argument("--graph", action="store_true",
                    help="capture one sweep in a HIP graph and time its replays")
    ap.add_argument("--extras", action="store_true",
                    help="also time the method's other branches (median and stochastic atlas, "
                         "one-shot segmentation, pyramid resampling, the network) on the same "
                         "cohort")
    ap.add_argument("--unet-rates", action="store_true",
                    help="only time the warm-start network (forward and one training step) "
                         "on one cohort of the time-to-loss workload, print its rates, exit")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 1 GiB copy stream (k_bw_copy) first: a kernel of known "
                         "traffic for calibrating HBM byte counters")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU: the DARC path here runs on a single MI355X and has "
              f"no multi-GPU mode (asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)

    from synthetic.cohorts import WORKLOADS

    w = WORKLOADS[args.workload]
    batch = args.batch if args.batch is not None else (MAX_BATCH if w.n > MAX_BATCH else 0)
    # large cohorts are generated in a process pool (same images), sized to the
    # CPU share of one GPU
    workers = min(16, os.cpu_count() or 1)
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle sample")
        cpu = cpu_baseline(w)
        log(f"CPU oracle: {cpu['sample']}")

    import torch

    from paper_2508_10743_amd import darc as D

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    D.lib()
    if args.unet_rates:
        from paper_2508_10743_amd import unet as N
        from paper_2508_10743_amd import warmstart as WS
        from synthetic.cohorts import make_cohort, random_velocity

        wt = WORKLOADS[TTL_WORKLOAD]
        imgs = torch.from_numpy(make_cohort(wt)).to(dev)
        v = torch.from_numpy(random_velocity(7, wt.n, wt.dims, 2.0)).to(dev)
        t = WS.Triple(D.atlas_update(imgs, None), imgs, v)
        rates = WS.unet_rates(N.UNet(seed=0, device=dev), t)
        print(json.dumps({"workload": wt.name, "unet": rates}), flush=True)
        return
    attainable = None
    if not args.no_attainable:
        attainable = attainable_bandwidth(dev)
        log(f"attainable bandwidth (GB/s): {attainable}")
    if args.calib_copy:
        import ctypes

        a = torch.full((1 << 28,), 1.0, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        # k_bw_copy reads 1 GiB and writes 1 GiB
        assert D.lib().darc_bw_copy(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()),
                                    1 << 30, 0,
                                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)) == 0
        torch.cuda.synchronize()
        del a, b

    profile = not args.no_profile and not args.graph
    res, cohort = run_workload(D, w, batch, args.steps, args.warmup, dev, profile=profile,
                               graph=args.graph, keep=args.extras,
                               workers=workers if w.n >= 32 else 1, autotune=args.autotune)
    roofline = roofline_of(w, res["kernels"], attainable) if profile else None
    extras = time_extras(D, cohort, w) if args.extras else None
    del cohort
    torch.cuda.empty_cache()

    second = None
    if not args.no_second and args.workload == DEFAULT_WORKLOAD:
        w2 = WORKLOADS[SECOND_WORKLOAD]
        r2, _ = run_workload(D, w2, 0, max(3, args.steps // 4), 1, dev, profile=True,
                             workers=workers)
        second = {k: r2[k] for k in ("workload", "ms_per_step", "value", "group_loss")}
        second["n_subjects"] = w2.n
        second["dims"] = list(w2.dims)
        second["roofline"] = roofline_of(w2, r2["kernels"], attainable)
        second["kernels"] = r2["kernels"]

    ttl = None
    if not args.no_time_to_loss and args.workload == DEFAULT_WORKLOAD:
        from paper_2508_10743_amd import warmstart as WS

        log(f"time-to-loss trial on {TTL_WORKLOAD}")
        t0 = time.perf_counter()
        # 500 training cohorts of 4: 2000 (atlas, subject) pairs
        ttl = WS.time_to_loss(WORKLOADS[TTL_WORKLOAD], range(2000, 2500), range(3000, 3008), dev,
                              workers=workers, progress=log)
        log(f"time-to-loss trial took {time.perf_counter() - t0:.1f} s: plain "
            f"{ttl['plain_s']:.3f} s, warm {ttl.get('warm_s')} s "
            f"({ttl['warm_reached']}/{ttl['test_cohorts']} reached)")

    out = {
        "metric": "subject-voxel-iters/s per DARC sweep",
        "value": res["value"],
        "unit": "subject-voxel-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": w.name,
            "level": "full resolution",
            "n_subjects": w.n,
            "dims": list(w.dims),
            "metric": f"{w.metric}{w.win if w.metric == 'lncc' else ''}",
            "k2": w.k2,
            "n_sq": w.n_sq,
            "smooth_sigma": w.smooth_sigma,
            "lam": w.lam,
            "batch": batch or w.n,
        },
        "group_loss": res["group_loss"],
        "roofline": roofline,
        "attainable_GBs": attainable,
        "cpu_baseline": cpu,
        "time_to_loss": ttl,
        "autotuned": res.get("autotuned"),
        "second_workload": second,
        "kernels": res["kernels"],
    }
    if extras is not None:
        out["extras"] = extras
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
