"""Seeded synthetic cohorts (images + run settings) for the DARC hot path.

The paper evaluates on OASIS brains (192x160x224) and cardiac MRI
(96x128x128) (Section 5, implementation details).  Neither dataset is
available, so every workload here is a seeded phantom of the stated shape:

* ``blobs``: a cohort template made of 8 Gaussian blobs (sigma 2-5 voxels,
  amplitude U[0,1], centres U[0.2,0.8]*dims), drawn once per cohort so that a
  group atlas exists;
* ``brain``: three nested smoothed ellipsoids with levels 0.2/0.5/0.8 plus
  N(0, 0.02^2) noise per subject;
* ``compartments``: an outer ellipsoid and four offset inner ones at
  0.2/0.35/0.5/0.65/0.8.

Subject i is the template evaluated at ``x + d_i(x)``, where ``d_i`` is a
smooth random displacement drawn as a sum of random Fourier features with a
Gaussian spectrum (correlation length ``corr_len`` voxels) scaled so that
``max_x |d_i(x)|_2`` equals the stated maximum displacement.  The template is
a closed-form function of continuous coordinates, so no resampling is needed
to build a subject.  All generation runs in FP64 and is cast to FP32 at the end.
"""

from __future__ import annotations

import dataclasses
from typing import Dict, Optional, Tuple

import numpy as np
from scipy.special import erfc


@dataclasses.dataclass(frozen=True)
class Workload:
    """A synthetic cohort plus the DARC settings it is run with."""

    name: str
    n: int
    dims: Tuple[int, int, int]
    phantom: str            # "blobs" | "brain" | "compartments"
    max_disp: float         # voxels, max |d(x)|_2 of the subject deformation
    corr_len: float         # voxels, correlation length of the deformation
    noise_sd: float
    seed: int
    # method settings (Eq. (2)-(3) and Algorithm 1 of the paper)
    metric: str             # "mse" | "lncc"
    win: int                # LNCC window (odd)
    ncc_eps: float
    lam: float              # diffusion regulariser weight
    smooth_sigma: float     # Gaussian smoothing of v after each step (0 = off)
    n_sq: int               # scaling-and-squaring steps
    k1: int                 # sweeps
    k2: int                 # inner iterations per subject per sweep
    lr: float = 1e-2
    beta1: float = 0.9
    beta2: float = 0.999
    adam_eps: float = 1e-8

    @property
    def voxels(self) -> int:
        return int(np.prod(self.dims))


WORKLOADS: Dict[str, Workload] = {
    w.name: w
    for w in [
        Workload("blobs-4x32^3-mse", 4, (32, 32, 32), "blobs", 3.0, 4.0, 0.0, 1001,
                 "mse", 9, 1e-5, 0.01, 0.0, 7, 10, 5),
        Workload("brain-16x160x192x160-lncc9", 16, (160, 192, 160), "brain", 8.0, 8.0, 0.02,
                 1002, "lncc", 9, 1e-5, 0.0, 1.5, 7, 20, 5),
        Workload("blobs-64x128^3-lncc9", 64, (128, 128, 128), "blobs", 3.0, 4.0, 0.0, 1003,
                 "lncc", 9, 1e-5, 0.01, 0.0, 7, 10, 5),
        Workload("blobs-4x96x112x96-mse", 4, (96, 112, 96), "blobs", 3.0, 4.0, 0.0, 1004,
                 "mse", 9, 1e-5, 0.01, 0.0, 7, 10, 5),
        Workload("compartments-200x160x192x224-lncc9", 200, (160, 192, 224), "compartments",
                 10.0, 8.0, 0.0, 1005, "lncc", 9, 1e-5, 0.0, 1.5, 7, 30, 5),
    ]
}


# --------------------------------------------------------------------------
# random smooth fields


def smooth_random_field(rng: np.random.Generator, dims, max_norm: float,
                        corr_len: float, n_modes: int = 32) -> np.ndarray:
    """Random smooth 3-vector field ``[3, D0, D1, D2]`` (FP64).

    Each component is ``Re sum_m z_m exp(i k_m . x)`` with wave vectors
    ``k_m ~ N(0, I / corr_len^2)`` and complex normal ``z_m`` (random Fourier
    features of a Gaussian covariance).  The field is scaled so that
    ``max_x |f(x)|_2 == max_norm``.
    """
    d0, d1, d2 = dims
    axes = [np.arange(d, dtype=np.float64) for d in dims]
    out = np.empty((3, d0, d1, d2), dtype=np.float64)
    for c in range(3):
        k = rng.normal(0.0, 1.0 / corr_len, size=(n_modes, 3))
        z = rng.normal(size=n_modes) + 1j * rng.normal(size=n_modes)
        e0 = z[:, None] * np.exp(1j * k[:, 0:1] * axes[0][None, :])    # [M, D0]
        e1 = np.exp(1j * k[:, 1:2] * axes[1][None, :])                 # [M, D1]
        e2 = np.exp(1j * k[:, 2:3] * axes[2][None, :])                 # [M, D2]
        ab = (e0[:, :, None] * e1[:, None, :]).reshape(n_modes, d0 * d1)  # [M, D0*D1]
        out[c] = (ab.T @ e2).real.reshape(d0, d1, d2)
    norm = np.sqrt((out ** 2).sum(axis=0)).max()
    if norm > 0:
        out *= max_norm / norm
    return out


# --------------------------------------------------------------------------
# closed-form templates


def blob_template_params(rng: np.random.Generator, dims, n_blobs: int = 8):
    dims_a = np.asarray(dims, dtype=np.float64)
    centres = rng.uniform(0.2, 0.8, size=(n_blobs, 3)) * dims_a
    sigmas = rng.uniform(2.0, 5.0, size=n_blobs)
    amps = rng.uniform(0.0, 1.0, size=n_blobs)
    return centres, sigmas, amps


def eval_blobs(params, y: np.ndarray) -> np.ndarray:
    """Sum of Gaussian blobs at continuous positions ``y`` (``[3, ...]``)."""
    centres, sigmas, amps = params
    out = np.zeros(y.shape[1:], dtype=np.float64)
    for c, s, a in zip(centres, sigmas, amps):
        r2 = sum((y[d] - c[d]) ** 2 for d in range(3))
        out += a * np.exp(-r2 / (2.0 * s * s))
    return out


def _soft_ellipsoid(y: np.ndarray, centre, radii, edge_sigma: float) -> np.ndarray:
    rho = np.sqrt(sum(((y[d] - centre[d]) / radii[d]) ** 2 for d in range(3)))
    signed = (rho - 1.0) * float(np.mean(radii))       # ~ signed distance in voxels
    return 0.5 * erfc(signed / (np.sqrt(2.0) * edge_sigma))


def eval_nested_ellipsoids(dims, y: np.ndarray, edge_sigma: float = 2.0) -> np.ndarray:
    """Brain-like phantom: nested ellipsoids with tissue levels 0.2/0.5/0.8."""
    dims_a = np.asarray(dims, dtype=np.float64)
    centre = (dims_a - 1.0) / 2.0
    r1 = np.array([0.38, 0.40, 0.38]) * dims_a
    s1 = _soft_ellipsoid(y, centre, r1, edge_sigma)
    s2 = _soft_ellipsoid(y, centre, 0.7 * r1, edge_sigma)
    s3 = _soft_ellipsoid(y, centre, 0.4 * r1, edge_sigma)
    return 0.2 * s1 + 0.3 * s2 + 0.3 * s3


def eval_compartments(dims, y: np.ndarray, edge_sigma: float = 2.0) -> np.ndarray:
    """Five-compartment phantom: outer ellipsoid + four offset inner ones."""
    dims_a = np.asarray(dims, dtype=np.float64)
    centre = (dims_a - 1.0) / 2.0
    r0 = np.array([0.40, 0.42, 0.40]) * dims_a
    out = 0.2 * _soft_ellipsoid(y, centre, r0, edge_sigma)
    offsets = np.array([[0.12, 0.0, 0.0], [-0.12, 0.0, 0.0], [0.0, 0.14, 0.1], [0.0, -0.14, -0.1]])
    for lvl, off in zip([0.35, 0.5, 0.65, 0.8], offsets):
        out += (lvl - 0.2) * _soft_ellipsoid(y, centre + off * dims_a, 0.12 * dims_a, edge_sigma)
    return out


# --------------------------------------------------------------------------
# cohorts


def _subject(w: Workload, n: int, dims, seed: int, i: int) -> np.ndarray:
    """Subject ``i`` of the cohort: its own spawned seed, so that subjects can
    be generated in any order or process with identical results."""
    template_ss, *subject_ss = np.random.SeedSequence(seed).spawn(n + 1)
    if w.phantom == "blobs":
        params = blob_template_params(np.random.default_rng(template_ss), dims)
        evaluate = lambda y: eval_blobs(params, y)  # noqa: E731
    elif w.phantom == "brain":
        evaluate = lambda y: eval_nested_ellipsoids(dims, y)  # noqa: E731
    elif w.phantom == "compartments":
        evaluate = lambda y: eval_compartments(dims, y)  # noqa: E731
    else:
        raise ValueError(f"unknown phantom {w.phantom!r}")
    rng = np.random.default_rng(subject_ss[i])
    grid = np.stack(np.meshgrid(*[np.arange(d, dtype=np.float64) for d in dims], indexing="ij"))
    disp = smooth_random_field(rng, dims, w.max_disp, w.corr_len)
    img = evaluate(grid + disp)
    if w.noise_sd > 0:
        img += rng.normal(0.0, w.noise_sd, size=img.shape)
    return img.astype(np.float32)


def make_cohort(w: Workload, n: Optional[int] = None, dims=None, seed: Optional[int] = None,
                workers: int = 1):
    """Return ``images`` ``[n, D0, D1, D2]`` FP32 for workload ``w``.

    ``n``/``dims``/``seed`` override the workload's values (smaller test cases
    with the same recipe).  ``workers`` > 1 generates subjects in that many
    processes (same images).
    """
    n = w.n if n is None else n
    dims = tuple(w.dims if dims is None else dims)
    seed = w.seed if seed is None else seed
    images = np.empty((n,) + dims, dtype=np.float32)
    if workers > 1 and n > 1:
        from concurrent.futures import ProcessPoolExecutor
        with ProcessPoolExecutor(max_workers=min(workers, n)) as ex:
            futs = [ex.submit(_subject, w, n, dims, seed, i) for i in range(n)]
            for i, f in enumerate(futs):
                images[i] = f.result()
    else:
        for i in range(n):
            images[i] = _subject(w, n, dims, seed, i)
    return images


def make_cohorts(w: Workload, seeds, n: Optional[int] = None, dims=None, workers: int = 1):
    """``make_cohort(w, n, dims, seed)`` for every seed in ``seeds``, with the
    subjects of all cohorts spread over ``workers`` processes (same images as
    one cohort at a time)."""
    n = w.n if n is None else n
    dims = tuple(w.dims if dims is None else dims)
    seeds = [int(s) for s in seeds]
    out = [np.empty((n,) + dims, dtype=np.float32) for _ in seeds]
    jobs = [(c, i) for c in range(len(seeds)) for i in range(n)]
    if workers > 1 and len(jobs) > 1:
        from concurrent.futures import ProcessPoolExecutor
        with ProcessPoolExecutor(max_workers=min(workers, len(jobs))) as ex:
            futs = [ex.submit(_subject, w, n, dims, seeds[c], i) for c, i in jobs]
            for (c, i), f in zip(jobs, futs):
                out[c][i] = f.result()
    else:
        for c, i in jobs:
            out[c][i] = _subject(w, n, dims, seeds[c], i)
    return out


def _velocity(ss, dims, max_norm: float, corr_len: float) -> np.ndarray:
    return smooth_random_field(np.random.default_rng(ss), dims, max_norm,
                               corr_len).astype(np.float32)


def random_velocity(seed: int, n: int, dims, max_norm: float, corr_len: float = 4.0,
                    workers: int = 1) -> np.ndarray:
    """Seeded smooth velocity fields ``[n, 3, D0, D1, D2]`` FP32 for test inputs
    (``workers`` processes give the same fields)."""
    sss = np.random.SeedSequence(seed).spawn(n)
    dims = tuple(dims)
    out = np.empty((n, 3) + dims, dtype=np.float32)
    if workers > 1 and n > 1:
        from concurrent.futures import ProcessPoolExecutor
        with ProcessPoolExecutor(max_workers=min(workers, n)) as ex:
            futs = [ex.submit(_velocity, ss, dims, max_norm, corr_len) for ss in sss]
            for i, f in enumerate(futs):
                out[i] = f.result()
    else:
        for i, ss in enumerate(sss):
            out[i] = _velocity(ss, dims, max_norm, corr_len)
    return out


def random_volume(seed: int, shape, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """Seeded uniform FP32 array (test inputs such as upstream gradients)."""
    return np.random.default_rng(seed).uniform(lo, hi, size=shape).astype(np.float32)
