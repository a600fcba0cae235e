"""FP64 CPU oracle for the DARC hot path (test infrastructure only).

This module is the slow, plain reference that the HIP path is checked
against.  Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import it; the product path never does.  It shares no code with
the HIP library or its Python binding.

Everything follows Section 3 ("Methodology") of the paper, An Efficient
Model-Driven Groupwise Approach for Atlas Construction (DARC):

* objective: Eq. (1)-(2), sum over subjects of a dissimilarity between the
  warped subject and the atlas plus a diffusion regulariser, under the
  centrality constraint sum_i phi_i = 0;
* coordinate descent: Eq. (3) (per-subject argmin with the atlas fixed,
  centring, atlas argmin), Algorithm 1 (``diffeo_pairwise_reg`` and
  ``main``);
* phi = Exp(v) by scaling and squaring seven times (Section 3,
  "Diffeomorphisms");
* centrality activation: fourth line of Eq. (3) (Section 3, "Centrality
  activation function");
* MSE atlas closed form: the first equation of Section 3, "Dissimilarity
  metrics" (mean of the warped subjects); L1 atlas closed form: the second
  equation there (voxelwise median); NCC atlas by minibatch stochastic
  gradient descent: the last paragraph there and Algorithm 1
  (``SGD_for_atlas``);
* one-shot segmentation, Section 4, Eq. (oneshot): atlas labels carried to
  subject i by Exp(-v_i), scored by Dice (Section 5);
* factor-2 resampling between levels of a coarse-to-fine schedule (not in the
  paper: a reading for large cohorts, see ``down2``/``up2``).

Where the paper is silent this oracle reads it as follows: positions are in
voxel units with voxel centres at integers; sampling is trilinear, with zero
padding for images and border clamping for fields; the deformation phi is
handled as a displacement u = phi - id (the only reading under which
sum_i phi_i = 0 makes sense); NCC is the squared local NCC over a centred odd
window with zero-padded sums; the diffusion regulariser acts on the
displacement and is a mean of squared forward differences; the optimiser is
Adam with Kingma & Ba's constants (lr 1e-2 as in Section 5); the velocities
and Adam moments persist across sweeps.

Conventions: a volume is ``[D0, D1, D2]`` (D2 fastest), a field is
``[3, D0, D1, D2]`` whose component c displaces axis c, positions are voxel
coordinates with voxel centres at integers.  All arithmetic is FP64.
"""

from __future__ import annotations

import dataclasses
from typing import List, Tuple

import numpy as np

# ---------------------------------------------------------------------------
# trilinear sampling (the warping operator "o" of Eq. (2))


def identity_grid(dims) -> np.ndarray:
    """Voxel coordinates ``[3, D0, D1, D2]`` (the identity map x)."""
    return np.stack(np.meshgrid(*[np.arange(d, dtype=np.float64) for d in dims], indexing="ij"))


def _cells_zero(pos: np.ndarray):
    """Cell index and fraction per axis for zero-padded sampling."""
    i = np.floor(pos)
    return i.astype(np.int64), pos - i


def _cells_border(pos: np.ndarray, dims):
    """Cell index, fraction and clamp flag per axis for border sampling.

    The position is clamped into [0, D-1]; the cell is [min(floor p, D-2), +1]
    so that p == D-1 falls in the last cell with fraction 1.
    """
    idx, frac, clamped = [], [], []
    for d in range(3):
        p = pos[d]
        D = dims[d]
        lo, hi = p < 0.0, p > D - 1.0
        pc = np.clip(p, 0.0, D - 1.0)
        i = np.minimum(np.floor(pc), D - 2).astype(np.int64)
        idx.append(i)
        frac.append(pc - i)
        clamped.append(lo | hi)
    return np.stack(idx), np.stack(frac), np.stack(clamped)


def _corner_values(vol: np.ndarray, idx: np.ndarray, zero_pad: bool):
    """Return the 8 corner values ``c[a][b][c]`` of ``vol`` around ``idx``."""
    dims = vol.shape
    out = {}
    for a in (0, 1):
        for b in (0, 1):
            for c in (0, 1):
                j0, j1, j2 = idx[0] + a, idx[1] + b, idx[2] + c
                if zero_pad:
                    ok = ((j0 >= 0) & (j0 < dims[0]) & (j1 >= 0) & (j1 < dims[1])
                          & (j2 >= 0) & (j2 < dims[2]))
                    val = vol[np.clip(j0, 0, dims[0] - 1), np.clip(j1, 0, dims[1] - 1),
                              np.clip(j2, 0, dims[2] - 1)]
                    out[a, b, c] = np.where(ok, val, 0.0)
                else:
                    out[a, b, c] = vol[j0, j1, j2]
    return out


def _lerp(a, b, t):
    return a + t * (b - a)


def _trilinear_from_corners(cv, t):
    """Nested linear interpolation along axis 2, then 1, then 0; returns the
    value and its derivatives with respect to the three fractions."""
    t0, t1, t2 = t
    c00 = _lerp(cv[0, 0, 0], cv[0, 0, 1], t2)
    c01 = _lerp(cv[0, 1, 0], cv[0, 1, 1], t2)
    c10 = _lerp(cv[1, 0, 0], cv[1, 0, 1], t2)
    c11 = _lerp(cv[1, 1, 0], cv[1, 1, 1], t2)
    c0 = _lerp(c00, c01, t1)
    c1 = _lerp(c10, c11, t1)
    val = _lerp(c0, c1, t0)
    d0 = c1 - c0
    d1 = _lerp(c01 - c00, c11 - c10, t0)
    e00 = cv[0, 0, 1] - cv[0, 0, 0]
    e01 = cv[0, 1, 1] - cv[0, 1, 0]
    e10 = cv[1, 0, 1] - cv[1, 0, 0]
    e11 = cv[1, 1, 1] - cv[1, 1, 0]
    d2 = _lerp(_lerp(e00, e01, t1), _lerp(e10, e11, t1), t0)
    return val, np.stack([d0, d1, d2])


def sample_zero(img: np.ndarray, pos: np.ndarray):
    """Trilinear sample of an image with zero padding.

    Returns ``(value, dvalue/dpos [3, ...])``; the derivative is that of the
    interpolant inside the cell [floor p, floor p + 1] (right-sided at
    integer positions).
    """
    idx, t = _cells_zero(pos)
    cv = _corner_values(img, idx, zero_pad=True)
    return _trilinear_from_corners(cv, t)


def sample_border(field: np.ndarray, pos: np.ndarray):
    """Trilinear sample of every component of ``field`` with border clamping.

    Returns ``(values [C, ...], jac [C, 3, ...])`` where ``jac[c, d]`` is the
    derivative of component c with respect to position axis d (zero on an
    axis whose coordinate was clamped).
    """
    dims = field.shape[1:]
    idx, t, clamped = _cells_border(pos, dims)
    vals, jacs = [], []
    for c in range(field.shape[0]):
        cv = _corner_values(field[c], idx, zero_pad=False)
        v, d = _trilinear_from_corners(cv, t)
        d = np.where(clamped, 0.0, d)
        vals.append(v)
        jacs.append(d)
    return np.stack(vals), np.stack(jacs)


def scatter_border(pos: np.ndarray, values: np.ndarray, dims) -> np.ndarray:
    """Adjoint of ``sample_border`` with respect to the sampled field.

    Every sample position p(x) sends ``w_k(x) * values[:, x]`` to each of its
    8 (clamped) corners k, with trilinear weights w_k.  ``values`` is
    ``[C, ...]`` with the same trailing shape as ``pos[0]``.
    """
    idx, t, _ = _cells_border(pos, dims)
    V = int(np.prod(dims))
    C = values.shape[0]
    flat_vals = values.reshape(C, -1)
    out = np.zeros((C, V), dtype=np.float64)
    lin_all, w_all = [], []
    for a in (0, 1):
        for b in (0, 1):
            for c in (0, 1):
                lin = ((idx[0] + a) * dims[1] + (idx[1] + b)) * dims[2] + (idx[2] + c)
                w = ((t[0] if a else 1.0 - t[0]) * (t[1] if b else 1.0 - t[1])
                     * (t[2] if c else 1.0 - t[2]))
                lin_all.append(lin.reshape(-1))
                w_all.append(w.reshape(-1))
    lin_all = np.concatenate(lin_all)
    w_all = np.concatenate(w_all)
    for ch in range(C):
        out[ch] = np.bincount(lin_all, weights=w_all * np.tile(flat_vals[ch], 8), minlength=V)
    return out.reshape((C,) + tuple(dims))


# ---------------------------------------------------------------------------
# Exp(v) by scaling and squaring (Section 3, "Diffeomorphisms")


def exp_svf(v: np.ndarray, n_sq: int = 7) -> Tuple[np.ndarray, List[np.ndarray]]:
    """Displacement u = Exp(v) - id by scaling and squaring.

    u_0 = v / 2^N; u_{t+1}(x) = u_t(x) + u_t(x + u_t(x)) (the map composed with
    itself), N = ``n_sq`` times.  Returns ``(u_N, [u_0, ..., u_{N-1}])``.
    """
    v = np.asarray(v, dtype=np.float64)
    dims = v.shape[1:]
    x = identity_grid(dims)
    u = v / (2.0 ** n_sq)
    steps = []
    for _ in range(n_sq):
        steps.append(u)
        s, _ = sample_border(u, x + u)
        u = u + s
    return u, steps


def squaring_step(u_t: np.ndarray) -> np.ndarray:
    """One self-composition u_t -> u_{t+1} (used to check single GPU steps)."""
    u_t = np.asarray(u_t, dtype=np.float64)
    s, _ = sample_border(u_t, identity_grid(u_t.shape[1:]) + u_t)
    return u_t + s


def squaring_step_bwd(u_t: np.ndarray, g_next: np.ndarray) -> np.ndarray:
    """Adjoint of one self-composition: g_t = (d u_{t+1} / d u_t)^T g_{t+1}.

    d u_{t+1}(x) = d u_t(x) + J_t(x) d u_t(x) + S(d u_t, p_t(x)), with J_t the
    position derivative of the sampled field at p_t(x) = x + u_t(x).  The
    transpose gives the direct term, J_t^T g and the scatter of g through the
    trilinear weights.
    """
    u_t = np.asarray(u_t, dtype=np.float64)
    g_next = np.asarray(g_next, dtype=np.float64)
    dims = u_t.shape[1:]
    pos = identity_grid(dims) + u_t
    _, jac = sample_border(u_t, pos)                 # [c, d, ...]
    jtg = np.einsum("cd...,c...->d...", jac, g_next)
    return g_next + jtg + scatter_border(pos, g_next, dims)


def squaring_step_bwd_at(u_t: np.ndarray, g_next: np.ndarray, points: np.ndarray) -> np.ndarray:
    """``squaring_step_bwd(u_t, g_next)`` evaluated only at the voxels
    ``points`` (``[3, P]`` integer coordinates); returns ``[3, P]``.

    Same sum as the full adjoint, taken one output voxel y at a time: the
    direct term g(y) + J_t(y)^T g(y), plus w_k(x) g(x) over every source x
    whose cell has y as corner k.  Such an x satisfies |x_d + u_d(x) - y_d| < 1
    (or is clamped onto y), so |x_d - y_d| <= max|u_d| + 1 and a window of that
    radius around y contains all of them.
    """
    u_t = np.asarray(u_t, dtype=np.float64)
    g_next = np.asarray(g_next, dtype=np.float64)
    dims = u_t.shape[1:]
    pts = np.asarray(points, dtype=np.int64)
    y = pts.astype(np.float64)
    uy = u_t[:, pts[0], pts[1], pts[2]]
    gy = g_next[:, pts[0], pts[1], pts[2]]
    _, jac = sample_border(u_t, y + uy)
    out = gy + np.einsum("cdp,cp->dp", jac, gy)
    R = [int(np.ceil(np.abs(u_t[d]).max())) + 1 for d in range(3)]
    offs = np.stack(np.meshgrid(*[np.arange(-r, r + 1) for r in R], indexing="ij")).reshape(3, -1)
    for p in range(pts.shape[1]):
        xs = pts[:, p:p + 1] + offs
        keep = np.all((xs >= 0) & (xs < np.array(dims)[:, None]), axis=0)
        xs = xs[:, keep]
        ux = u_t[:, xs[0], xs[1], xs[2]]
        idx, t, _ = _cells_border(xs.astype(np.float64) + ux, dims)
        gx = g_next[:, xs[0], xs[1], xs[2]]
        for a in (0, 1):
            for b in (0, 1):
                for c in (0, 1):
                    hit = ((idx[0] + a == pts[0, p]) & (idx[1] + b == pts[1, p])
                           & (idx[2] + c == pts[2, p]))
                    w = ((t[0] if a else 1.0 - t[0]) * (t[1] if b else 1.0 - t[1])
                         * (t[2] if c else 1.0 - t[2]))
                    out[:, p] += (gx * (w * hit)).sum(axis=1)
    return out


def exp_svf_bwd(steps: List[np.ndarray], g_u: np.ndarray) -> np.ndarray:
    """Gradient with respect to v of a loss whose gradient w.r.t. u_N is ``g_u``."""
    n_sq = len(steps)
    g = np.asarray(g_u, dtype=np.float64)
    for t in reversed(range(n_sq)):
        g = squaring_step_bwd(steps[t], g)
    return g / (2.0 ** n_sq)


# ---------------------------------------------------------------------------
# warping, dissimilarities, regulariser


def warp3d(img: np.ndarray, u: np.ndarray) -> np.ndarray:
    """(I o phi)(x) = I(x + u(x)), trilinear, zero outside the volume."""
    img = np.asarray(img, dtype=np.float64)
    val, _ = sample_zero(img, identity_grid(img.shape) + np.asarray(u, dtype=np.float64))
    return val


def warp3d_bwd(img: np.ndarray, u: np.ndarray, g_out: np.ndarray) -> np.ndarray:
    """Gradient w.r.t. u: g_out(x) * grad_p I(p) at p = x + u(x)."""
    img = np.asarray(img, dtype=np.float64)
    _, grad = sample_zero(img, identity_grid(img.shape) + np.asarray(u, dtype=np.float64))
    return np.asarray(g_out, dtype=np.float64)[None] * grad


def mse(warped: np.ndarray, atlas: np.ndarray):
    """MSE dissimilarity (Section 3, "Dissimilarity metrics") and its gradient."""
    diff = np.asarray(warped, dtype=np.float64) - np.asarray(atlas, dtype=np.float64)
    V = diff.size
    return float((diff ** 2).sum() / V), 2.0 * diff / V


def l1(warped: np.ndarray, atlas: np.ndarray):
    """L1 dissimilarity mean_x |Iw - A| (Section 3, "Dissimilarity metrics")
    and its subgradient sign(Iw - A) / V, taking 0 where Iw = A."""
    diff = np.asarray(warped, dtype=np.float64) - np.asarray(atlas, dtype=np.float64)
    V = diff.size
    return float(np.abs(diff).sum() / V), np.sign(diff) / V


def box_sum(f: np.ndarray, win: int) -> np.ndarray:
    """Sum of f over the win^3 cube centred at each voxel, zero outside."""
    r = win // 2
    out = np.asarray(f, dtype=np.float64)
    for ax in range(3):
        pad = [(0, 0)] * 3
        pad[ax] = (r + 1, r)
        c = np.cumsum(np.pad(out, pad), axis=ax)
        D = out.shape[ax]
        hi = np.take(c, np.arange(2 * r + 1, 2 * r + 1 + D), axis=ax)
        lo = np.take(c, np.arange(0, D), axis=ax)
        out = hi - lo
    return out


def lncc(warped: np.ndarray, atlas: np.ndarray, win: int = 9, eps: float = 1e-5):
    """Squared local NCC dissimilarity D = -mean_x cc(x) and dD/dwarped.

    Window statistics use zero-padded win^3 sums with the fixed count
    N = win^3; cc = cross^2 / (Ivar * Jvar + eps).
    """
    I = np.asarray(warped, dtype=np.float64)
    J = np.asarray(atlas, dtype=np.float64)
    N = float(win ** 3)
    V = I.size
    S_I, S_J = box_sum(I, win), box_sum(J, win)
    S_II, S_JJ, S_IJ = box_sum(I * I, win), box_sum(J * J, win), box_sum(I * J, win)
    cross = S_IJ - S_I * S_J / N
    ivar = S_II - S_I * S_I / N
    jvar = S_JJ - S_J * S_J / N
    den = ivar * jvar + eps
    cc = cross * cross / den
    loss = -float(cc.sum()) / V
    alpha = 2.0 * cross / den
    beta = 2.0 * cross * cross * jvar / (den * den)
    ibar, jbar = S_I / N, S_J / N
    grad = -(J * box_sum(alpha, win) - box_sum(alpha * jbar, win)
             - I * box_sum(beta, win) + box_sum(beta * ibar, win)) / V
    return loss, grad


def diffusion_reg(u: np.ndarray):
    """Diffusion regulariser ||grad phi||^2 of Eq. (2) on the displacement.

    R(u) = (1/3) sum_d mean over components and voxels with a forward
    neighbour along d of (u_c(x + e_d) - u_c(x))^2.  Returns ``(R, dR/du)``.
    """
    u = np.asarray(u, dtype=np.float64)
    dims = u.shape[1:]
    V = int(np.prod(dims))
    R = 0.0
    g = np.zeros_like(u)
    for d in range(3):
        cnt = 3.0 * (dims[d] - 1) * (V // dims[d])
        diff = np.diff(u, axis=d + 1)                   # u(x+e_d) - u(x)
        R += float((diff ** 2).sum()) / cnt / 3.0
        w = 2.0 / cnt / 3.0
        sl_hi = [slice(None)] * 4
        sl_lo = [slice(None)] * 4
        sl_hi[d + 1] = slice(1, None)
        sl_lo[d + 1] = slice(None, -1)
        g[tuple(sl_hi)] += w * diff
        g[tuple(sl_lo)] -= w * diff
    return R, g


def gaussian_weights(sigma: float) -> np.ndarray:
    r = int(3.0 * sigma + 0.5)
    k = np.arange(-r, r + 1, dtype=np.float64)
    w = np.exp(-0.5 * k * k / (sigma * sigma))
    return w / w.sum()


def gauss_smooth(f: np.ndarray, sigma: float) -> np.ndarray:
    """Separable Gaussian smoothing of each component (leading axes kept),
    radius int(3 sigma + 0.5), replicated border."""
    w = gaussian_weights(sigma)
    r = len(w) // 2
    out = np.asarray(f, dtype=np.float64)
    nd = out.ndim
    for ax in range(nd - 3, nd):
        D = out.shape[ax]
        acc = np.zeros_like(out)
        for k in range(-r, r + 1):
            src = np.clip(np.arange(D) + k, 0, D - 1)
            acc += w[k + r] * np.take(out, src, axis=ax)
        out = acc
    return out


# ---------------------------------------------------------------------------
# optimiser, centring, atlas


def adam_step(v, m, s, g, t: int, lr=1e-2, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba, bias-corrected); ``t`` is the new step count."""
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * np.asarray(g, np.float64)
    s = beta2 * np.asarray(s, np.float64) + (1.0 - beta2) * np.asarray(g, np.float64) ** 2
    mhat = m / (1.0 - beta1 ** t)
    shat = s / (1.0 - beta2 ** t)
    v = np.asarray(v, np.float64) - lr * mhat / (np.sqrt(shat) + eps)
    return v, m, s


def center(u: np.ndarray):
    """Centrality activation, Eq. (3) fourth line: u_i - (1/n) sum_j u_j.

    ``u`` is ``[n, 3, D0, D1, D2]``; returns ``(u_hat, mean)``.
    """
    u = np.asarray(u, dtype=np.float64)
    mean = u.mean(axis=0)
    return u - mean[None], mean


def atlas_mean(images: np.ndarray, u_hat: np.ndarray) -> np.ndarray:
    """MSE atlas closed form: A = (1/n) sum_i I_i o phi_hat_i."""
    return np.mean([warp3d(images[i], u_hat[i]) for i in range(len(images))], axis=0)


def atlas_median(images: np.ndarray, u_hat: np.ndarray) -> np.ndarray:
    """L1 atlas closed form: the voxelwise median of the warped subjects.
    For even n every value between the two middle ones minimises the L1
    sum; this takes their average."""
    return np.median(np.stack([warp3d(images[i], u_hat[i]) for i in range(len(images))]), axis=0)


def lncc_atlas_grad(warped: np.ndarray, atlas: np.ndarray, win: int = 9, eps: float = 1e-5):
    """LNCC D(Iw, A) and dD/dA.  cc is symmetric in its two images, so the
    gradient with respect to A is the one with respect to the first image
    once the two are exchanged."""
    return lncc(atlas, warped, win, eps)


def atlas_sgd(warped: np.ndarray, atlas0: np.ndarray, epochs: int, batch: int, win: int = 9,
              eps: float = 1e-5, lr: float = 1e-2, beta1: float = 0.9, beta2: float = 0.999,
              adam_eps: float = 1e-8):
    """Minibatch stochastic atlas update for NCC (Section 3, last paragraph
    of "Dissimilarity metrics"; Algorithm 1, ``SGD_for_atlas``): ``epochs``
    passes over the warped subjects in minibatches of ``batch`` (in subject
    order); each minibatch takes one Adam step on A along the gradient of the
    minibatch mean of D(Iw_i, A).  A starts from ``atlas0``; the Adam moments
    start at zero.  Returns (A, per-minibatch losses taken before each step)."""
    warped = np.asarray(warped, dtype=np.float64)
    n = len(warped)
    A = np.array(atlas0, dtype=np.float64)
    m = np.zeros_like(A)
    s = np.zeros_like(A)
    t = 0
    losses = []
    for _ in range(epochs):
        for b0 in range(0, n, batch):
            idx = range(b0, min(n, b0 + batch))
            loss, g = 0.0, np.zeros_like(A)
            for i in idx:
                li, gi = lncc_atlas_grad(warped[i], A, win, eps)
                loss += li
                g += gi
            loss /= len(idx)
            g /= len(idx)
            t += 1
            A, m, s = adam_step(A, m, s, g, t, lr, beta1, beta2, adam_eps)
            losses.append(loss)
    return A, losses


# ---------------------------------------------------------------------------
# per-subject registration and one coordinate-descent sweep


@dataclasses.dataclass
class SweepParams:
    metric: str = "mse"          # "mse" | "lncc" | "l1"
    win: int = 9
    ncc_eps: float = 1e-5
    lam: float = 0.01
    smooth_sigma: float = 0.0    # Gaussian smoothing of v after each step (0 = off)
    n_sq: int = 7
    k2: int = 5
    lr: float = 1e-2
    beta1: float = 0.9
    beta2: float = 0.999
    adam_eps: float = 1e-8
    center_mode: str = "displacement"   # "displacement" | "velocity"
    reinit_v: bool = False
    atlas_mode: str = "auto"     # "mean" | "median" | "sgd"; auto: median for L1, else mean
    k3: int = 20                 # SGD atlas epochs
    atlas_batch: int = 4         # SGD atlas minibatch
    atlas_lr: float = 1e-2
    sgd_init: str = "warm"       # SGD atlas start: "warm" (A^k) | "initial" (A^0 of main)

    def resolved_atlas_mode(self) -> str:
        if self.atlas_mode != "auto":
            return self.atlas_mode
        return "median" if self.metric == "l1" else "mean"


def dissimilarity(warped, atlas, p: SweepParams):
    if p.metric == "mse":
        return mse(warped, atlas)
    if p.metric == "lncc":
        return lncc(warped, atlas, p.win, p.ncc_eps)
    if p.metric == "l1":
        return l1(warped, atlas)
    raise ValueError(p.metric)


def atlas_update(images, u_hat, atlas, p: SweepParams) -> np.ndarray:
    """Step 3 of a sweep: the closed form of the metric (mean for MSE,
    median for L1) or the minibatch stochastic update (NCC).

    Algorithm 1's ``SGD_for_atlas`` opens with ``A = initialize()``, which the
    paper leaves unspecified.  ``sgd_init = "warm"`` starts from the current
    atlas A^k; ``"initial"`` takes the literal reading: the same
    ``initialize()`` as ``main``, i.e. A^0, the mean of the unwarped
    subjects."""
    mode = p.resolved_atlas_mode()
    if mode == "mean":
        return atlas_mean(images, u_hat)
    if mode == "median":
        return atlas_median(images, u_hat)
    if mode == "sgd":
        warped = np.stack([warp3d(images[i], u_hat[i]) for i in range(len(images))])
        if p.sgd_init == "warm":
            start = atlas
        elif p.sgd_init == "initial":
            start = initial_atlas(images)
        else:
            raise ValueError(p.sgd_init)
        return atlas_sgd(warped, start, p.k3, p.atlas_batch, p.win, p.ncc_eps, p.atlas_lr,
                         p.beta1, p.beta2, p.adam_eps)[0]
    raise ValueError(mode)


def subject_loss_grad(img, v, atlas, p: SweepParams):
    """Loss of one subject, data term + lam * R (Algorithm 1, inner loop), and
    its gradient with respect to v."""
    u, steps = exp_svf(v, p.n_sq)
    w = warp3d(img, u)
    D, g_w = dissimilarity(w, atlas, p)
    g_u = warp3d_bwd(img, u, g_w)
    loss = D
    if p.lam != 0.0:
        R, g_r = diffusion_reg(u)
        loss += p.lam * R
        g_u = g_u + p.lam * g_r
    return loss, exp_svf_bwd(steps, g_u)


def group_loss(images, u_hat, atlas, p: SweepParams) -> float:
    """(1/n) sum_i [ D(I_i o phi_hat_i, A) + lam R(u_hat_i) ]: Eq. (2) at the
    centred deformations, divided by n."""
    total = 0.0
    for i in range(len(images)):
        D, _ = dissimilarity(warp3d(images[i], u_hat[i]), atlas, p)
        total += D
        if p.lam != 0.0:
            total += p.lam * diffusion_reg(u_hat[i])[0]
    return total / len(images)


def initial_atlas(images) -> np.ndarray:
    """A^0: mean of the unwarped subjects."""
    return np.asarray(images, dtype=np.float64).mean(axis=0)


def sweep(images, v, m, s, step: int, atlas, p: SweepParams):
    """One coordinate-descent sweep, Eq. (3) / Algorithm 1 ``main`` body.

    Step 1: K2 Adam iterations per subject against the fixed atlas (subjects
    are independent, so their order does not matter).  Step 2: centring.
    Step 3: the atlas update of ``atlas_update``.  Returns a dict with the new
    state, the inner losses ``[n, K2]`` (each taken before its step), the
    centred displacements and the group loss.
    """
    n = len(images)
    v = np.array(v, dtype=np.float64)
    m = np.array(m, dtype=np.float64)
    s = np.array(s, dtype=np.float64)
    if p.reinit_v:
        v[:] = 0.0
        m[:] = 0.0
        s[:] = 0.0
        step = 0
    inner = np.zeros((n, p.k2))
    for i in range(n):
        for k in range(p.k2):
            loss, g = subject_loss_grad(images[i], v[i], atlas, p)
            inner[i, k] = loss
            v[i], m[i], s[i] = adam_step(v[i], m[i], s[i], g, step + k + 1,
                                         p.lr, p.beta1, p.beta2, p.adam_eps)
            if p.smooth_sigma > 0.0:
                v[i] = gauss_smooth(v[i], p.smooth_sigma)
    step += p.k2
    if p.center_mode == "velocity":
        v, _ = center(v)
        u_hat = np.stack([exp_svf(v[i], p.n_sq)[0] for i in range(n)])
    else:
        u = np.stack([exp_svf(v[i], p.n_sq)[0] for i in range(n)])
        u_hat, _ = center(u)
    atlas = atlas_update(images, u_hat, atlas, p)
    F = group_loss(images, u_hat, atlas, p)
    return dict(v=v, m=m, s=s, step=step, atlas=atlas, u_hat=u_hat,
                inner_losses=inner, group_loss=F)


# ---------------------------------------------------------------------------
# diagnostics (Section 5, evaluation metrics)


def jacobian_det(u: np.ndarray) -> np.ndarray:
    """det(I + grad u) with central differences (one-sided at the edges)."""
    u = np.asarray(u, dtype=np.float64)
    J = np.empty((3, 3) + u.shape[1:])
    for c in range(3):
        grads = np.gradient(u[c])
        for d in range(3):
            J[c, d] = grads[d] + (1.0 if c == d else 0.0)
    return (J[0, 0] * (J[1, 1] * J[2, 2] - J[1, 2] * J[2, 1])
            - J[0, 1] * (J[1, 0] * J[2, 2] - J[1, 2] * J[2, 0])
            + J[0, 2] * (J[1, 0] * J[2, 1] - J[1, 1] * J[2, 0]))


def centrality_error(u: np.ndarray) -> float:
    """mean_x |(1/n) sum_i u_i(x)|_2 in voxels."""
    mean = np.asarray(u, dtype=np.float64).mean(axis=0)
    return float(np.sqrt((mean ** 2).sum(axis=0)).mean())


# ---------------------------------------------------------------------------
# one-shot segmentation (Section 4, Eq. (oneshot)) and its score


def warp_labels_nearest(labels: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Labels carried by a displacement: out(x) = L(round(x + u(x))), label 0
    outside the volume.  Nearest-neighbour keeps labels integral.  The
    position and its rounding, floor(p + 1/2), are taken in FP32 (the
    precision of the fields), so the same FP32 displacement gives the same
    labels on any IEEE FP32 machine."""
    labels = np.asarray(labels)
    u32 = np.asarray(u, dtype=np.float32)
    dims = labels.shape
    grid = np.meshgrid(*[np.arange(d, dtype=np.float32) for d in dims], indexing="ij")
    ks, inside = [], np.ones(dims, dtype=bool)
    for d in range(3):
        p = grid[d] + u32[d]                    # FP32 add
        k = np.floor(p + np.float32(0.5))       # FP32 add, then floor
        inside &= (k >= 0) & (k < dims[d])      # a NaN position is outside
        ks.append(k)
    idx = [np.where(inside, k, 0).astype(np.int64) for k in ks]
    return np.where(inside, labels[idx[0], idx[1], idx[2]], 0).astype(labels.dtype)


def segment_one_shot(atlas_labels: np.ndarray, v: np.ndarray, n_sq: int = 7) -> np.ndarray:
    """I_i^(S) = A^(S) o Exp(-v_i): the atlas labels carried to a subject by
    the inverse deformation, Exp(-v) (Section 4, Eq. (oneshot))."""
    u_inv, _ = exp_svf(-np.asarray(v, dtype=np.float64), n_sq)
    return warp_labels_nearest(atlas_labels, u_inv)


def dice_counts(a: np.ndarray, b: np.ndarray, num_labels: int) -> np.ndarray:
    """Per label l: (|a = l and b = l|, |a = l|, |b = l|) as int64 ``[L, 3]``.
    Dice_l = 2 c0 / (c1 + c2)."""
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    out = np.zeros((num_labels, 3), dtype=np.int64)
    for lab in range(num_labels):
        ia, ib = a == lab, b == lab
        out[lab] = (np.count_nonzero(ia & ib), np.count_nonzero(ia), np.count_nonzero(ib))
    return out


# ---------------------------------------------------------------------------
# factor-2 resampling between the levels of a coarse-to-fine schedule.  The
# paper runs one resolution; a pyramid is a reading for large cohorts.  Coarse
# voxel k averages fine voxels 2k and 2k+1 per axis, so its centre sits at fine
# coordinate 2k + 1/2 and fine voxel x sits at coarse coordinate (x - 1/2) / 2.


def down2(f: np.ndarray) -> np.ndarray:
    """Average of each 2x2x2 block over the last three axes (even sizes)."""
    f = np.asarray(f, dtype=np.float64)
    *lead, D0, D1, D2 = f.shape
    assert D0 % 2 == 0 and D1 % 2 == 0 and D2 % 2 == 0
    r = f.reshape(*lead, D0 // 2, 2, D1 // 2, 2, D2 // 2, 2)
    return r.mean(axis=(-5, -3, -1))


def up2(f: np.ndarray, scale: float = 1.0) -> np.ndarray:
    """Trilinear upsampling of a ``[C, d0, d1, d2]`` field to twice the size:
    out(x) = scale * S_B(f, (x - 1/2) / 2), border clamped.  ``scale = 2``
    turns a coarse displacement (coarse voxels) into fine voxels."""
    f = np.asarray(f, dtype=np.float64)
    dims = tuple(2 * d for d in f.shape[1:])
    pos = (identity_grid(dims) - 0.5) / 2.0
    vals, _ = sample_border(f, pos)
    return scale * vals


def level_start(images, v, p: SweepParams):
    """State at the start of a level: atlas from the centred Exp of the given
    velocities (v = 0 gives the mean of the subjects), Adam moments at zero."""
    n = len(images)
    if p.center_mode == "velocity":
        v, _ = center(v)
        u_hat = np.stack([exp_svf(v[i], p.n_sq)[0] for i in range(n)])
    else:
        u_hat, _ = center(np.stack([exp_svf(v[i], p.n_sq)[0] for i in range(n)]))
    atlas0 = np.asarray(images, dtype=np.float64).mean(axis=0)
    atlas = atlas_update(images, u_hat, atlas0, p)
    return np.array(v, dtype=np.float64), atlas


def pyramid(images, levels: int, sweeps, p: SweepParams):
    """Coarse-to-fine: the cohort at 1/2^(levels-1) ... 1 of its size (2x2x2
    averaging), ``sweeps[l]`` sweeps at level l (0 = coarsest); velocities are
    carried to the next level by ``up2(v, 2)``.  The coarsest level starts
    like a plain run (v = 0, A^0 the mean of the subjects); every finer level
    from ``level_start``.  Returns the finest state."""
    pyr = [np.asarray(images, dtype=np.float64)]
    for _ in range(levels - 1):
        pyr.append(down2(pyr[-1]))
    pyr = pyr[::-1]
    v = np.zeros((len(images), 3) + pyr[0].shape[1:])
    out = None
    for lev in range(levels):
        imgs = pyr[lev]
        if lev > 0:
            v = np.stack([up2(v[i], 2.0) for i in range(len(imgs))])
            v, atlas = level_start(imgs, v, p)
        else:
            atlas = initial_atlas(imgs)
        m = np.zeros_like(v)
        s = np.zeros_like(v)
        step = 0
        for _ in range(sweeps[lev]):
            out = sweep(imgs, v, m, s, step, atlas, p)
            v, m, s, step, atlas = out["v"], out["m"], out["s"], out["step"], out["atlas"]
    return out
