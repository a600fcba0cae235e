"""Python binding of libdarc: torch tensors in, C ABI calls out.

torch supplies device memory and the current HIP stream; every step of the
DARC hot path runs in libdarc's HIP kernels.  Each function checks shapes,
dtypes and devices, passes raw pointers and sizes to the matching ``darc_*``
entry point on ``torch.cuda.current_stream()``, and raises
:class:`DarcError` on a non-zero status.  Nothing here computes.

Shapes: images ``[n, D0, D1, D2]`` FP32, fields ``[n, 3, D0, D1, D2]`` FP32
(component c displaces axis c, voxel units), all contiguous on one device.
"""

from __future__ import annotations

import ctypes
import dataclasses
from typing import Optional, Tuple

import torch

from . import _lib as L
from ._lib import DarcError  # noqa: F401

METRICS = {"mse": L.DARC_MSE, "lncc": L.DARC_LNCC, "l1": L.DARC_L1}
ATLAS_MODES = {"mean": L.DARC_ATLAS_MEAN, "median": L.DARC_ATLAS_MEDIAN, "sgd": L.DARC_ATLAS_SGD}
FUSED_MODES = {"auto": L.DARC_FUSED_AUTO, "off": L.DARC_FUSED_OFF, "on": L.DARC_FUSED_ON}
SGD_INITS = {"warm": L.DARC_SGD_INIT_WARM, "initial": L.DARC_SGD_INIT_INITIAL}
CENTER_MODES = {"displacement": L.DARC_CENTER_DISPLACEMENT, "velocity": L.DARC_CENTER_VELOCITY}


def lib() -> ctypes.CDLL:
    return L.load()


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _p(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev(name: str, t: torch.Tensor, dtype=torch.float32, ndim: Optional[int] = None) -> None:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must live in GPU memory (got device {t.device})")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype} (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if ndim is not None and t.dim() != ndim:
        raise ValueError(f"{name} must have {ndim} dims (got shape {tuple(t.shape)})")


def _field(name: str, t: torch.Tensor) -> Tuple[int, int, int, int]:
    _dev(name, t, ndim=5)
    if t.shape[1] != 3:
        raise ValueError(f"{name} must be [n, 3, D0, D1, D2] (got {tuple(t.shape)})")
    n, _, d0, d1, d2 = t.shape
    return n, d0, d1, d2


def _images(name: str, t: torch.Tensor) -> Tuple[int, int, int, int]:
    _dev(name, t, ndim=4)
    n, d0, d1, d2 = t.shape
    return n, d0, d1, d2


def _same(a_name, a, b_name, b):
    if tuple(a) != tuple(b):
        raise ValueError(f"{a_name} {tuple(a)} and {b_name} {tuple(b)} do not match")


def _call(fn: str, *args) -> None:
    lb = lib()
    L.check(lb, fn, getattr(lb, fn)(*args))


def _workspace(nbytes: int, device) -> Optional[torch.Tensor]:
    if nbytes == 0:
        return None
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


# --------------------------------------------------------------------- Exp(v)


def exp_svf(v: torch.Tensor, n_sq: int = 7, checkpoints: bool = True):
    """u = Exp(v) - id by scaling and squaring; returns ``(u, ckpt)``.

    ``ckpt`` is ``[n_sq-1, n, 3, D0, D1, D2]`` (u_1 .. u_{n_sq-1}) when
    ``checkpoints`` and ``n_sq >= 2``, else None.
    """
    n, d0, d1, d2 = _field("v", v)
    u = torch.empty_like(v)
    ckpt = None
    if checkpoints and n_sq >= 2:
        ckpt = torch.empty((n_sq - 1,) + tuple(v.shape), dtype=v.dtype, device=v.device)
    ws = _workspace(lib().darc_exp_svf_ws_bytes(n, d0, d1, d2, n_sq, int(ckpt is not None)),
                    v.device)
    _call("darc_exp_svf", _p(v), _p(u), _p(ckpt), n, d0, d1, d2, n_sq, _p(ws),
          0 if ws is None else ws.numel(), _stream())
    return u, ckpt


def exp_svf_bwd(v: torch.Tensor, ckpt: Optional[torch.Tensor], g_u: torch.Tensor,
                n_sq: int = 7) -> torch.Tensor:
    """dL/dv given dL/du, through the n_sq squaring steps (recomputed from v
    when ``ckpt`` is None)."""
    n, d0, d1, d2 = _field("v", v)
    _same("g_u", g_u.shape, "v", v.shape)
    _field("g_u", g_u)
    if ckpt is not None:
        _dev("ckpt", ckpt, ndim=6)
        _same("ckpt", ckpt.shape, "expected", (n_sq - 1,) + tuple(v.shape))
    g_v = torch.empty_like(v)
    ws = _workspace(lib().darc_exp_svf_bwd_ws_bytes(n, d0, d1, d2, n_sq, int(ckpt is not None)),
                    v.device)
    _call("darc_exp_svf_bwd", _p(v), _p(ckpt), _p(g_u), _p(g_v), n, d0, d1, d2, n_sq, _p(ws),
          0 if ws is None else ws.numel(), _stream())
    return g_v


# ----------------------------------------------------------------------- warp


def warp3d(img: torch.Tensor, u: torch.Tensor) -> torch.Tensor:
    """out_i(x) = I_i(x + u_i(x)), trilinear, zero padding."""
    n, d0, d1, d2 = _images("img", img)
    _same("u", u.shape, "expected", (n, 3, d0, d1, d2))
    _field("u", u)
    out = torch.empty_like(img)
    _call("darc_warp3d", _p(img), _p(u), _p(out), n, d0, d1, d2, _stream())
    return out


def warp3d_bwd(img: torch.Tensor, u: torch.Tensor, g_out: torch.Tensor,
               g_u: Optional[torch.Tensor] = None) -> torch.Tensor:
    """g_u += g_out * grad I(x + u); a zero g_u is created when None."""
    n, d0, d1, d2 = _images("img", img)
    _same("u", u.shape, "expected", (n, 3, d0, d1, d2))
    _field("u", u)
    _same("g_out", g_out.shape, "img", img.shape)
    _images("g_out", g_out)
    if g_u is None:
        g_u = torch.zeros_like(u)
    else:
        _same("g_u", g_u.shape, "u", u.shape)
        _field("g_u", g_u)
    _call("darc_warp3d_bwd", _p(img), _p(u), _p(g_out), _p(g_u), n, d0, d1, d2, _stream())
    return g_u


# ------------------------------------------------------------ dissimilarity


def sim_grad(warped: torch.Tensor, atlas: torch.Tensor, metric: str = "mse", win: int = 9,
             eps: float = 1e-5, grad: bool = True):
    """Per-subject dissimilarity (FP64 ``[n]``) and, if ``grad``, dD/dwarped."""
    n, d0, d1, d2 = _images("warped", warped)
    _dev("atlas", atlas, ndim=3)
    _same("atlas", atlas.shape, "volume", (d0, d1, d2))
    m = METRICS[metric]
    loss = torch.zeros(n, dtype=torch.float64, device=warped.device)
    g = torch.empty_like(warped) if grad else None
    ws = _workspace(lib().darc_sim_grad_ws_bytes(m, n, d0, d1, d2) if grad else 0, warped.device)
    _call("darc_sim_grad", _p(warped), _p(atlas), m, win, eps, _p(loss), _p(g), n, d0, d1, d2,
          _p(ws), 0 if ws is None else ws.numel(), _stream())
    return loss, g


def sim_grad_noalloc(warped: torch.Tensor, atlas: torch.Tensor, loss: torch.Tensor,
                     g: Optional[torch.Tensor], metric: str = "lncc", win: int = 9,
                     eps: float = 1e-5) -> None:
    """``sim_grad`` into caller-provided outputs through the entry point that
    allocates nothing (its scratch is the library's per-GPU array):
    ``loss[i] += D_i`` (FP64 ``[n]``) and, if ``g`` is given, g = dD/dwarped."""
    n, d0, d1, d2 = _images("warped", warped)
    _dev("atlas", atlas, ndim=3)
    _same("atlas", atlas.shape, "volume", (d0, d1, d2))
    _dev("loss", loss, dtype=torch.float64, ndim=1)
    _same("loss", loss.shape, "expected", (n,))
    if g is not None:
        _images("g", g)
        _same("g", g.shape, "warped", warped.shape)
    _call("darc_sim_grad_noalloc", _p(warped), _p(atlas), METRICS[metric], win, eps, _p(loss),
          _p(g), n, d0, d1, d2, _stream())


# ----------------------------------------------------------------- smoothing


def gauss_smooth(x: torch.Tensor, sigma: float) -> torch.Tensor:
    """Separable Gaussian of every component of ``[n, ncomp, D0, D1, D2]``."""
    _dev("x", x, ndim=5)
    n, nc, d0, d1, d2 = x.shape
    out = torch.empty_like(x)
    _call("darc_smooth3d", _p(x), _p(out), n, nc, d0, d1, d2, L.DARC_GAUSS, sigma, None, None, 0,
          _stream())
    return out


def diffusion(u: torch.Tensor, lam: float, out: Optional[torch.Tensor] = None,
              with_loss: bool = True):
    """(out += lam dR/du, lam R(u_i) per subject as FP64 ``[n]``)."""
    _dev("u", u, ndim=5)
    n, nc, d0, d1, d2 = u.shape
    if out is None:
        out = torch.zeros_like(u)
    else:
        _same("out", out.shape, "u", u.shape)
        _dev("out", out, ndim=5)
    loss = torch.zeros(n, dtype=torch.float64, device=u.device) if with_loss else None
    _call("darc_smooth3d", _p(u), _p(out), n, nc, d0, d1, d2, L.DARC_DIFFUSION, lam, _p(loss),
          None, 0, _stream())
    return out, loss


# ------------------------------------------------- optimiser, centring, atlas


def adam_step(v, m, s, g, t: int, lr=1e-2, beta1=0.9, beta2=0.999, eps=1e-8) -> None:
    """One in-place Adam step on v (m, s updated); t is the new step count."""
    for name, x in (("v", v), ("m", m), ("s", s), ("g", g)):
        _dev(name, x)
        _same(name, x.shape, "v", v.shape)
    _call("darc_adam_step", _p(v), _p(m), _p(s), _p(g), v.numel(), t, lr, beta1, beta2, eps,
          _stream())


def center(u: torch.Tensor) -> torch.Tensor:
    """In place u_i <- u_i - mean_j u_j; returns the mean ``[3, D0, D1, D2]``."""
    n, d0, d1, d2 = _field("u", u)
    mean = torch.empty((3, d0, d1, d2), dtype=u.dtype, device=u.device)
    _call("darc_center", _p(u), _p(mean), n, d0, d1, d2, _stream())
    return mean


def atlas_update(images: torch.Tensor, u: Optional[torch.Tensor],
                 mean: Optional[torch.Tensor] = None) -> torch.Tensor:
    """A(x) = (1/n) sum_i I_i(x + u_i(x) - mean(x)); ``u = None`` gives the
    mean of the unwarped images (A^0)."""
    n, d0, d1, d2 = _images("images", images)
    if u is not None:
        _same("u", u.shape, "expected", (n, 3, d0, d1, d2))
        _field("u", u)
    if mean is not None:
        _dev("mean", mean, ndim=4)
        _same("mean", mean.shape, "expected", (3, d0, d1, d2))
    atlas = torch.empty((d0, d1, d2), dtype=images.dtype, device=images.device)
    _call("darc_atlas_update", _p(images), _p(u), _p(mean), _p(atlas), n, d0, d1, d2, _stream())
    return atlas


def atlas_median(images: torch.Tensor, u: torch.Tensor,
                 mean: Optional[torch.Tensor] = None) -> torch.Tensor:
    """A(x) = median_i I_i(x + u_i(x) - mean(x)) (the L1 atlas; even n
    averages the two middle samples)."""
    n, d0, d1, d2 = _images("images", images)
    _same("u", u.shape, "expected", (n, 3, d0, d1, d2))
    _field("u", u)
    if mean is not None:
        _dev("mean", mean, ndim=4)
        _same("mean", mean.shape, "expected", (3, d0, d1, d2))
    atlas = torch.empty((d0, d1, d2), dtype=images.dtype, device=images.device)
    _call("darc_atlas_median", _p(images), _p(u), _p(mean), _p(atlas), n, d0, d1, d2, _stream())
    return atlas


def atlas_sgd(warped: torch.Tensor, atlas: torch.Tensor, epochs: int = 20, batch: int = 4,
              win: int = 9, eps: float = 1e-5, lr: float = 1e-2, beta1: float = 0.9,
              beta2: float = 0.999, adam_eps: float = 1e-8) -> torch.Tensor:
    """In-place minibatch Adam on the atlas against the LNCC of the warped
    subjects; returns the per-minibatch losses (FP64)."""
    n, d0, d1, d2 = _images("warped", warped)
    _dev("atlas", atlas, ndim=3)
    _same("atlas", atlas.shape, "volume", (d0, d1, d2))
    b = min(batch, n)
    nbatch = (n + b - 1) // b
    losses = torch.zeros(epochs * nbatch, dtype=torch.float64, device=warped.device)
    ws = _workspace(lib().darc_atlas_sgd_ws_bytes(n, d0, d1, d2, b), warped.device)
    _call("darc_atlas_sgd", _p(warped), _p(atlas), n, d0, d1, d2, b, epochs, win, eps, lr, beta1,
          beta2, adam_eps, _p(losses), _p(ws), 0 if ws is None else ws.numel(), _stream())
    return losses


# ---------------------------------------------------- one-shot segmentation


def _labels(name: str, t: torch.Tensor, ndim: int) -> None:
    _dev(name, t, dtype=torch.uint8, ndim=ndim)


def warp_labels(labels: torch.Tensor, u: torch.Tensor) -> torch.Tensor:
    """out_i(x) = labels(round(x + u_i(x))), 0 outside; labels ``[D0, D1, D2]``
    uint8, u ``[n, 3, D0, D1, D2]``."""
    _labels("labels", labels, 3)
    n, d0, d1, d2 = _field("u", u)
    _same("labels", labels.shape, "volume", (d0, d1, d2))
    out = torch.empty((n, d0, d1, d2), dtype=torch.uint8, device=u.device)
    _call("darc_warp_labels", _p(labels), _p(u), _p(out), n, d0, d1, d2, _stream())
    return out


def segment(labels: torch.Tensor, v: torch.Tensor, n_sq: int = 7) -> torch.Tensor:
    """One-shot segmentation: the atlas labels carried to each subject by
    Exp(-v_i)."""
    _labels("labels", labels, 3)
    n, d0, d1, d2 = _field("v", v)
    _same("labels", labels.shape, "volume", (d0, d1, d2))
    out = torch.empty((n, d0, d1, d2), dtype=torch.uint8, device=v.device)
    ws = _workspace(lib().darc_segment_ws_bytes(n, d0, d1, d2, n_sq), v.device)
    _call("darc_segment", _p(labels), _p(v), _p(out), n, d0, d1, d2, n_sq, _p(ws),
          0 if ws is None else ws.numel(), _stream())
    return out


def dice_counts(a: torch.Tensor, b: torch.Tensor, num_labels: int) -> torch.Tensor:
    """Per subject and label: (|a = l and b = l|, |a = l|, |b = l|) as int64
    ``[n, num_labels, 3]``; a and b are ``[n, ...]`` uint8."""
    _dev("a", a, dtype=torch.uint8)
    _dev("b", b, dtype=torch.uint8)
    _same("a", a.shape, "b", b.shape)
    n = a.shape[0]
    V = a[0].numel() if n else 0
    counts = torch.zeros((n, num_labels, 3), dtype=torch.int64, device=a.device)
    _call("darc_dice_counts", _p(a), _p(b), n, V, num_labels, _p(counts), _stream())
    return counts


# ---------------------------------------------------------------- resampling


def down2(x: torch.Tensor) -> torch.Tensor:
    """2x2x2 block means over the last three (even) axes of a contiguous
    FP32 tensor ``[..., D0, D1, D2]``."""
    _dev("x", x)
    *lead, d0, d1, d2 = x.shape
    nchan = x[..., 0, 0, 0].numel()
    out = torch.empty(tuple(lead) + (d0 // 2, d1 // 2, d2 // 2), dtype=x.dtype, device=x.device)
    _call("darc_down2", _p(x), _p(out), nchan, d0, d1, d2, _stream())
    return out


def up2(x: torch.Tensor, scale: float = 1.0) -> torch.Tensor:
    """Trilinear (border) upsampling of ``[..., d0, d1, d2]`` to twice the
    size, out(x) = scale * x_coarse((x - 1/2) / 2)."""
    _dev("x", x)
    *lead, d0, d1, d2 = x.shape
    nchan = x[..., 0, 0, 0].numel()
    out = torch.empty(tuple(lead) + (2 * d0, 2 * d1, 2 * d2), dtype=x.dtype, device=x.device)
    _call("darc_up2", _p(x), _p(out), nchan, 2 * d0, 2 * d1, 2 * d2, scale, _stream())
    return out


# ---------------------------------------------------------------------- sweep


@dataclasses.dataclass
class SweepParams:
    """Settings of one coordinate-descent sweep (mirrors ``darc_params``)."""

    metric: str = "mse"
    win: int = 9
    ncc_eps: float = 1e-5
    lam: float = 0.01
    smooth_sigma: float = 0.0
    n_sq: int = 7
    k2: int = 5
    lr: float = 1e-2
    beta1: float = 0.9
    beta2: float = 0.999
    adam_eps: float = 1e-8
    center_mode: str = "displacement"
    reinit_v: bool = False
    batch: int = 0  # subjects per launch; 0 = all
    atlas_mode: str = "auto"  # mean | median | sgd; auto: median for L1, else mean
    k3: int = 20  # stochastic atlas: epochs
    atlas_batch: int = 4  # stochastic atlas: subjects per minibatch
    atlas_lr: float = 1e-2  # stochastic atlas: Adam learning rate
    sgd_init: str = "warm"  # stochastic atlas start: warm (A^k) | initial (A^0, Alg. 1 literal)
    fused: str = "auto"  # one launch per inner iteration: auto | off | on (MSE/L1, no smoothing)

    def resolved_atlas_mode(self) -> str:
        if self.atlas_mode != "auto":
            return self.atlas_mode
        return "median" if self.metric == "l1" else "mean"

    def to_c(self, k2: Optional[int] = None) -> L.DarcParams:
        return L.DarcParams(METRICS[self.metric], self.win, self.ncc_eps, self.lam,
                            self.smooth_sigma, self.n_sq, self.k2 if k2 is None else k2, self.lr,
                            self.beta1, self.beta2, self.adam_eps,
                            CENTER_MODES[self.center_mode], int(self.reinit_v), self.batch,
                            ATLAS_MODES[self.resolved_atlas_mode()], self.k3, self.atlas_batch,
                            self.atlas_lr, SGD_INITS[self.sgd_init], FUSED_MODES[self.fused])


class Cohort:
    """Device state of one DARC run: images, velocities, Adam moments, atlas.

    ``images`` is ``[n, D0, D1, D2]`` FP32 on the GPU.  Velocities and moments
    start at zero and the atlas at the mean of the unwarped subjects
    (computed by ``darc_atlas_update`` with zero displacements).

    With ``device_step=True`` the Adam step counter lives in device memory and
    the sweep reads and advances it there, so one captured sweep
    (:meth:`capture`) can be replayed any number of times.
    """

    def __init__(self, images: torch.Tensor, params: SweepParams, keep_u_hat: bool = True,
                 device_step: bool = False, v0: Optional[torch.Tensor] = None):
        n, d0, d1, d2 = _images("images", images)
        self.images = images
        self.params = params
        dev = images.device
        shape = (n, 3, d0, d1, d2)
        self.m = torch.zeros(shape, dtype=torch.float32, device=dev)
        self.s = torch.zeros_like(self.m)
        if v0 is None:
            self.v = torch.zeros_like(self.m)
        else:
            _field("v0", v0)
            _same("v0", v0.shape, "expected", shape)
            self.v = v0  # adopted, not copied
        self.u_hat = torch.zeros_like(self.m) if keep_u_hat else None
        # A^0: the mean of the unwarped subjects
        self.atlas = atlas_update(images, None)
        self.step = 0
        self.sweeps = 0
        self.step_dev = torch.zeros(1, dtype=torch.int64, device=dev) if device_step else None
        self._state = L.DarcState()
        self._cparams = params.to_c()
        self._cparams_start = params.to_c(k2=0)
        self._refresh_state()
        nbytes = lib().darc_sweep_ws_bytes(ctypes.byref(self._state), ctypes.byref(self._cparams))
        if nbytes == 0:
            raise DarcError("darc_sweep_ws_bytes", L.DARC_EINVAL,
                            lib().darc_last_error().decode(errors="replace"))
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.losses = torch.zeros(n * params.k2 + 1, dtype=torch.float64, device=dev)

    def _refresh_state(self) -> None:
        n, d0, d1, d2 = self.images.shape
        st = self._state
        st.images = self.images.data_ptr()
        st.v = self.v.data_ptr()
        st.m = self.m.data_ptr()
        st.s = self.s.data_ptr()
        st.atlas = self.atlas.data_ptr()
        st.u_hat = None if self.u_hat is None else self.u_hat.data_ptr()
        st.step = self.step
        st.step_dev = None if self.step_dev is None else self.step_dev.data_ptr()
        st.n, st.d0, st.d1, st.d2 = n, d0, d1, d2

    def sweep(self) -> torch.Tensor:
        """Enqueue one sweep; returns the device losses ``[n*k2 + 1]`` (FP64):
        per-subject inner losses, then the group loss."""
        self._refresh_state()
        _call("darc_sweep", ctypes.byref(self._state), ctypes.byref(self._cparams),
              _p(self.losses), _p(self.ws), self.ws.numel(), _stream())
        self.step = int(self._state.step)
        self.sweeps += 1
        return self.losses

    def group_loss(self) -> float:
        return float(self.losses[-1].item())

    def level_start(self) -> torch.Tensor:
        """Steps 2 and 3 of a sweep without step 1 (k2 = 0): centred Exp of
        the current velocities, the atlas update from the current atlas, and
        the group loss (written to ``losses[0]``).  The start of a level of a
        coarse-to-fine schedule."""
        self._refresh_state()
        _call("darc_sweep", ctypes.byref(self._state), ctypes.byref(self._cparams_start),
              _p(self.losses), _p(self.ws), self.ws.numel(), _stream())
        return self.losses[:1]

    def autotune(self) -> tuple:
        """Time the candidate launch shapes on this cohort's shapes -- the
        squaring steps' marching depth (8 to 64 planes) or plane-parallel
        shape, the window kernels' chunk length and (MSE / L1 without
        smoothing) one fused inner iteration against separate launches --
        and keep the fastest for later launches; returns (squaring shape:
        planes per chunk or -1 for plane-parallel, window-kernel chunk,
        fused choice: 1 fused, 2 separate, 0 not tuned).  Only workspace
        memory is written; the cohort state is left as it is."""
        self._refresh_state()
        chosen = (ctypes.c_int * 3)()
        _call("darc_autotune", ctypes.byref(self._state), ctypes.byref(self._cparams),
              _p(self.ws), self.ws.numel(), _stream(), chosen)
        return int(chosen[0]), int(chosen[1]), int(chosen[2])

    def capture(self) -> "SweepGraph":
        """Capture one sweep into a HIP graph (needs ``device_step=True``).
        Capturing runs nothing; every replay performs one sweep."""
        if self.step_dev is None:
            raise ValueError("capture() needs a cohort built with device_step=True")
        if self.params.reinit_v:
            raise ValueError("a captured sweep with reinit_v would reset on every replay")
        self._refresh_state()
        graph = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream(device=self.images.device)
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            graph.capture_begin()
            try:
                _call("darc_sweep", ctypes.byref(self._state), ctypes.byref(self._cparams),
                      _p(self.losses), _p(self.ws), self.ws.numel(), _stream())
            finally:
                graph.capture_end()
        torch.cuda.current_stream().wait_stream(side)
        return SweepGraph(self, graph)


class Pyramid:
    """Coarse-to-fine DARC: the cohort at 1/2^(levels-1), ..., 1/2, 1 of its
    size (2x2x2 block means of the images).  Each level starts from the
    velocities of the coarser one carried up by ``up2(v, 2)`` (fresh Adam
    moments and step count, the atlas re-derived by :meth:`Cohort.level_start`)
    and runs :meth:`sweep` as often as the caller wants before
    :meth:`next_level`."""

    def __init__(self, images: torch.Tensor, params: SweepParams, levels: int,
                 keep_u_hat: bool = True):
        if levels < 1:
            raise ValueError("levels must be >= 1")
        pyr = [images]
        for _ in range(levels - 1):
            pyr.append(down2(pyr[-1]))
        self.images = pyr[::-1]
        self.params = params
        self.keep_u_hat = keep_u_hat
        self.level = 0
        self.cohort = Cohort(self.images[0], params, keep_u_hat)

    @property
    def levels(self) -> int:
        return len(self.images)

    def sweep(self) -> torch.Tensor:
        return self.cohort.sweep()

    def next_level(self) -> Cohort:
        if self.level + 1 >= self.levels:
            raise ValueError("already at the finest level")
        v = up2(self.cohort.v, 2.0)
        self.level += 1
        self.cohort = Cohort(self.images[self.level], self.params, self.keep_u_hat, v0=v)
        self.cohort.level_start()
        return self.cohort


class SweepGraph:
    """A captured sweep of a :class:`Cohort`; :meth:`replay` runs one sweep."""

    def __init__(self, cohort: Cohort, graph):
        self.cohort = cohort
        self.graph = graph

    def replay(self) -> torch.Tensor:
        self.graph.replay()
        c = self.cohort
        c.step += c.params.k2
        c.sweeps += 1
        return c.losses


SHAPE_KINDS = {"squaring": L.DARC_SHAPE_SQUARING, "window": L.DARC_SHAPE_WINDOW,
               "fused": L.DARC_SHAPE_FUSED}


def set_launch_shape(kind: str, dims, n: int, value: int) -> None:
    """Set one entry of the autotuner's table for volumes ``dims`` and ``n``
    subjects per launch, or for every shape without an entry of its own
    (``dims=None``): kind "squaring": tile depth, 1 marching at the built-in
    depth, -1 one plane per block; "window": tile depth; "fused": 1 fused, 2
    separate; 0 resets."""
    d0, d1, d2 = dims if dims is not None else (0, 0, 0)
    n = n if dims is not None else 0
    _call("darc_set_launch_shape", SHAPE_KINDS[kind], d0, d1, d2, n, value)


def fused_barrier_ticks(ticks: int) -> None:
    """Bound of one grid-barrier wait of the fused iteration (ticks of the
    100 MHz counter; negative restores the one-second default)."""
    _call("darc_fused_barrier_ticks", int(ticks))


def autotune_clear() -> None:
    """Forget every tuned launch shape (the built-in heuristic applies again)."""
    _call("darc_autotune_clear")


# -------------------------------------------------------------- kernel timing


def profile_enable(on: bool = True) -> None:
    _call("darc_profile_enable", int(on))


def profile_reset() -> None:
    _call("darc_profile_reset")


def profile_collect() -> dict:
    """{kernel class: (launches, total ms)} since the last reset."""
    lb = lib()
    k = lb.darc_profile_num_classes()
    counts = (ctypes.c_longlong * k)()
    ms = (ctypes.c_double * k)()
    L.check(lb, "darc_profile_collect", lb.darc_profile_collect(counts, ms, k))
    return {lb.darc_profile_name(i).decode(): (int(counts[i]), float(ms[i])) for i in range(k)}
