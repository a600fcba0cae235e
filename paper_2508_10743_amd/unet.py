"""The learned warm start: a 3-D U-Net from an (atlas, subject) pair to an
initial velocity field, run by libdarc's BF16 matrix-core convolutions.

DARC registers every subject from v = 0; a network trained on earlier DARC
results can propose v_i directly, and the coordinate descent then starts from
that proposal (``Cohort(images, params, v0=UNet(...)(atlas, images))``).
Plain DARC from v = 0 stays the fallback.  This module holds the parameters
(seeded initialisation, packing into the kernels' layout on the host) and the
ctypes calls; every convolution runs in ``darc_conv3d`` /
``darc_unet_forward``.
"""

from __future__ import annotations

import ctypes
from typing import List, Optional, Tuple

import numpy as np
import torch

from . import _lib as L
from .darc import _call, _dev, _field, _images, _p, _stream, _workspace, lib

# (cin, cout, stride, activation) of e0 e1 e2 e3 d2 d1 d0 out
LAYERS: List[Tuple[int, int, int, bool]] = [
    (2, 16, 1, True), (16, 32, 2, True), (32, 64, 2, True), (64, 128, 2, True),
    (192, 64, 1, True), (96, 32, 1, True), (48, 16, 1, True), (16, 3, 1, False)]
SLOPE = 0.2


def bf16_round(x: np.ndarray) -> np.ndarray:
    """FP32 values rounded to BF16 (nearest even), returned as FP32."""
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(
        torch.bfloat16).to(torch.float32).numpy()


def pack_weights(w: np.ndarray, ksize: int = 3) -> np.ndarray:
    """[cout][cin][k][k][k] -> the kernels' [cout][kpad] layout (FP32 values;
    channels padded to a multiple of 8, K to darc_conv3d_kpad)."""
    cout, cin = w.shape[:2]
    cin_p = (cin + 7) // 8 * 8
    taps = ksize ** 3
    kpad = lib().darc_conv3d_kpad(cin_p, ksize)
    t = np.zeros((cout, taps, cin_p), np.float32)
    t[:, :, :cin] = np.moveaxis(w.reshape(cout, cin, taps), 1, 2)
    out = np.zeros((cout, kpad), np.float32)
    out[:, :taps * cin_p] = t.reshape(cout, -1)
    return out


def to_bf16_device(x: np.ndarray, device) -> torch.Tensor:
    """Upload FP32 values as BF16 (rounded to nearest even)."""
    return torch.from_numpy(np.ascontiguousarray(x, np.float32)).to(torch.bfloat16).to(device)


class UNet:
    """Parameters of the warm-start network.  ``weights[l]`` is
    ``[cout][cin][3][3][3]`` FP32 holding BF16-representable values,
    ``biases[l]`` ``[cout]`` FP32 (He-normal initialisation from ``seed``)."""

    def __init__(self, seed: int = 0, device=None):
        rng = np.random.default_rng(seed)
        self.weights, self.biases = [], []
        for cin, cout, _, _ in LAYERS:
            std = np.sqrt(2.0 / (27 * cin)) * (0.1 if cout == 3 else 1.0)
            self.weights.append(bf16_round(rng.normal(0.0, std, (cout, cin, 3, 3, 3))))
            self.biases.append(rng.normal(0.0, 0.01, cout).astype(np.float32))
        self.device = device or torch.device("cuda", 0)
        self._packed: Optional[Tuple[torch.Tensor, torch.Tensor]] = None

    def packed(self) -> Tuple[torch.Tensor, torch.Tensor]:
        """(weights BF16, biases FP32) on the device in darc_unet_layout order."""
        if self._packed is None:
            lb = lib()
            ws, bs = [], []
            for l, (w, b) in enumerate(zip(self.weights, self.biases)):
                cin, cout, kpad = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
                wo, bo = ctypes.c_size_t(), ctypes.c_size_t()
                L.check(lb, "darc_unet_layout", lb.darc_unet_layout(
                    l, ctypes.byref(cin), ctypes.byref(cout), ctypes.byref(kpad),
                    ctypes.byref(wo), ctypes.byref(bo)))
                pw = pack_weights(w)
                assert pw.shape == (cout.value, kpad.value) and wo.value == sum(x.size for x in ws)
                ws.append(pw)
                bs.append(b)
            self._packed = (to_bf16_device(np.concatenate([x.ravel() for x in ws]), self.device),
                            torch.from_numpy(np.concatenate(bs)).to(self.device))
        return self._packed

    def __call__(self, atlas: torch.Tensor, images: torch.Tensor) -> torch.Tensor:
        """v = UNet(A, I_i) for every subject: FP32 ``[n, 3, D0, D1, D2]``."""
        n, d0, d1, d2 = _images("images", images)
        _dev("atlas", atlas, ndim=3)
        w, b = self.packed()
        v = torch.empty((n, 3, d0, d1, d2), dtype=torch.float32, device=images.device)
        ws = _workspace(lib().darc_unet_ws_bytes(n, d0, d1, d2), images.device)
        _call("darc_unet_forward", _p(w), _p(b), _p(atlas), _p(images), _p(v), n, d0, d1, d2,
              _p(ws), 0 if ws is None else ws.numel(), _stream())
        return v


def conv3d(x0: torch.Tensor, w: torch.Tensor, bias: Optional[torch.Tensor], cout: int,
           stride: int = 1, ksize: int = 3, act: bool = False, slope: float = SLOPE,
           x1: Optional[torch.Tensor] = None, up0: bool = False, out_planar: bool = False):
    """One convolution through ``darc_conv3d``.  x0/x1 channels-last BF16
    ``[n, D0, D1, D2, C]`` (x0 at half the dims when ``up0``); ``w`` packed
    BF16 ``[cout, kpad]``.  Returns BF16 channels-last, or FP32 planar
    ``[n, cout, D0', D1', D2']`` when ``out_planar``."""
    _dev("x0", x0, dtype=torch.bfloat16, ndim=5)
    n, h0, h1, h2, c0 = x0.shape
    d0, d1, d2 = (2 * h0, 2 * h1, 2 * h2) if up0 else (h0, h1, h2)
    c1 = 0
    if x1 is not None:
        _dev("x1", x1, dtype=torch.bfloat16, ndim=5)
        c1 = x1.shape[4]
    _dev("w", w, dtype=torch.bfloat16, ndim=2)
    o = tuple((d - 1) // stride + 1 for d in (d0, d1, d2))
    y16 = y32 = None
    if out_planar:
        y32 = torch.empty((n, cout) + o, dtype=torch.float32, device=x0.device)
    else:
        y16 = torch.empty((n,) + o + (cout,), dtype=torch.bfloat16, device=x0.device)
    _call("darc_conv3d", _p(x0), c0, int(up0), _p(x1), c1, n, d0, d1, d2, ksize, stride, _p(w),
          _p(bias), cout, int(act), slope, _p(y16), _p(y32), _stream())
    return y32 if out_planar else y16


def conv3d_grad(dz: torch.Tensor, x0: torch.Tensor, w32: torch.Tensor, cout: int,
                stride: int = 1, x1: Optional[torch.Tensor] = None, up0: bool = False,
                input_grad: bool = True):
    """Adjoint of :func:`conv3d` (ksize 3) through ``darc_conv3d_grad``: dz
    channels-last BF16 ``[n, O0, O1, O2, cz]``; w32 packed FP32 ``[cout, kpad]``.
    Returns (dw FP32 ``[cout, kpad]``, db ``[cout]``, dx FP32 channels-last
    ``[n, D0, D1, D2, c0 + c1]`` or None)."""
    _dev("dz", dz, dtype=torch.bfloat16, ndim=5)
    _dev("x0", x0, dtype=torch.bfloat16, ndim=5)
    n, h0, h1, h2, c0 = x0.shape
    d0, d1, d2 = (2 * h0, 2 * h1, 2 * h2) if up0 else (h0, h1, h2)
    c1 = 0 if x1 is None else x1.shape[4]
    cz = dz.shape[4]
    dw = torch.zeros_like(w32)
    db = torch.zeros(cout, dtype=torch.float32, device=dz.device)
    dx = wt = None
    if input_grad:
        dx = torch.empty((n, d0, d1, d2, c0 + c1), dtype=torch.float32, device=dz.device)
        wt = torch.empty((c0 + c1, lib().darc_conv3d_kpad(cz, 3)), dtype=torch.bfloat16,
                         device=dz.device)
    _call("darc_conv3d_grad", _p(dz), cz, _p(x0), c0, int(up0), _p(x1), c1, n, d0, d1, d2,
          stride, _p(w32), cout, _p(dw), _p(db), _p(dx), _p(wt), _stream())
    return dw, db, dx


def unpack_weights(packed: np.ndarray, cin: int, ksize: int = 3) -> np.ndarray:
    """Inverse of :func:`pack_weights`: [cout][kpad] -> [cout][cin][k][k][k]."""
    cout = packed.shape[0]
    cin_p = (cin + 7) // 8 * 8
    taps = ksize ** 3
    t = packed[:, :taps * cin_p].reshape(cout, taps, cin_p)[:, :, :cin]
    return np.moveaxis(t, 2, 1).reshape(cout, cin, ksize, ksize, ksize)


class Trainer:
    """Adam training of a :class:`UNet` on (atlas, subject, target velocity)
    triples through ``darc_unet_train_step``: FP32 master weights and moments
    on the device, the BF16 copy refreshed after every step (and used by the
    network's forward pass from then on)."""

    def __init__(self, net: UNet, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
                 eps: float = 1e-8):
        self.net, self.lr, self.beta1, self.beta2, self.eps = net, lr, beta1, beta2, eps
        dev = net.device
        w = np.concatenate([pack_weights(w).ravel() for w in net.weights])
        b = np.concatenate(net.biases)
        self.w = torch.from_numpy(w).to(dev)
        self.b = torch.from_numpy(b).to(dev)
        self.mw, self.sw = torch.zeros_like(self.w), torch.zeros_like(self.w)
        self.mb, self.sb = torch.zeros_like(self.b), torch.zeros_like(self.b)
        self.dw, self.db = torch.zeros_like(self.w), torch.zeros_like(self.b)
        self.wq = to_bf16_device(w, dev)
        assert self.w.numel() == lib().darc_unet_num_weights()
        assert self.b.numel() == lib().darc_unet_num_biases()
        self.state = L.DarcUnetTrain(*[t.data_ptr() for t in (self.w, self.b, self.mw, self.sw,
                                                             self.mb, self.sb, self.wq, self.dw,
                                                             self.db)], 0)
        net._packed = (self.wq, self.b)

    def _ws(self, images):
        n, d0, d1, d2 = _images("images", images)
        return _workspace(lib().darc_unet_train_ws_bytes(n, d0, d1, d2), images.device)

    def step(self, atlas: torch.Tensor, images: torch.Tensor, targets: torch.Tensor) -> torch.Tensor:
        """One Adam step; returns the loss before it (FP64 device scalar)."""
        n, d0, d1, d2 = _images("images", images)
        _field("targets", targets)
        loss = torch.zeros(1, dtype=torch.float64, device=images.device)
        ws = self._ws(images)
        _call("darc_unet_train_step", ctypes.byref(self.state), _p(atlas), _p(images),
              _p(targets), self.lr, self.beta1, self.beta2, self.eps, _p(loss), n, d0, d1, d2,
              _p(ws), ws.numel(), _stream())
        return loss

    def gradients(self, atlas: torch.Tensor, images: torch.Tensor, targets: torch.Tensor):
        """(loss, [(dw [cout][cin][3][3][3], db [cout]) per layer]) at the current
        weights, on the host."""
        n, d0, d1, d2 = _images("images", images)
        loss = torch.zeros(1, dtype=torch.float64, device=images.device)
        ws = self._ws(images)
        _call("darc_unet_backward", _p(self.wq), _p(self.w), _p(self.b), _p(atlas), _p(images),
              _p(targets), _p(self.dw), _p(self.db), _p(loss), None, n, d0, d1, d2, _p(ws),
              ws.numel(), _stream())
        dw, db = self.dw.cpu().numpy(), self.db.cpu().numpy()
        out, wo, bo = [], 0, 0
        for cin, cout, _, _ in LAYERS:
            kpad = lib().darc_conv3d_kpad((cin + 7) // 8 * 8, 3)
            out.append((unpack_weights(dw[wo:wo + cout * kpad].reshape(cout, kpad), cin),
                        db[bo:bo + cout]))
            wo += cout * kpad
            bo += cout
        return float(loss.item()), out
