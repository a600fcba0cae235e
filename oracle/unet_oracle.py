"""FP64 CPU oracle of the learned warm start's network (test infrastructure
only: the test-suite, the smoke check and the benchmark's CPU leg may use
it; the product path never does).

The warm start maps an (atlas, subject) pair to an initial velocity field
for the subject's registration; DARC then starts from it instead of v = 0.
The network is a 3-D U-Net with 16/32/64/128 channels over four levels:

    e0 = act(conv(cat(A, I), 2 -> 16))            full resolution
    e1 = act(conv_s2(e0, 16 -> 32))               1/2
    e2 = act(conv_s2(e1, 32 -> 64))               1/4
    e3 = act(conv_s2(e2, 64 -> 128))              1/8
    d2 = act(conv(cat(up(e3), e2), 192 -> 64))    1/4
    d1 = act(conv(cat(up(d2), e1), 96 -> 32))     1/2
    d0 = act(conv(cat(up(d1), e0), 48 -> 16))     full
    v  = conv(d0, 16 -> 3)

conv: 3x3x3, zero padding 1, bias; conv_s2: the same with stride 2; up:
nearest-neighbour doubling; act: leaky ReLU with slope 0.2.

Precision points, as the MFMA kernels use them: every conv reads BF16
inputs and BF16 weights and accumulates exactly here (FP64; FP32 on the
GPU); every activation is stored as BF16 (round to nearest even); the final
velocity is FP32.  ``bf16`` below rounds an FP64/FP32 array to the BF16
grid and returns it as FP64.
"""

from __future__ import annotations

import numpy as np

SLOPE = 0.2
CHANNELS = (16, 32, 64, 128)


def bf16(x: np.ndarray) -> np.ndarray:
    """Round to the nearest BF16 value (ties to even), via FP32; NaN kept."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32)
    out = np.where(np.isnan(f), f, out)
    return out.astype(np.float64)


def conv3d(x: np.ndarray, w: np.ndarray, b: np.ndarray, stride: int = 1) -> np.ndarray:
    """3x3x3 convolution (cross-correlation, as in deep-learning frameworks),
    zero padding 1.  x [Cin, D0, D1, D2], w [Cout, Cin, 3, 3, 3], b [Cout];
    returns [Cout, D0', D1', D2'] with D' = (D - 1) // stride + 1."""
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    cin, D0, D1, D2 = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1)))
    O0, O1, O2 = (D0 - 1) // stride + 1, (D1 - 1) // stride + 1, (D2 - 1) // stride + 1
    out = np.zeros((w.shape[0], O0, O1, O2))
    for a in range(3):
        for bb in range(3):
            for c in range(3):
                patch = xp[:, a:a + stride * O0:stride, bb:bb + stride * O1:stride,
                           c:c + stride * O2:stride]
                out += np.tensordot(w[:, :, a, bb, c], patch, axes=([1], [0]))
    return out + np.asarray(b, dtype=np.float64)[:, None, None, None]


def leaky(x: np.ndarray) -> np.ndarray:
    return np.where(x > 0, x, SLOPE * x)


def up2_nearest(x: np.ndarray) -> np.ndarray:
    return x.repeat(2, axis=-3).repeat(2, axis=-2).repeat(2, axis=-1)


def layer_specs():
    """(name, cin, cout, stride, activation) of the eight convolutions."""
    c0, c1, c2, c3 = CHANNELS
    return [("e0", 2, c0, 1, True), ("e1", c0, c1, 2, True), ("e2", c1, c2, 2, True),
            ("e3", c2, c3, 2, True), ("d2", c3 + c2, c2, 1, True), ("d1", c2 + c1, c1, 1, True),
            ("d0", c1 + c0, c0, 1, True), ("out", c0, 3, 1, False)]


def forward(params: dict, atlas: np.ndarray, image: np.ndarray) -> np.ndarray:
    """v = UNet(A, I) for one subject; params[name] = (w, b) in FP64 holding
    BF16 weight values and FP32 biases."""
    act = lambda name, x, stride=1: bf16(leaky(conv3d(x, *params[name], stride)))
    x = bf16(np.stack([atlas, image]))
    e0 = act("e0", x)
    e1 = act("e1", e0, 2)
    e2 = act("e2", e1, 2)
    e3 = act("e3", e2, 2)
    d2 = act("d2", np.concatenate([up2_nearest(e3), e2]))
    d1 = act("d1", np.concatenate([up2_nearest(d2), e1]))
    d0 = act("d0", np.concatenate([up2_nearest(d1), e0]))
    return conv3d(d0, *params["out"])


def flops(dims) -> float:
    """Multiply-adds x 2 of one forward pass at volume dims."""
    total = 0.0
    V = float(np.prod(dims))
    for name, cin, cout, stride, _ in layer_specs():
        level = {"e0": 0, "e1": 1, "e2": 2, "e3": 3, "d2": 2, "d1": 1, "d0": 0, "out": 0}[name]
        total += 2.0 * 27 * cin * cout * V / 8 ** level
    return total
