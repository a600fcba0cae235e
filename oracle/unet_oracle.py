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


# ---------------------------------------------------------------------------
# training: gradient of the mean squared velocity error
#
# The backward pass mirrors the kernels' precision points: each layer's
# output gradient dz = dy * act'(y) is rounded to BF16 (act'(y) = 1 where the
# stored output y > 0, else the slope), weights are the BF16 values, and
# everything else is exact here (FP32 accumulation on the GPU).  With
# ``rounded=False`` no rounding is applied anywhere, which is what the pins
# compare with automatic differentiation.


def conv3d_input_grad(dz: np.ndarray, w: np.ndarray, in_dims, stride: int = 1) -> np.ndarray:
    """Adjoint of ``conv3d`` with respect to its input: the stride-1
    convolution, zero padding 1, of dz (spread onto the zero-dilated input
    grid for stride 2) with the taps flipped and the channel axes exchanged."""
    dz = np.asarray(dz, dtype=np.float64)
    if stride == 2:
        dil = np.zeros((dz.shape[0],) + tuple(in_dims))
        dil[:, ::2, ::2, ::2] = dz
        dz = dil
    wt = np.transpose(np.asarray(w, dtype=np.float64)[:, :, ::-1, ::-1, ::-1], (1, 0, 2, 3, 4))
    return conv3d(dz, wt, np.zeros(wt.shape[0]))


def conv3d_weight_grad(dz: np.ndarray, x: np.ndarray, stride: int = 1):
    """(dL/dw [Cout, Cin, 3, 3, 3], dL/db [Cout]) of ``conv3d`` given the
    output gradient dz and the input x."""
    dz = np.asarray(dz, dtype=np.float64)
    xp = np.pad(np.asarray(x, dtype=np.float64), ((0, 0), (1, 1), (1, 1), (1, 1)))
    O0, O1, O2 = dz.shape[1:]
    dw = np.zeros((dz.shape[0], x.shape[0], 3, 3, 3))
    for a in range(3):
        for bb in range(3):
            for c in range(3):
                patch = xp[:, a:a + stride * O0:stride, bb:bb + stride * O1:stride,
                           c:c + stride * O2:stride]
                dw[:, :, a, bb, c] = np.tensordot(dz, patch, axes=([1, 2, 3], [1, 2, 3]))
    return dw, dz.sum(axis=(1, 2, 3))


def down2_sum(x: np.ndarray) -> np.ndarray:
    """Adjoint of ``up2_nearest``: the sum over each 2x2x2 block."""
    C, D0, D1, D2 = x.shape
    return x.reshape(C, D0 // 2, 2, D1 // 2, 2, D2 // 2, 2).sum(axis=(2, 4, 6))


def backward(params: dict, atlas: np.ndarray, images: np.ndarray, targets: np.ndarray,
             rounded: bool = True):
    """Loss mean((UNet(A, I_i) - v_i)^2) over all subjects and entries, and its
    gradients {layer: (dw, db)}."""
    rb = bf16 if rounded else (lambda a: np.asarray(a, dtype=np.float64))
    n = len(images)
    count = n * targets[0].size
    grads = {name: (0.0, 0.0) for name, *_ in layer_specs()}
    loss = 0.0
    for i in range(n):
        inp, out = {}, {}

        def layer(name, x, stride=1, act=True):
            inp[name] = x
            z = conv3d(x, *params[name], stride)
            out[name] = rb(leaky(z)) if act else z
            return out[name]

        x = rb(np.stack([atlas, images[i]]))
        e0 = layer("e0", x)
        e1 = layer("e1", e0, 2)
        e2 = layer("e2", e1, 2)
        e3 = layer("e3", e2, 2)
        d2 = layer("d2", np.concatenate([up2_nearest(e3), e2]))
        d1 = layer("d1", np.concatenate([up2_nearest(d2), e1]))
        d0 = layer("d0", np.concatenate([up2_nearest(d1), e0]))
        v = layer("out", d0, act=False)
        diff = v - targets[i]
        loss += float((diff ** 2).sum()) / count
        dy = {"out": 2.0 * diff / count}
        strides = {name: s for name, _, _, s, _ in layer_specs()}
        acts = {name: a for name, _, _, _, a in layer_specs()}
        for name in ("out", "d0", "d1", "d2", "e3", "e2", "e1", "e0"):
            g = dy[name]
            if acts[name]:
                g = g * np.where(out[name] > 0, 1.0, SLOPE)
            dz = rb(g)
            dw, db = conv3d_weight_grad(dz, inp[name], strides[name])
            grads[name] = (grads[name][0] + dw, grads[name][1] + db)
            if name == "e0":
                break
            dx = conv3d_input_grad(dz, params[name][0], inp[name].shape[1:], strides[name])
            if name == "out":
                dy["d0"] = dx
            elif name in ("d0", "d1", "d2"):
                deep, skip = {"d0": ("d1", "e0"), "d1": ("d2", "e1"), "d2": ("e3", "e2")}[name]
                cd = params[deep][0].shape[0]
                dy[deep] = down2_sum(dx[:cd])
                dy[skip] = dx[cd:]
            else:
                prev = {"e3": "e2", "e2": "e1", "e1": "e0"}[name]
                dy[prev] = dy[prev] + dx
    return loss, grads
