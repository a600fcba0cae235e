"""Pins of the warm-start network's oracle: BF16 rounding against PyTorch's
conversion and hand-checked ties, convolutions against PyTorch's conv3d and
a brute-force loop, nearest doubling against interpolate.  CPU only."""

import numpy as np
import pytest
import torch

from oracle import unet_oracle as U


def test_bf16_rounding_ties_and_library():
    one = 1.0
    assert U.bf16(np.array([one]))[0] == 1.0
    assert U.bf16(np.array([1 + 2.0 ** -8]))[0] == 1.0              # tie -> even
    assert U.bf16(np.array([1 + 3 * 2.0 ** -8]))[0] == 1 + 2.0 ** -6  # tie -> even (up)
    assert U.bf16(np.array([1 + 2.0 ** -8 + 2.0 ** -20]))[0] == 1 + 2.0 ** -7
    x = np.random.default_rng(0).normal(size=10000).astype(np.float32) * 10.0 ** \
        np.random.default_rng(1).integers(-20, 20, size=10000)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(U.bf16(x), ref)
    assert np.isnan(U.bf16(np.array([np.nan]))[0])


@pytest.mark.parametrize("stride", [1, 2])
def test_conv3d_matches_torch(stride):
    rng = np.random.default_rng(2)
    x = rng.normal(size=(5, 6, 8, 7))
    w = rng.normal(size=(4, 5, 3, 3, 3))
    b = rng.normal(size=4)
    ref = torch.nn.functional.conv3d(torch.from_numpy(x)[None], torch.from_numpy(w),
                                     torch.from_numpy(b), stride=stride, padding=1)[0].numpy()
    out = U.conv3d(x, w, b, stride)
    assert out.shape == ref.shape
    assert np.abs(out - ref).max() <= 1e-12 * np.abs(ref).max()


def test_conv3d_brute_force():
    rng = np.random.default_rng(3)
    x = rng.normal(size=(2, 3, 4, 3))
    w = rng.normal(size=(2, 2, 3, 3, 3))
    b = np.array([0.5, -1.0])
    out = U.conv3d(x, w, b)
    for co in range(2):
        for o in np.ndindex(3, 4, 3):
            acc = b[co]
            for ci in range(2):
                for a, bb, c in np.ndindex(3, 3, 3):
                    p = (o[0] + a - 1, o[1] + bb - 1, o[2] + c - 1)
                    if all(0 <= p[d] < (3, 4, 3)[d] for d in range(3)):
                        acc += w[co, ci, a, bb, c] * x[(ci,) + p]
            assert out[(co,) + o] == pytest.approx(acc, abs=1e-12)


def test_nearest_doubling_and_shapes():
    x = np.arange(2 * 2 * 3 * 2, dtype=np.float64).reshape(2, 2, 3, 2)
    ref = torch.nn.functional.interpolate(torch.from_numpy(x)[None], scale_factor=2,
                                          mode="nearest")[0].numpy()
    assert np.array_equal(U.up2_nearest(x), ref)
    rng = np.random.default_rng(4)
    params = {}
    for name, cin, cout, _, _ in U.layer_specs():
        params[name] = (U.bf16(rng.normal(0, 0.2, (cout, cin, 3, 3, 3))), rng.normal(0, 0.01, cout))
    v = U.forward(params, rng.uniform(size=(8, 8, 16)), rng.uniform(size=(8, 8, 16)))
    assert v.shape == (3, 8, 8, 16) and np.isfinite(v).all()
    assert U.flops((96, 112, 96)) == pytest.approx(sum(
        2 * 27 * ci * co * 96 * 112 * 96 / 8 ** lev for ci, co, lev in
        [(2, 16, 0), (16, 32, 1), (32, 64, 2), (64, 128, 3), (192, 64, 2), (96, 32, 1),
         (48, 16, 0), (16, 3, 0)]))


def _torch_net(params):
    import torch.nn.functional as F

    tp = {k: (torch.from_numpy(w).requires_grad_(True), torch.from_numpy(b).requires_grad_(True))
          for k, (w, b) in params.items()}

    def fwd(a, i):
        act = lambda x: F.leaky_relu(x, U.SLOPE)
        conv = lambda x, k, s=1: F.conv3d(x, tp[k][0], tp[k][1], stride=s, padding=1)
        up = lambda x: F.interpolate(x, scale_factor=2, mode="nearest")
        x = torch.stack([a, i])[None]
        e0 = act(conv(x, "e0"))
        e1 = act(conv(e0, "e1", 2))
        e2 = act(conv(e1, "e2", 2))
        e3 = act(conv(e2, "e3", 2))
        d2 = act(conv(torch.cat([up(e3), e2], 1), "d2"))
        d1 = act(conv(torch.cat([up(d2), e1], 1), "d1"))
        d0 = act(conv(torch.cat([up(d1), e0], 1), "d0"))
        return conv(d0, "out")[0]

    return tp, fwd


def test_unrounded_backward_matches_autograd():
    rng = np.random.default_rng(5)
    params = {name: (rng.normal(0, 0.3, (co, ci, 3, 3, 3)), rng.normal(0, 0.05, co))
              for name, ci, co, _, _ in U.layer_specs()}
    dims = (8, 8, 16)
    atlas = rng.uniform(size=dims)
    imgs = rng.uniform(size=(2,) + dims)
    tgt = rng.normal(0, 0.1, (2, 3) + dims)
    loss, grads = U.backward(params, atlas, imgs, tgt, rounded=False)
    tp, fwd = _torch_net(params)
    tl = sum(((fwd(torch.from_numpy(atlas), torch.from_numpy(imgs[i])) - torch.from_numpy(tgt[i])) ** 2).sum()
             for i in range(2)) / tgt.size
    tl.backward()
    assert loss == pytest.approx(float(tl), rel=1e-12)
    for name, (w, b) in tp.items():
        assert np.abs(grads[name][0] - w.grad.numpy()).max() <= 1e-10 * np.abs(w.grad.numpy()).max()
        assert np.abs(grads[name][1] - b.grad.numpy()).max() <= 1e-10 * np.abs(b.grad.numpy()).max() + 1e-15


def test_input_gradient_of_strided_conv_is_the_adjoint():
    rng = np.random.default_rng(6)
    x = rng.normal(size=(3, 6, 8, 4))
    w = rng.normal(size=(5, 3, 3, 3, 3))
    for s in (1, 2):
        y = U.conv3d(x, w, np.zeros(5), s)
        dz = rng.normal(size=y.shape)
        dx = U.conv3d_input_grad(dz, w, x.shape[1:], s)
        # <conv(x), dz> = <x, conv^T(dz)>
        assert float((y * dz).sum()) == pytest.approx(float((x * dx).sum()), rel=1e-12)
