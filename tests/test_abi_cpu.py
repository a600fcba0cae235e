"""CPU checks of the C ABI: the library loads, exports every symbol that
include/darc.h declares, mirrors its structs, and rejects bad arguments
before touching the GPU.  No kernel runs here."""

import ctypes
import os
import re

import numpy as np
import pytest

from paper_2508_10743_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "darc.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(darc_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        pytest.fail("libdarc.so is not built: run python -m paper_2508_10743_amd.build")
    return L.load()


def test_header_and_binding_declare_the_same_symbols():
    assert header_functions() == sorted(L.PROTOTYPES)


def test_library_exports_every_declared_symbol(lib):
    for name in header_functions():
        assert hasattr(lib, name), name


def test_struct_layouts_match(lib):
    assert lib.darc_sizeof_state() == ctypes.sizeof(L.DarcState)
    assert lib.darc_sizeof_params() == ctypes.sizeof(L.DarcParams)
    assert lib.darc_abi_version() == L.DARC_ABI_VERSION


def _status(lib, rc, expect):
    assert rc == expect, lib.darc_last_error()
    if expect != L.DARC_OK:
        assert lib.darc_last_error()


def test_bad_dims_and_pointers_are_rejected_without_a_gpu(lib):
    dummy = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    _status(lib, lib.darc_warp3d(dummy, dummy, dummy, 1, 1, 4, 4, None), L.DARC_EINVAL)
    _status(lib, lib.darc_warp3d(dummy, dummy, dummy, -1, 4, 4, 4, None), L.DARC_EINVAL)
    _status(lib, lib.darc_warp3d(None, dummy, dummy, 1, 4, 4, 4, None), L.DARC_EINVAL)
    _status(lib, lib.darc_warp3d(dummy, dummy, dummy, 1, 1 << 10, 1 << 10, 1 << 10, None),
            L.DARC_EINVAL)
    _status(lib, lib.darc_exp_svf(dummy, dummy, None, 1, 4, 4, 4, 7, None, 0, None),
            L.DARC_EINVAL)  # u aliases v
    _status(lib, lib.darc_exp_svf(dummy, ctypes.c_void_p(0x2000), None, 1, 4, 4, 4, 17, None, 0,
                                  None), L.DARC_EINVAL)
    # n_sq >= 2 without checkpoints needs a workspace
    _status(lib, lib.darc_exp_svf(dummy, ctypes.c_void_p(0x2000), None, 1, 4, 4, 4, 7, None, 0,
                                  None), L.DARC_EWORKSPACE)
    # without checkpoints the squarings are recomputed: a workspace is required
    _status(lib, lib.darc_exp_svf_bwd(dummy, None, dummy, ctypes.c_void_p(0x2000), 1, 4, 4, 4, 7,
                                      None, 0, None), L.DARC_EWORKSPACE)
    assert lib.darc_exp_svf_bwd_ws_bytes(1, 4, 4, 4, 7, 0) > lib.darc_exp_svf_bwd_ws_bytes(
        1, 4, 4, 4, 7, 1)
    _status(lib, lib.darc_sim_grad(dummy, dummy, 1, 4, 1e-5, dummy, None, 1, 4, 4, 4, None, 0,
                                   None), L.DARC_EINVAL)  # even window
    _status(lib, lib.darc_sim_grad(dummy, dummy, 1, 13, 1e-5, dummy, None, 1, 4, 4, 4, None, 0,
                                   None), L.DARC_EUNSUPPORTED)
    _status(lib, lib.darc_sim_grad(dummy, dummy, 7, 9, 1e-5, dummy, None, 1, 4, 4, 4, None, 0,
                                   None), L.DARC_EINVAL)  # unknown metric
    _status(lib, lib.darc_smooth3d(dummy, dummy, 1, 3, 4, 4, 4, L.DARC_GAUSS, 1.5, None, None, 0,
                                   None), L.DARC_EINVAL)  # in == out
    _status(lib, lib.darc_smooth3d(dummy, ctypes.c_void_p(0x2000), 1, 3, 4, 4, 4, L.DARC_GAUSS,
                                   4.0, None, None, 0, None), L.DARC_EUNSUPPORTED)
    _status(lib, lib.darc_adam_step(dummy, dummy, dummy, dummy, 10, 0, 1e-2, 0.9, 0.999, 1e-8,
                                    None), L.DARC_EINVAL)
    _status(lib, lib.darc_adam_step(dummy, dummy, dummy, dummy, 10, 1, 1e-2, 1.0, 0.999, 1e-8,
                                    None), L.DARC_EINVAL)
    _status(lib, lib.darc_atlas_update(dummy, dummy, None, dummy, 0, 4, 4, 4, None), L.DARC_EINVAL)
    _status(lib, lib.darc_atlas_median(dummy, dummy, None, dummy, 513, 4, 4, 4, None),
            L.DARC_EUNSUPPORTED)
    _status(lib, lib.darc_atlas_sgd(dummy, dummy, 4, 4, 4, 4, 0, 1, 9, 1e-5, 1e-2, 0.9, 0.999,
                                    1e-8, None, dummy, 1 << 30, None), L.DARC_EINVAL)  # batch 0
    _status(lib, lib.darc_atlas_sgd(dummy, dummy, 4, 4, 4, 4, 2, 1, 9, 1e-5, 1e-2, 0.9, 0.999,
                                    1e-8, None, dummy, 16, None), L.DARC_EWORKSPACE)
    _status(lib, lib.darc_segment(dummy, dummy, dummy, 1, 4, 4, 4, 0, dummy, 1 << 30, None),
            L.DARC_EINVAL)  # n_sq 0
    _status(lib, lib.darc_segment(dummy, dummy, dummy, 1, 4, 4, 4, 7, dummy, 16, None),
            L.DARC_EWORKSPACE)
    _status(lib, lib.darc_dice_counts(dummy, dummy, 1, 64, 257, dummy, None), L.DARC_EINVAL)
    _status(lib, lib.darc_down2(dummy, ctypes.c_void_p(0x2000), 1, 6, 6, 5, None), L.DARC_EINVAL)
    _status(lib, lib.darc_up2(dummy, dummy, 1, 6, 6, 6, 2.0, None), L.DARC_EINVAL)  # aliasing
    assert lib.darc_segment_ws_bytes(2, 4, 4, 4, 7) == 2 * lib.darc_segment_ws_bytes(2, 4, 4, 4, 1)


def test_empty_batches_are_no_ops(lib):
    # n = 0 is valid and enqueues nothing
    assert lib.darc_warp3d(None, None, None, 0, 4, 4, 4, None) == L.DARC_OK
    assert lib.darc_exp_svf(None, None, None, 0, 4, 4, 4, 7, None, 0, None) == L.DARC_OK
    assert lib.darc_center(None, None, 0, 4, 4, 4, None) == L.DARC_OK
    assert lib.darc_adam_step(None, None, None, None, 0, 1, 1e-2, 0.9, 0.999, 1e-8,
                              None) == L.DARC_OK


def _params(**kw):
    base = dict(metric=0, win=9, ncc_eps=1e-5, lam=0.01, smooth_sigma=0.0, n_sq=7, k2=5, lr=1e-2,
                beta1=0.9, beta2=0.999, adam_eps=1e-8, center_mode=0, reinit_v=0, batch=0,
                atlas_mode=0, k3=20, atlas_batch=4, atlas_lr=1e-2)
    base.update(kw)
    return L.DarcParams(**base)


def test_sweep_validation_and_workspace_sizes(lib):
    d = ctypes.c_void_p(0x1000)
    st = L.DarcState(d.value, d.value, d.value, d.value, d.value, None, 0, None, 4, 8, 8, 8)
    p = _params()
    V = 8 * 8 * 8
    nbytes = lib.darc_sweep_ws_bytes(ctypes.byref(st), ctypes.byref(p))
    # checkpoints (6) + uN, gU, gA, gB, gV fields for 4 subjects, u_hat, losses
    f = 4 * 3 * V * 4
    assert nbytes >= 11 * f + 4 * 8
    p_lncc = _params(metric=1, smooth_sigma=1.5)
    assert lib.darc_sweep_ws_bytes(ctypes.byref(st), ctypes.byref(p_lncc)) > nbytes
    p_b1 = _params(batch=1)
    assert lib.darc_sweep_ws_bytes(ctypes.byref(st), ctypes.byref(p_b1)) < nbytes
    # the stochastic atlas needs the warped subjects and its own scratch
    p_sgd = _params(metric=1, atlas_mode=2)
    assert lib.darc_sweep_ws_bytes(ctypes.byref(st), ctypes.byref(p_sgd)) >= \
        lib.darc_sweep_ws_bytes(ctypes.byref(st), ctypes.byref(_params(metric=1))) + 4 * V * 4
    # k2 = 0 (atlas and group loss only) and the L1 metric are valid
    assert lib.darc_sweep_ws_bytes(ctypes.byref(st), ctypes.byref(_params(k2=0))) > 0
    assert lib.darc_sweep_ws_bytes(ctypes.byref(st), ctypes.byref(_params(metric=2,
                                                                           atlas_mode=1))) > 0
    for bad in (_params(k2=-1), _params(n_sq=0), _params(metric=1, win=8), _params(lam=-1.0),
                _params(beta2=1.0), _params(center_mode=3), _params(smooth_sigma=5.0),
                _params(metric=3), _params(atlas_mode=3), _params(atlas_mode=2),
                _params(metric=1, atlas_mode=2, k3=0), _params(metric=1, atlas_mode=2,
                                                                atlas_batch=0),
                _params(metric=1, atlas_mode=2, atlas_lr=0.0)):
        assert lib.darc_sweep_ws_bytes(ctypes.byref(st), ctypes.byref(bad)) == 0
        rc = lib.darc_sweep(ctypes.byref(st), ctypes.byref(bad), d, d, 1 << 30, None)
        assert rc in (L.DARC_EINVAL, L.DARC_EUNSUPPORTED)
    # workspace too small / misaligned
    assert lib.darc_sweep(ctypes.byref(st), ctypes.byref(p), d, d, 16, None) == L.DARC_EWORKSPACE
    assert lib.darc_sweep(ctypes.byref(st), ctypes.byref(p), d, ctypes.c_void_p(0x1004),
                          1 << 30, None) == L.DARC_EWORKSPACE


def test_fastdiv_formula_is_exact():
    """The multiply-high division used for voxel coordinates (Granlund &
    Montgomery round-up variant) is exact for every dividend below 2^31."""
    rng = np.random.default_rng(0)
    dividends = np.concatenate([np.arange(0, 1 << 16, dtype=np.uint64),
                                rng.integers(0, 1 << 31, size=200000, dtype=np.uint64),
                                np.array([(1 << 31) - 1], dtype=np.uint64)])
    for d in [1, 2, 3, 7, 8, 9, 13, 32, 37, 96, 112, 128, 160, 192, 224, 1000, 65535, 123457]:
        l = 0
        while (1 << l) < d:
            l += 1
        m = ((1 << 32) * ((1 << l) - d)) // d + 1
        assert m < (1 << 32)
        hi = (dividends * np.uint64(m)) >> np.uint64(32)
        q = (hi + dividends) >> np.uint64(l)
        assert np.array_equal(q, dividends // np.uint64(d)), d


def test_xcd_remap_is_a_bijection():
    """The block remap that gives each XCD a contiguous range of tiles."""
    for total in [1, 7, 8, 9, 63, 64, 65, 1000, 4097]:
        b = np.arange(total)
        per, rem = total // 8, total % 8
        xcd, j = b % 8, b // 8
        mapped = np.where(xcd < rem, xcd * (per + 1) + j, rem * (per + 1) + (xcd - rem) * per + j)
        assert np.array_equal(np.sort(mapped), b)
