"""ctypes declarations of libdarc's C ABI (``include/darc.h``).

This module only describes the exported symbols (names, argument and result
types, the two structs); loading the in-tree ``libdarc.so`` happens in
:func:`load`.  Every argument is a plain pointer or integer: no torch type
crosses the boundary.
"""

from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_float, c_int, c_longlong, c_size_t, c_void_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdarc.so")

DARC_ABI_VERSION = 4

DARC_OK = 0
DARC_EINVAL = -1
DARC_EHIP = -2
DARC_EWORKSPACE = -3
DARC_EUNSUPPORTED = -4

DARC_MSE = 0
DARC_LNCC = 1
DARC_L1 = 2
DARC_ATLAS_MEAN = 0
DARC_ATLAS_MEDIAN = 1
DARC_ATLAS_SGD = 2
DARC_SGD_INIT_WARM = 0
DARC_SGD_INIT_INITIAL = 1
DARC_FUSED_AUTO = 0
DARC_FUSED_OFF = 1
DARC_FUSED_ON = 2
DARC_SHAPE_SQUARING = 0
DARC_SHAPE_WINDOW = 1
DARC_SHAPE_FUSED = 2
DARC_GAUSS = 0
DARC_DIFFUSION = 1
DARC_CENTER_DISPLACEMENT = 0
DARC_CENTER_VELOCITY = 1

STATUS_NAMES = {
    DARC_EINVAL: "DARC_EINVAL",
    DARC_EHIP: "DARC_EHIP",
    DARC_EWORKSPACE: "DARC_EWORKSPACE",
    DARC_EUNSUPPORTED: "DARC_EUNSUPPORTED",
}


class DarcState(ctypes.Structure):
    """Mirror of ``darc_state``."""

    _fields_ = [
        ("images", c_void_p),
        ("v", c_void_p),
        ("m", c_void_p),
        ("s", c_void_p),
        ("atlas", c_void_p),
        ("u_hat", c_void_p),
        ("step", c_longlong),
        ("step_dev", c_void_p),
        ("n", c_int),
        ("d0", c_int),
        ("d1", c_int),
        ("d2", c_int),
    ]


class DarcParams(ctypes.Structure):
    """Mirror of ``darc_params``."""

    _fields_ = [
        ("metric", c_int),
        ("win", c_int),
        ("ncc_eps", c_float),
        ("lam", c_float),
        ("smooth_sigma", c_float),
        ("n_sq", c_int),
        ("k2", c_int),
        ("lr", c_float),
        ("beta1", c_double),
        ("beta2", c_double),
        ("adam_eps", c_float),
        ("center_mode", c_int),
        ("reinit_v", c_int),
        ("batch", c_int),
        ("atlas_mode", c_int),
        ("k3", c_int),
        ("atlas_batch", c_int),
        ("atlas_lr", c_float),
        ("sgd_init", c_int),
        ("fused", c_int),
    ]


class DarcUnetTrain(ctypes.Structure):
    """Mirror of ``darc_unet_train``."""

    _fields_ = [(name, c_void_p) for name in ("w", "b", "mw", "sw", "mb", "sb", "wq", "dw", "db")] + [
        ("step", c_longlong)]


_P = c_void_p  # device pointer
_I = c_int
_Z = c_size_t

PROTOTYPES = {
    "darc_abi_version": (c_int, []),
    "darc_last_error": (c_char_p, []),
    "darc_exp_svf_ws_bytes": (c_size_t, [_I, _I, _I, _I, _I, _I]),
    "darc_exp_svf": (c_int, [_P, _P, _P, _I, _I, _I, _I, _I, _P, _Z, _P]),
    "darc_exp_svf_bwd_ws_bytes": (c_size_t, [_I, _I, _I, _I, _I, _I]),
    "darc_exp_svf_bwd": (c_int, [_P, _P, _P, _P, _I, _I, _I, _I, _I, _P, _Z, _P]),
    "darc_warp3d": (c_int, [_P, _P, _P, _I, _I, _I, _I, _P]),
    "darc_warp3d_bwd": (c_int, [_P, _P, _P, _P, _I, _I, _I, _I, _P]),
    "darc_sim_grad_ws_bytes": (c_size_t, [_I, _I, _I, _I, _I]),
    "darc_sim_grad": (c_int, [_P, _P, _I, _I, c_float, _P, _P, _I, _I, _I, _I, _P, _Z, _P]),
    "darc_sim_grad_noalloc_max_bytes": (c_size_t, []),
    "darc_sim_grad_noalloc": (c_int, [_P, _P, _I, _I, c_float, _P, _P, _I, _I, _I, _I, _P]),
    "darc_smooth3d": (c_int, [_P, _P, _I, _I, _I, _I, _I, _I, c_float, _P, _P, _Z, _P]),
    "darc_adam_step": (c_int, [_P, _P, _P, _P, c_longlong, c_longlong, c_float, c_double,
                               c_double, c_float, _P]),
    "darc_center": (c_int, [_P, _P, _I, _I, _I, _I, _P]),
    "darc_atlas_update": (c_int, [_P, _P, _P, _P, _I, _I, _I, _I, _P]),
    "darc_atlas_median": (c_int, [_P, _P, _P, _P, _I, _I, _I, _I, _P]),
    "darc_atlas_sgd_ws_bytes": (c_size_t, [_I, _I, _I, _I, _I]),
    "darc_atlas_sgd": (c_int, [_P, _P, _I, _I, _I, _I, _I, _I, _I, c_float, c_float, c_double,
                               c_double, c_float, _P, _P, _Z, _P]),
    "darc_warp_labels": (c_int, [_P, _P, _P, _I, _I, _I, _I, _P]),
    "darc_segment_ws_bytes": (c_size_t, [_I, _I, _I, _I, _I]),
    "darc_segment": (c_int, [_P, _P, _P, _I, _I, _I, _I, _I, _P, _Z, _P]),
    "darc_dice_counts": (c_int, [_P, _P, _I, c_longlong, _I, _P, _P]),
    "darc_conv3d_kpad": (c_int, [_I, _I]),
    "darc_conv3d": (c_int, [_P, _I, _I, _P, _I, _I, _I, _I, _I, _I, _I, _P, _P, _I, _I, c_float,
                            _P, _P, _P]),
    "darc_conv3d_grad": (c_int, [_P, _I, _P, _I, _I, _P, _I, _I, _I, _I, _I, _I, _P, _I, _P, _P,
                                 _P, _P, _P]),
    "darc_unet_layout": (c_int, [_I, POINTER(c_int), POINTER(c_int), POINTER(c_int),
                                 POINTER(c_size_t), POINTER(c_size_t)]),
    "darc_unet_ws_bytes": (c_size_t, [_I, _I, _I, _I]),
    "darc_unet_num_weights": (c_size_t, []),
    "darc_unet_num_biases": (c_int, []),
    "darc_unet_train_ws_bytes": (c_size_t, [_I, _I, _I, _I]),
    "darc_unet_backward": (c_int, [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _I, _I, _I, _I, _P, _Z,
                                   _P]),
    "darc_unet_train_step": (c_int, [POINTER(DarcUnetTrain), _P, _P, _P, c_float, c_double,
                                     c_double, c_float, _P, _I, _I, _I, _I, _P, _Z, _P]),
    "darc_unet_forward": (c_int, [_P, _P, _P, _P, _P, _I, _I, _I, _I, _P, _Z, _P]),
    "darc_down2": (c_int, [_P, _P, _I, _I, _I, _I, _P]),
    "darc_up2": (c_int, [_P, _P, _I, _I, _I, _I, c_float, _P]),
    "darc_sizeof_state": (c_size_t, []),
    "darc_sizeof_params": (c_size_t, []),
    "darc_sweep_ws_bytes": (c_size_t, [POINTER(DarcState), POINTER(DarcParams)]),
    "darc_sweep": (c_int, [POINTER(DarcState), POINTER(DarcParams), _P, _P, _Z, _P]),
    "darc_autotune": (c_int, [POINTER(DarcState), POINTER(DarcParams), _P, _Z, _P,
                              POINTER(c_int)]),
    "darc_autotune_clear": (c_int, []),
    "darc_fused_barrier_ticks": (c_int, [c_longlong]),
    "darc_set_launch_shape": (c_int, [_I, _I, _I, _I, _I, _I]),
    "darc_profile_enable": (c_int, [_I]),
    "darc_profile_reset": (c_int, []),
    "darc_profile_num_classes": (c_int, []),
    "darc_profile_name": (c_char_p, [_I]),
    "darc_profile_collect": (c_int, [POINTER(c_longlong), POINTER(c_double), _I]),
    "darc_bw_copy": (c_int, [_P, _P, _Z, _I, _P]),
    "darc_bw_read": (c_int, [_P, _Z, _P, _I, _P]),
    "darc_bw_write": (c_int, [_P, _Z, _I, _P]),
}


class DarcError(RuntimeError):
    """A libdarc call returned a negative status."""

    def __init__(self, fn: str, status: int, message: str):
        super().__init__(f"{fn}: {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def declare(lib: ctypes.CDLL) -> ctypes.CDLL:
    """Attach argument and result types of every ABI symbol to ``lib``."""
    for name, (res, args) in PROTOTYPES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


def check(lib: ctypes.CDLL, fn: str, status: int) -> None:
    if status != DARC_OK:
        raise DarcError(fn, status, lib.darc_last_error().decode(errors="replace"))


_LIB = None


def load() -> ctypes.CDLL:
    """Load the in-tree libdarc.so (built by ``paper_2508_10743_amd.build``).

    torch is imported first so that its HIP runtime is the one the library
    binds to (both carry the soname libamdhip64.so.7).  A missing library is
    an error: there is no fallback implementation.
    """
    global _LIB
    if _LIB is not None:
        return _LIB
    import torch  # noqa: F401  (loads the HIP runtime libdarc links against)

    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2508_10743_amd.build`")
    lib = declare(ctypes.CDLL(LIB_PATH))
    if lib.darc_abi_version() != DARC_ABI_VERSION:
        raise ImportError(f"libdarc ABI {lib.darc_abi_version()} != {DARC_ABI_VERSION}")
    if lib.darc_sizeof_state() != ctypes.sizeof(DarcState) or \
            lib.darc_sizeof_params() != ctypes.sizeof(DarcParams):
        raise ImportError("libdarc struct layout does not match the binding")
    _LIB = lib
    return lib
