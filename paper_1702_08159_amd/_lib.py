"""ctypes loader of libmckernel.so (the C interface of include/mckernel.h).

torch is imported first so that the library binds to the HIP runtime torch
already loaded (one runtime per process, shared streams and memory).
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (must be loaded before the HIP library)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmckernel.so")

MCK_OK = 0
STATUS_NAMES = {0: "MCK_OK", 1: "MCK_ERR_INVALID_ARG", 2: "MCK_ERR_UNSUPPORTED", 3: "MCK_ERR_HIP",
                4: "MCK_ERR_NO_MEMORY"}
MCK_CALIB_RBF = 0
MCK_CALIB_MATERN = 1

_lib = None

# name -> (restype, argtypes)
_i64, _u32, _f64, _vp, _int = ctypes.c_int64, ctypes.c_uint32, ctypes.c_double, ctypes.c_void_p, ctypes.c_int
SIGNATURES = {
    "mck_padded_dim": (_i64, [_i64]),
    "mck_status_string": (ctypes.c_char_p, [_int]),
    "mck_last_error": (ctypes.c_char_p, []),
    "mck_fwht": (_int, [_vp, _i64, _i64, _vp]),
    "mck_fastfood_params": (_int, [_u32, _i64, _i64, _f64, _int, _vp, _vp, _vp, _vp, _vp, _vp]),
    "mck_fastfood_forward": (_int, [_vp, _i64, _i64, _i64, _u32, _f64, _int, _vp, _vp]),
    "mck_fastfood_project": (_int, [_vp, _i64, _i64, _i64, _u32, _f64, _int, _vp, _vp]),
    "mck_fastfood_forward_t": (_int, [_vp, _int, _i64, _i64, _i64, _u32, _f64, _int, _vp, _int, _vp]),
    "mck_fastfood_forward_batched": (_int, [_vp, _i64, _vp]),
    "mck_fastfood_forward_scaled": (_int, [_vp, _int, _vp, _i64, _i64, _i64, _u32, _f64, _int, _vp, _int, _vp, _vp]),
    "mck_forward_tuning_get": (_int, [_i64, _vp]),
    "mck_forward_tuning_set": (_int, [_i64, _vp]),
    "mck_autotune_forward_batched": (_int, [_vp, _i64, ctypes.c_int32, _vp]),
    "mck_batched_graph_create": (_int, [_vp, _i64, _vp, _vp]),
    "mck_batched_graph_launch": (_int, [_vp, _vp]),
    "mck_batched_graph_destroy": (None, [_vp]),
    "mck_fastfood_backward": (_int, [_vp, _vp, _i64, _i64, _i64, _u32, _f64, _int, _vp, _vp, _vp, _vp, _vp]),
    "mck_fastfood_forward_p": (_int, [_vp, _i64, _i64, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp]),
    "mck_fastfood_backward_p": (_int, [_vp, _vp, _i64, _i64, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                       _vp, _vp]),
    "mck_fastfood_backward_p_noalloc": (_int, [_vp, _vp, _i64, _i64, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp,
                                               _vp, _vp, _vp]),
    "mck_gen_boxmuller": (_int, [_vp, _vp, _i64, _vp, _vp, _vp]),
    "mck_softmax_xent": (_int, [_vp, _vp, _i64, _i64, _vp, _vp, _vp, _vp]),
    "mck_axpy": (_int, [_vp, _vp, _i64, ctypes.c_float, _vp]),
    "mck_head_logits": (_int, [_vp, _vp, _vp, _i64, _i64, _i64, _vp, _vp]),
    "mck_head_backward": (_int, [_vp, _vp, _vp, _i64, _i64, _i64, _vp, _vp, _vp]),
    "mck_fastfood_train_step": (_int, [_vp, _vp, _i64, _i64, _i64, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp,
                                        ctypes.c_float, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "mck_backward_launch_shape": (_int, [_i64, _i64, _i64, _vp]),
    "mck_shutdown": (None, []),
}


class Instance(ctypes.Structure):
    """mck_instance of the C interface."""
    _fields_ = [("x", _vp), ("batch", _i64), ("d", _i64), ("E", _i64), ("seed", _u32), ("sigma", _f64),
                ("calib", _int), ("phi", _vp)]


class ForwardTuning(ctypes.Structure):
    """mck_forward_tuning of the C interface."""
    _fields_ = [("split", ctypes.c_int32), ("waves", ctypes.c_int32)]


class BackwardShape(ctypes.Structure):
    """mck_backward_shape of the C interface."""
    _fields_ = [("rows_per_pass", ctypes.c_int32), ("passes", ctypes.c_int32), ("esplit", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("rowblocks", _i64)]


class MckError(RuntimeError):
    def __init__(self, status: int, fn: str, msg: str):
        super().__init__("%s failed: %s (%s)" % (fn, STATUS_NAMES.get(status, status), msg))
        self.status = status


def lib():
    """The loaded library; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmckernel.so is not built: run `python -m paper_1702_08159_amd.build` "
                               "(or __graft_entry__.build())")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def call(name: str, *args) -> None:
    st = getattr(lib(), name)(*args)
    if st != MCK_OK:
        msg = lib().mck_last_error().decode(errors="replace")
        raise MckError(st, name, msg)
