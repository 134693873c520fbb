"""ctypes view of the C ABI in include/lmag.h (argument marshalling only).

Loads the in-tree liblmag.so built by ``paper_2511_13330_amd.build``; there is
no fallback: a missing library raises at import time of the first call.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblmag.so")

LMAG_OK = 0
LMAG_E_INVALID = -1
LMAG_E_NOSYSTEM = -2
LMAG_E_NOMEM = -3
LMAG_E_DEVICE = -4
LMAG_E_UNSUPPORTED = -5
LMAG_F32 = 32
LMAG_F64 = 64
LMAG_ZOH = 0
LMAG_FOH = 1
LMAG_SCORE_PROJECTED = 1
LMAG_SCORE_LINEAR = 2

STATUS_NAMES = {0: "LMAG_OK", -1: "LMAG_E_INVALID", -2: "LMAG_E_NOSYSTEM",
                -3: "LMAG_E_NOMEM", -4: "LMAG_E_DEVICE", -5: "LMAG_E_UNSUPPORTED"}

c_void_p = ctypes.c_void_p
c_int = ctypes.c_int
c_double = ctypes.c_double
c_size_t = ctypes.c_size_t
c_int32_p = ctypes.POINTER(ctypes.c_int32)
c_int64_p = ctypes.POINTER(ctypes.c_int64)
c_double_p = ctypes.POINTER(ctypes.c_double)


class SystemDesc(ctypes.Structure):
    _fields_ = [("d", c_int), ("n_static", c_int), ("H_static", c_double_p),
                ("n_ctrl", c_int), ("H_ctrl", c_double_p), ("n_jump", c_int),
                ("L_jump", c_double_p), ("precision", c_int), ("magnus_order", c_int),
                ("hold", c_int), ("workspace_bytes_max", c_size_t),
                ("chunk_slices", c_int), ("basis", c_int)]


class Batch(ctypes.Structure):
    _fields_ = [("n_items", c_int), ("n_slices", c_int32_p), ("slice_offset", c_int64_p),
                ("amps", c_void_p), ("static_coef", c_void_p), ("ctrl_scale", c_void_p),
                ("dt", c_double), ("n_groups", c_int), ("group_of_item", c_int32_p)]


# name -> (restype, argtypes); every symbol include/lmag.h and include/lmag_debug.h declare
SIGNATURES = {
    "lmag_version": (ctypes.c_char_p, []),
    "lmag_create": (c_int, [ctypes.POINTER(c_void_p), c_int]),
    "lmag_destroy": (None, [c_void_p]),
    "lmag_last_error": (ctypes.c_char_p, [c_void_p]),
    "lmag_set_system": (c_int, [c_void_p, ctypes.POINTER(SystemDesc)]),
    "lmag_propagate": (c_int, [c_void_p, ctypes.POINTER(Batch), c_void_p, c_void_p]),
    "lmag_fidelity_and_grad": (c_int, [c_void_p, ctypes.POINTER(Batch), c_void_p, c_int,
                                       c_int32_p, c_void_p, c_void_p, c_void_p]),
    "lmag_fidelity_and_grad_noalloc": (c_int, [c_void_p, ctypes.POINTER(Batch), c_void_p, c_int,
                                               c_int32_p, c_void_p, c_void_p, c_void_p]),
    "lmag_logical_score_and_grad": (c_int, [c_void_p, ctypes.POINTER(Batch), c_int, c_int, c_double_p,
                                            c_void_p, c_int, c_int32_p, c_void_p, c_void_p, c_void_p]),
    "lmag_sync": (c_int, [c_void_p, c_void_p]),
    "lmag_mlp_forward": (c_int, [c_void_p, c_int, c_int, c_int, c_void_p, c_void_p, c_void_p,
                                 c_int, ctypes.c_float, c_void_p, c_void_p, c_void_p]),
    "lmag_mlp_backward": (c_int, [c_void_p, c_int, c_int, c_int, c_void_p, c_void_p, c_void_p,
                                  c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                  c_void_p]),
    "lmag_mlp_mse": (c_int, [c_void_p, ctypes.c_int64, c_void_p, c_void_p, c_void_p, c_void_p,
                             c_void_p, c_void_p]),
    "lmag_cast_bf16": (c_int, [c_void_p, c_void_p, c_void_p, ctypes.c_int64, c_void_p]),
    "lmag_autotune": (c_int, [c_void_p, ctypes.POINTER(Batch), c_void_p, c_int, c_int32_p, c_int,
                              c_int32_p, c_double_p, c_void_p]),
    "lmag_load_tuning": (c_int, [c_void_p, ctypes.c_char_p]),
    "lmag_adam_project": (c_int, [c_void_p, c_int, ctypes.c_int64, c_int, c_void_p, c_void_p,
                                  c_void_p, c_void_p, c_int, c_double, c_double, c_double,
                                  c_double, c_double, c_double, c_double, c_void_p, c_void_p]),
    "lmag_pade_coefficients": (c_int, [c_int, c_double_p]),
    "lmag_pade_theta": (c_int, [c_int, c_int, c_double_p]),
    "lmag_last_selection_histogram": (c_int, [c_void_p, c_int64_p]),
    "lmag_set_profiling": (c_int, [c_void_p, c_int]),
    "lmag_read_profile": (c_int, [c_void_p, c_double_p, c_int64_p]),
    "lmag_last_plan": (c_int, [c_void_p, c_int64_p]),
    "lmag_debug_phase_cycles": (c_int, [c_void_p, c_int, c_int64_p]),
    "lmag_debug_tile_gemm": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_int,
                                     c_void_p]),
    "lmag_debug_tile_inverse": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p]),
    "lmag_debug_block_gemm": (c_int, [c_void_p, c_int, c_int, c_void_p, c_void_p, c_void_p, c_int,
                                      c_void_p]),
    "lmag_debug_tile_expm": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p]),
}

_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} not found: build it with "
                               "`python -m paper_2511_13330_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class LmagError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status, ctx=None):
    if status != LMAG_OK:
        msg = lib().lmag_last_error(ctx).decode() if ctx else ""
        raise LmagError(status, msg)
