"""ctypes binding of libjc (include/jc.h): argument marshalling only.

Every step of the Jacobi3D path runs in the HIP kernels of libjc.so; this
module only declares the C signatures and turns negative status codes into
exceptions.  There is no fallback: if the library is missing the import of
this module fails.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libjc.so")

JC_OK = 0
JC_MAXITER = 1
JC_ERR_INVALID = -1
JC_ERR_NOMEM = -2
JC_ERR_DEVICE = -3
JC_ERR_STATE = -4
JC_ERR_NONFINITE = -5
JC_STATIC_SCRATCH_BYTES = 16 << 20     # jc_group_bind_static: per-device static scratch

JC_F64, JC_F32, JC_BF16, JC_NONE = 0, 1, 2, -1
JC_FIELD_U, JC_FIELD_B = 0, 1
JC_MODE_STAGED, JC_MODE_FUSED = 0, 1
JC_EXCHANGE_DEVICE, JC_EXCHANGE_HOST, JC_EXCHANGE_METADATA = 0, 1, 2
(JC_K_SWEEP, JC_K_PACK, JC_K_EXCHANGE, JC_K_UNPACK, JC_K_RESIDUAL, JC_K_FUSED,
 JC_K_IR_INNER, JC_K_IR_OUTER, JC_K_SWEEP2, JC_K_SWEEP3, JC_K_RESIDENT) = range(11)

_NAMES = {JC_ERR_INVALID: "JC_ERR_INVALID", JC_ERR_NOMEM: "JC_ERR_NOMEM",
          JC_ERR_DEVICE: "JC_ERR_DEVICE", JC_ERR_STATE: "JC_ERR_STATE",
          JC_ERR_NONFINITE: "JC_ERR_NONFINITE"}


class JcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (_NAMES.get(code, "JC_ERR"), code, msg))
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("with_source", ctypes.c_int), ("ir_dtype", ctypes.c_int),
                ("ir_enable", ctypes.c_int), ("tile_y", ctypes.c_int), ("z_chunk", ctypes.c_int),
                ("use_graphs", ctypes.c_int), ("debug_epochs", ctypes.c_int), ("tile_x", ctypes.c_int),
                ("exchange", ctypes.c_int), ("temporal", ctypes.c_int), ("overlap", ctypes.c_int),
                ("sweeps_per_launch", ctypes.c_int), ("resident", ctypes.c_int)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int64), ("outer", ctypes.c_int64), ("rel_resid", ctypes.c_double),
                ("abs_resid", ctypes.c_double), ("r0", ctypes.c_double), ("status", ctypes.c_int),
                ("history", ctypes.POINTER(ctypes.c_double)), ("history_cap", ctypes.c_int64),
                ("history_len", ctypes.c_int64)]


I64 = ctypes.c_int64
I64P = ctypes.POINTER(ctypes.c_int64)
VP = ctypes.c_void_p
CTX = ctypes.c_void_p

# name: (restype, argtypes); mirrors include/jc.h
SIGNATURES = {
    "jc_footprint": (ctypes.c_int, [I64P, I64P, ctypes.POINTER(Options), ctypes.POINTER(ctypes.c_size_t)]),
    "jc_footprint_rectilinear": (ctypes.c_int, [I64P, ctypes.POINTER(I64P), I64P, ctypes.POINTER(Options),
                                                ctypes.POINTER(ctypes.c_size_t)]),
    "jc_min_surface_parts": (ctypes.c_int, [I64P, I64, I64P]),
    "jc_create": (ctypes.c_int, [I64P, I64P, ctypes.POINTER(Options), ctypes.POINTER(CTX)]),
    "jc_create_rectilinear": (ctypes.c_int, [I64P, ctypes.POINTER(I64P), I64P, ctypes.POINTER(Options),
                                             ctypes.POINTER(CTX)]),
    "jc_bind": (ctypes.c_int, [CTX, VP, ctypes.c_size_t, VP]),
    "jc_destroy": (None, [CTX]),
    "jc_last_error": (ctypes.c_char_p, []),
    "jc_load_field": (ctypes.c_int, [CTX, ctypes.c_int, VP]),
    "jc_store_field": (ctypes.c_int, [CTX, ctypes.c_int, VP]),
    "jc_pack_faces": (ctypes.c_int, [CTX]),
    "jc_exchange": (ctypes.c_int, [CTX]),
    "jc_unpack_faces": (ctypes.c_int, [CTX]),
    "jc_sweep": (ctypes.c_int, [CTX]),
    "jc_iterate": (ctypes.c_int, [CTX, I64]),
    "jc_residual": (ctypes.c_int, [CTX, ctypes.POINTER(ctypes.c_double)]),
    "jc_solve": (ctypes.c_int, [CTX, ctypes.c_double, I64, I64, ctypes.POINTER(SolveInfo)]),
    "jc_solve_ir": (ctypes.c_int, [CTX, ctypes.c_int, ctypes.c_double, I64, ctypes.POINTER(SolveInfo)]),
    "jc_group_create": (ctypes.c_int, [ctypes.POINTER(CTX), ctypes.c_int, VP, ctypes.c_int,
                                       ctypes.POINTER(ctypes.c_int), ctypes.POINTER(VP)]),
    "jc_group_footprint": (ctypes.c_int, [VP, ctypes.POINTER(ctypes.c_size_t)]),
    "jc_group_bind": (ctypes.c_int, [VP, VP, ctypes.c_size_t]),
    "jc_group_bind_static": (ctypes.c_int, [VP]),
    "jc_group_check": (ctypes.c_int, [VP, ctypes.c_double, I64, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_int)]),
    "jc_set_pace": (ctypes.c_int, [CTX, I64]),
    "jc_get_pace": (I64, [CTX]),
    "jc_autotune_pace": (ctypes.c_int, [CTX, ctypes.c_int, I64P]),
    "jc_group_iterate": (ctypes.c_int, [VP, I64]),
    "jc_group_residuals": (ctypes.c_int, [VP, ctypes.POINTER(ctypes.c_double)]),
    "jc_group_destroy": (None, [VP]),
    "jc_synth_field": (ctypes.c_int, [VP, I64P, ctypes.c_uint64, ctypes.c_int, VP]),
    "jc_num_blocks": (I64, [CTX]),
    "jc_num_pairs": (I64, [CTX]),
    "jc_num_items": (I64, [CTX]),
    "jc_iterations": (I64, [CTX]),
    "jc_block_info": (ctypes.c_int, [CTX, I64, I64P]),
    "jc_pair_info": (ctypes.c_int, [CTX, I64, I64P]),
    "jc_tile_info": (ctypes.c_int, [CTX, I64P]),
    "jc_set_tiles": (ctypes.c_int, [CTX, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "jc_autotune": (ctypes.c_int, [CTX, ctypes.c_int, I64P]),
    "jc_set_temporal_tiles": (ctypes.c_int, [CTX, ctypes.c_int, ctypes.c_int]),
    "jc_temporal_info": (ctypes.c_int, [CTX, I64P]),
    "jc_set_timing": (ctypes.c_int, [CTX, ctypes.c_int]),
    "jc_kernel_time": (ctypes.c_int, [CTX, ctypes.c_int, ctypes.POINTER(ctypes.c_double), I64P]),
}


def _load():
    # torch ships its own HIP runtime; load it first so that libjc binds to
    # that same runtime (one runtime per process: shared memory and streams)
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError("libjc.so is not built (%s); run `python paper_2102_12416_amd/build.py`"
                          % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def last_error() -> str:
    msg = lib.jc_last_error()
    return msg.decode() if msg else ""


def check(code: int) -> int:
    """Raise JcError for a negative status; return it otherwise."""
    if code < 0:
        raise JcError(code, last_error())
    return code


def i64(values):
    arr = (ctypes.c_int64 * len(values))(*[int(v) for v in values])
    return arr
