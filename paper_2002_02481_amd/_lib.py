"""ctypes declarations of liblvmc.so (include/lvmc.h).

Argument marshalling only: every step of the pricing path runs in the HIP
library.  There is no fallback: if the library is missing the import of the
binding raises.
"""
from __future__ import annotations

import ctypes as C
import os
import re

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIBRARY = os.path.join(PKG, "liblvmc.so")
HEADER = os.path.join(ROOT, "include", "lvmc.h")

LV_OK, LV_ERR_ARG, LV_ERR_GRID, LV_ERR_STEP, LV_ERR_NOMEM, LV_ERR_HIP, LV_ERR_UNSUPPORTED = range(7)
STATUS_NAMES = {0: "LV_OK", 1: "LV_ERR_ARG", 2: "LV_ERR_GRID", 3: "LV_ERR_STEP", 4: "LV_ERR_NOMEM",
                5: "LV_ERR_HIP", 6: "LV_ERR_UNSUPPORTED"}
LV_AXIS_LIN, LV_AXIS_LOG = 0, 1
LV_ADJ_DEFAULT, LV_ADJ_NONE, LV_ADJ_STORED, LV_ADJ_CHECKPOINT = 0, 1, 2, 3
KERNEL_KINDS = ("fwd", "rev", "fused", "merge", "table")
ADJOINT = {"default": 0, "none": 1, "stored": 2, "checkpoint": 3}


class lv_axis(C.Structure):
    _fields_ = [("n", C.c_int32), ("kind", C.c_int32), ("lo", C.c_double), ("hi", C.c_double)]


class lv_grid(C.Structure):
    _fields_ = [("spot", lv_axis), ("time", lv_axis)]


class lv_book(C.Structure):
    _fields_ = [("n_opt", C.c_int32), ("is_put", C.POINTER(C.c_int32)),
                ("strike", C.POINTER(C.c_double)), ("maturity", C.POINTER(C.c_double)),
                ("weight", C.POINTER(C.c_double))]


class lv_opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("adjoint", C.c_int32), ("ckpt_every", C.c_int32),
                ("use_graph", C.c_int32), ("block", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("copies", C.c_int32), ("window", C.c_int32), ("profile", C.c_int32),
                ("autotune", C.c_int32), ("fwd_block", C.c_int32), ("fwd_blocks_per_cu", C.c_int32),
                ("dense_adjoint", C.c_int32), ("profile_kinds", C.c_int32), ("scheme", C.c_int32),
                ("sigma_bf16", C.c_int32), ("rate", C.c_double)]


class lv_run_info(C.Structure):
    _fields_ = [("n_blocks", C.c_int32), ("block", C.c_int32), ("tile_paths", C.c_int32),
                ("waves_per_block", C.c_int32), ("fixed_point_bits", C.c_int32),
                ("adjoint", C.c_int32), ("precision", C.c_int32), ("graph_replayed", C.c_int32),
                ("copies", C.c_int32), ("window", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("autotuned", C.c_int32), ("fwd_block", C.c_int32), ("fwd_blocks_per_cu", C.c_int32),
                ("fwd_blocks", C.c_int32), ("overflow_terms", C.c_int64), ("hist_window", C.c_int32)]


class LVError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_vp, _dp, _i32, _i64, _u64 = C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.c_int64, C.c_uint64
_PG, _PB, _PO = C.POINTER(lv_grid), C.POINTER(lv_book), C.POINTER(lv_opts)

SIGNATURES = {
    "lv_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, _vp]),
    "lv_tuning_save": (C.c_int, [_vp, C.c_char_p, C.POINTER(C.c_int32)]),
    "lv_tuning_load": (C.c_int, [_vp, C.c_char_p, C.POINTER(C.c_int32)]),
    "lv_destroy": (None, [_vp]),
    "lv_set_stream": (C.c_int, [_vp, _vp]),
    "lv_last_error": (C.c_char_p, [_vp]),
    "lv_check": (C.c_int, [_PG, _vp, C.c_double, _PB, _i64, _i32, _PO]),
    "lv_price_and_grad": (C.c_int, [_vp, _PG, _vp, C.c_double, _PB, _i64, _i32, _u64, _PO,
                                    _vp, _vp, _vp, _vp]),
    "lv_price_and_grad_batch": (C.c_int, [_vp, _PG, _i32, _vp, C.c_double, _PB, _i64, _i32, _u64,
                                          _PO, _vp, _vp, _vp, _vp]),
    "lv_price_and_grad_dev": (C.c_int, [_vp, _PG, _i32, _vp, C.c_double, _PB, _i64, _i32, _u64,
                                        _PO, _vp, _vp, _vp, _vp]),
    "lv_price_and_grad_noalloc": (C.c_int, [_vp, _PG, _i32, _vp, C.c_double, _PB, _i64, _i32, _u64,
                                            _PO, _vp, _vp, _vp, _vp]),
    "lv_bump_grad_dev": (C.c_int, [_vp, _PG, _vp, C.c_double, _PB, _i64, _i32, _u64, _PO, C.c_double,
                                   _i32, _vp]),
    "lv_states_bytes": (C.c_int, [_i32, _i64, _i32, C.POINTER(C.c_size_t)]),
    "lv_forward_dev": (C.c_int, [_vp, _PG, _vp, C.c_double, _PB, _i64, _i32, _u64, _i32, C.c_double,
                                 _vp, _vp, _vp]),
    "lv_backward_dev": (C.c_int, [_vp, _PG, _vp, C.c_double, _PB, _i64, _i32, _u64, _i32, C.c_double,
                                  _vp, _vp, _vp, _vp]),
    "lv_per_option_grads_dev": (C.c_int, [_vp, _PG, _vp, C.c_double, _PB, _i64, _i32, _u64, _i32, C.c_double,
                                          _vp, _vp, _vp]),
    "lv_debug_philox": (C.c_int, [_vp, _u64, _u64, _i32, _u64, _i64, _vp]),
    "lv_debug_normals": (C.c_int, [_vp, _i32, _u64, _u64, _i64, _i32, _vp]),
    "lv_last_run_info": (C.c_int, [_vp, C.POINTER(lv_run_info)]),
    "lv_debug_block_partials": (C.c_int, [_vp, _vp, C.c_size_t]),
    "lv_debug_option_order": (C.c_int, [_PB, _i32, _vp]),
    "lv_kernel_times": (C.c_int, [_vp, _vp, _vp, _i32]),
    "lv_tuning_candidates": (C.c_int, [_PG, _PB, _i64, _i32, _PO, _vp, _i32, C.POINTER(C.c_int32)]),
}


def header_symbols(path: str = HEADER):
    """Function names declared in include/lvmc.h."""
    text = open(path).read()
    return sorted(set(re.findall(r"\b(lv_[a-z_0-9]+)\s*\(", text)))


_lib = None


def load(path: str = LIBRARY):
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run `python __graft_entry__.py` "
                           "(or paper_2002_02481_amd/build.py) first")
    # Load PyTorch's HIP runtime first: the library then binds to that same
    # runtime (same soname), so device pointers and streams are shared with torch
    # and the process holds a single HIP runtime.
    import torch  # noqa: F401
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
