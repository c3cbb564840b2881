"""ctypes declarations of the C ABI in include/fmm2d.h (libfmm2d.so).

Loading fails loudly when the library has not been built: there is no other
implementation behind these names.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfmm2d.so")

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, ECAPACITY = 0, -1, -2, -3, -4, -5
MODES = {"fp64": 0, "fp32": 1, "bf16x3": 2, "fp32_acc64": 3}
OPT_PARENT, OPT_SWAP_FINEST, OPT_SWAP_ALL = 1, 2, 4
VFLAG = 0x40000000
TREE_SHRINK = 1

_lib = None

# (name, restype, argtypes)
P = ctypes.c_void_p
I64 = ctypes.c_int64
I32 = ctypes.c_int
D = ctypes.c_double
F = ctypes.c_float
PP = ctypes.POINTER(ctypes.c_void_p)
PI64 = ctypes.POINTER(ctypes.c_int64)
PI32 = ctypes.POINTER(ctypes.c_int)
PD = ctypes.POINTER(ctypes.c_double)

SIGNATURES = [
    ("fmm2d_version", I32, []),
    ("fmm2d_create", I32, [PP, I32, P, P, P, P]),
    ("fmm2d_destroy", I32, [P]),
    ("fmm2d_last_error", ctypes.c_char_p, [P]),
    ("fmm2d_set_stream", I32, [P, P]),
    ("fmm2d_build_tree", I32, [P, P, P, I64, I32]),
    ("fmm2d_connectivity", I32, [P, D]),
    ("fmm2d_connectivity_opt", I32, [P, D, I32]),
    ("fmm2d_connectivity_relaxed", I32, [P, D, D, I32, I32, I32]),
    ("fmm2d_get_relax_bins", I32, [P, P, P]),
    ("fmm2d_evaluate", I32, [P, P, I32, I32, P]),
    ("fmm2d_evaluate_field", I32, [P, P, I32, I32, P, P, P]),
    ("fmm2d_direct", I32, [P, P, P, P, I64, P, I64, P]),
    ("fmm2d_direct_field", I32, [P, P, P, P, I64, P, I64, P, P]),
    ("fmm2d_direct_noalloc", I32, [P, P, P, P, I64, P, I64, P]),
    ("fmm2d_tree_info", I32, [P, PI64, PI32, PI64]),
    ("fmm2d_get_perm", I32, [P, P]),
    ("fmm2d_get_leaf_start", I32, [P, P]),
    ("fmm2d_get_rects", I32, [P, P]),
    ("fmm2d_get_geometry", I32, [P, P]),
    ("fmm2d_set_tree_options", I32, [P, I32]),
    ("fmm2d_list_sizes", I32, [P, I32, PI64, PI64]),
    ("fmm2d_get_lists", I32, [P, I32, P, P, P, P]),
    ("fmm2d_get_xlists", I32, [P, I32, PI64, P, P]),
    ("fmm2d_features", I32, [P, P, P, I64, D, P]),
    ("fmm2d_select", I32, [P, P, P, I64, D, P, PI32, PI32, PD, PI32]),
    ("fmm2d_select_build_tree", I32, [P, P, P, I64, D, P, PI32, PI32, PD, PI32]),
    ("fmm2d_mlp_nparams", I64, [I32]),
    ("fmm2d_mlp_forward", I32, [P, P, P, I64, I32, P]),
    ("fmm2d_mlp_grad", I32, [P, P, P, P, I64, I32, P, P]),
    ("fmm2d_mlp_adam", I32, [P, P, P, P, P, I64, I32, F, F]),
    ("fmm2d_timing", I32, [P, I32]),
    ("fmm2d_get_timings", I32, [P, P, P]),
]

# fmm2d_alloc_fn / fmm2d_free_fn
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)

NFEAT = 92
SELECT_HEADER = 194

PHASES = ["tree", "lists", "upward", "m2l", "l2l", "leaf", "other", "judge", "select", "near_kernel",
          "m2l_kernel", "exchange", "p2l_kernel", "m2p_kernel"]


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libfmm2d.so is not built (run __graft_entry__.build() or "
                           "python paper_1006_2269_amd/build.py): %s" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_names():
    return [s[0] for s in SIGNATURES]
