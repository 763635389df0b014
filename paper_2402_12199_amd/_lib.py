"""Loader of librigidnn.so (the HIP library) with ctypes signatures.

The product path has no fallback: if the library is missing or lacks a
symbol, importing the binding raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librigidnn.so")

P = C.c_void_p
I32 = C.c_int32
I64 = C.c_int64
F32 = C.c_float
F64 = C.c_double
SZ = C.c_size_t
DP = C.POINTER(C.c_double)
FP = C.POINTER(C.c_float)
IP = C.POINTER(C.c_int32)

# name -> (restype, argtypes)
SIGNATURES = {
    "rb_last_error": (C.c_char_p, []),
    "rb_ctx_create": (C.c_int, [C.POINTER(P), I32, IP, FP, DP, DP, F32, F32, F32]),
    "rb_ctx_destroy": (C.c_int, [P]),
    "rb_ctx_set_hphc": (C.c_int, [P, C.c_double, C.c_double, C.c_double, C.c_double]),
    "rb_pairlist_workspace_bytes": (SZ, [I32, DP, F64]),
    "rb_pairlist_build": (C.c_int, [I32, P, DP, F64, P, P, I32, P, P, C.c_int, P, SZ, P]),
    "rb_pair_descriptors": (C.c_int, [I32, P, P, DP, P, P, I32, F32, F32, P, P, P, P, P, P, F32, F32, P]),
    "rb_pair_descriptors_screened": (C.c_int, [I32, P, P, DP, P, P, I32, F32, F32, P, P, P, P, P, P, F32, F32, F32,
                                                P, P, P, P]),
    "rb_bead_pair_eval": (C.c_int, [P, I64, P, I32, I32, P, P, P]),
    "rb_bead_pair_forces": (C.c_int, [P, I32, P, P, P, DP, P, P, P, P, I32, P, P, P]),
    "rb_bead_pair_forces_screened": (C.c_int, [P, I32, P, P, P, DP, P, P, P, I32, F64, P, P, P, P, P, P, P]),
    "rb_bead_screen": (C.c_int, [P, I32, P, P, P, DP, P, P, P, P, I32, P, P, P, P, P]),
    "rb_accum_zero": (C.c_int, [I32, P, P]),
    "rb_accum_finalize": (C.c_int, [I32, P, P, P, P, P, P]),
    "rb_flags_check": (C.c_int, [IP]),
    "rb_nn_pair_eval": (C.c_int, [P, FP, C.c_int, I64, P, P, P]),
    "rb_nn_pair_grad": (C.c_int, [P, FP, C.c_int, I64, P, P, P, P, P, P]),
    "rb_nn_pair_forces": (C.c_int, [P, FP, C.c_int, I32, P, P, P, P, I32, P, P, I32, F32, F32, P, P,
                                    P]),
    "rb_cube_sym_descriptors": (C.c_int, [I64, P, I64, P, P, I64, P, P, P]),
    "rb_cyl_sym_descriptors": (C.c_int, [I64, P, I64, P, P, I64, P, P, P]),
    "rb_nn_pair_forces_cyl": (C.c_int, [P, FP, C.c_int, I32, P, P, P, P, I32, P, P, I32, F32, F32, P, P, P]),
    "rb_nn_pair_forces_routed": (C.c_int, [P, P, FP, C.c_int, C.c_int, I32, P, P, P, P, P, P, P, I32, P, P, P, P,
                                           I32, F32, F32, P, P, P]),
    "rb_nn_pair_grad_sym": (C.c_int, [P, FP, C.c_int, I64, P, P, P, P, P, P, P, P]),
    "rb_nn_pair_forces_sym": (C.c_int, [P, FP, C.c_int, I32, P, P, P, P, I32, P, P, P, P, I32, F32, F32, P, P,
                                        P]),
    "rb_rigid_workspace_bytes": (SZ, [I32]),
    "rb_rigid_step": (C.c_int, [P, C.c_int, I32, F64, P, P, P, P, P, P, P, P, F64, P, P, F64, P, P, P, P, SZ,
                                P]),
    "rb_rigid_step_fused": (C.c_int, [P, I32, F64, P, P, P, P, P, P, P, P, P, P, F64, P, P, F64, P, P, P, SZ,
                                      P]),
    "rb_rigid_step_fused_noalloc": (C.c_int, [P, I32, F64, P, P, P, P, P, P, P, P, P, P, F64, P, P, F64, P, P,
                                              P]),
    "rb_rigid_step_fused_noalloc_max_bodies": (SZ, []),
    "rb_nn_train_workspace_bytes": (SZ, [I32]),
    "rb_nn_train_fm_workspace_bytes": (SZ, [I32]),
    "rb_nn_train_step_fm": (C.c_int, [P, P, P, I32, FP, C.c_int, I32, P, I64, P, P, P, F32, F32, F32, F32, F32,
                                      F32, P, P, P, SZ, P]),
    "rb_nn_train_step": (C.c_int, [P, P, P, I32, FP, C.c_int, I32, P, I64, P, P, F32, F32, F32, F32,
                                   P, P, P, SZ, P]),
}

_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is not built; run `python -m paper_2402_12199_amd.build` "
                "(or __graft_entry__.build()) first")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)  # AttributeError if the symbol is missing
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class RigidNNError(RuntimeError):
    pass


def check(rc: int, what: str) -> None:
    if rc != 0:
        msg = lib().rb_last_error().decode(errors="replace")
        raise RigidNNError(f"{what} failed ({rc}): {msg}")
