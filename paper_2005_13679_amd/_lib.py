"""ctypes declarations for libmc.so (the C ABI in include/mc.h).

The library is loaded from this package directory.  There is no fallback: if
libmc.so is missing or fails to load, every call raises.
"""

from __future__ import annotations

import ctypes
import os
import threading

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmc.so")

MC_OK = 0
MC_EINVAL = -1
MC_ERANGE = -2
MC_ENOMEM = -3
MC_EHIP = -4

MC_OP_APPLY = 1
MC_OP_RHO1 = 2
MC_OP_RHO2 = 3
MC_OP_RHO1_DIRECT = 5
MC_OP_RHO2_DIRECT = 6
MC_OP_DOT = 4

MC_MAX_M = 32
MC_MAX_N = 65535
MC_TILE = 64
MC_DOT_BLOCKS = 1024

MC_CONJ_A = 1
MC_CONJ_X = 2
MC_CONJ_B = 4
MC_CONJ_Y = 8

c_i32, c_i64, c_p, c_sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t


MC_FORM_PAPER = 0     # double-jump map with M*M slots per removal pair (the paper's)
MC_FORM_REDUCED = 1   # true double jumps only; apply in the case-split form
FORMS = {"paper": MC_FORM_PAPER, "reduced": MC_FORM_REDUCED}


class TableSizes(ctypes.Structure):
    _fields_ = [
        ("dim", c_i64),
        ("tiles", c_i64),
        ("occ_bytes", c_i32),
        ("pair_words", c_i32),
        ("binom_bytes", c_i64),
        ("occ_bytes_total", c_i64),
        ("t1_bytes", c_i64),
        ("pmask_bytes", c_i64),
        ("t2_off_bytes", c_i64),
        ("t2_compact_entries", c_i64),
        ("t2r_compact_entries", c_i64),
    ]


class CTables(ctypes.Structure):
    _fields_ = [
        ("N", c_i32),
        ("M", c_i32),
        ("dim", c_i64),
        ("tiles", c_i64),
        ("binom_d", c_p),
        ("occ_d", c_p),
        ("t1_d", c_p),
        ("pmask_d", c_p),
        ("t2_off_d", c_p),
        ("t2_d", c_p),
        ("t2_entries", c_i64),
        ("t2_required", c_i64),
        ("form", c_i32),
        ("reserved", c_i32),
    ]


# name -> (restype, argtypes)
SIGNATURES = {
    "mc_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "mc_last_hip_error": (ctypes.c_int, []),
    "mc_dim": (c_i64, [c_i32, c_i32]),
    "mc_hash": (ctypes.c_int, [c_i32, c_i32, c_p, c_p]),
    "mc_unhash": (ctypes.c_int, [c_i32, c_i32, c_i64, c_p]),
    "mc_tables_size": (ctypes.c_int, [c_i32, c_i32, ctypes.POINTER(TableSizes)]),
    "mc_build_jump_tables": (ctypes.c_int, [c_i32, c_i32, ctypes.POINTER(CTables), c_p]),
    "mc_build_double_jumps": (ctypes.c_int, [c_i32, c_i32, ctypes.POINTER(CTables), c_p]),
    "mc_hash_batch": (ctypes.c_int, [c_i32, c_i32, ctypes.POINTER(CTables), c_p, c_p, c_i64, c_p]),
    "mc_unhash_batch": (ctypes.c_int, [c_i32, c_i32, ctypes.POINTER(CTables), c_p, c_p, c_i64, c_p]),
    "mc_t2_lookup": (ctypes.c_int, [c_i32, c_i32, ctypes.POINTER(CTables), c_p, c_p, c_i64, c_p]),
    "mc_workspace_size": (ctypes.c_int, [c_i32, c_i32, c_i32, ctypes.POINTER(c_sz)]),
    "mc_apply_stream_columns": (ctypes.c_int, [c_i32, c_i32, ctypes.POINTER(c_i32),
                                               ctypes.POINTER(c_i32)]),
    "mc_apply_H": (ctypes.c_int, [c_i32, c_i32, c_p, c_p, ctypes.POINTER(CTables), c_p, c_p,
                                  c_p, c_sz, c_p]),
    "mc_apply_H_adjoint": (ctypes.c_int, [c_i32, c_i32, c_p, c_p, ctypes.POINTER(CTables), c_p,
                                          c_p, c_p, c_sz, c_p]),
    "mc_zaxpby": (ctypes.c_int, [c_i64, c_p, c_p, c_p, c_p, ctypes.c_double, ctypes.c_uint32,
                                 c_p, c_p]),
    "mc_rho1": (ctypes.c_int, [c_i32, c_i32, ctypes.POINTER(CTables), c_p, c_p, c_p, c_sz, c_p]),
    "mc_rho2": (ctypes.c_int, [c_i32, c_i32, ctypes.POINTER(CTables), c_p, c_p, c_p, c_sz, c_p]),
    "mc_zdotc": (ctypes.c_int, [c_i64, c_p, c_p, c_p, c_p, c_sz, c_p]),
    "mc_zgemv_c": (ctypes.c_int, [c_i32, c_i64, c_p, c_i64, c_p, c_p, c_p, c_sz, c_p]),
    "mc_zgemv_sub": (ctypes.c_int, [c_i32, c_i64, c_p, c_i64, c_p, c_p, c_p]),
    "mc_normalize": (ctypes.c_int, [c_i64, c_p, c_p, c_p, c_p, c_sz, c_p]),
    "mc_tridiag_lowest": (ctypes.c_int, [c_i32, c_p, c_p, c_p]),
    "mc_zgemv_n": (ctypes.c_int, [c_i32, c_i64, c_p, c_i64, c_p, c_p, c_p]),
    "mc_apply_H_sparse": (ctypes.c_int, [c_i32, c_i32, c_p, c_p, ctypes.POINTER(CTables), c_p, c_p,
                                         c_p, c_sz, c_p]),
    "mc_apply_H_direct": (ctypes.c_int, [c_i32, c_i32, c_p, c_p, c_p, c_p, c_p, c_sz, c_p]),
    "mc_apply_H_direct_noalloc": (ctypes.c_int, [c_i32, c_i32, c_p, c_p, c_p, c_p, c_p]),
    "mc_rho1_direct": (ctypes.c_int, [c_i32, c_i32, c_p, c_p, c_p, c_sz, c_p]),
    "mc_rho2_direct": (ctypes.c_int, [c_i32, c_i32, c_p, c_p, c_p, c_sz, c_p]),
    "mc_tridiag_expv": (ctypes.c_int, [c_i32, c_p, c_p, ctypes.c_double, c_p]),
    "mc_lanczos_orth": (ctypes.c_int, [c_i64, c_p, c_p, c_p, c_p, c_p, c_p]),
    "mc_apply_H_direct_adjoint": (ctypes.c_int, [c_i32, c_i32, c_p, c_p, c_p, c_p, c_p, c_sz,
                                                 c_p]),
    "mc_is_hermitian": (ctypes.c_int, [c_i32, c_p, c_p, c_p, c_p]),
    "mc_tables_bytes": (ctypes.c_int, [c_i32, c_i32, c_i32, c_i32, ctypes.POINTER(c_i64)]),
    "mc_choose_double_jumps": (ctypes.c_int, [c_i32, c_p, c_p, c_i32, ctypes.c_double, c_p]),
    "mc_sil_coefficients": (ctypes.c_int, [c_i32, c_p, c_p, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double, c_p, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(c_i32)]),
}


class BatchItem(ctypes.Structure):
    _fields_ = [("tables", ctypes.POINTER(CTables)), ("h_d", c_p), ("g_d", c_p)]


class BatchSchedule(ctypes.Structure):
    _fields_ = [("blocks_per_cu", c_i32), ("order", c_i32), ("solo_tiles", c_i32),
                ("reserved", c_i32)]


SIGNATURES.update({
    "mc_batch_plan_size": (ctypes.c_int, [c_i32, ctypes.POINTER(BatchItem), ctypes.POINTER(c_sz)]),
    "mc_batch_create": (ctypes.c_int, [c_i32, ctypes.POINTER(BatchItem), ctypes.POINTER(BatchSchedule),
                                       c_p, c_sz, c_p, ctypes.POINTER(c_p)]),
    "mc_batch_destroy": (ctypes.c_int, [c_p]),
    "mc_batch_vector_length": (c_i64, [c_p]),
    "mc_batch_apply_H": (ctypes.c_int, [c_p, c_p, c_p, c_p]),
    "mc_batch_dot": (ctypes.c_int, [c_p, c_p, c_p, c_p, c_p]),
    "mc_batch_lanczos_orth": (ctypes.c_int, [c_p, c_p, c_p, c_p, c_p, c_p, c_p]),
    "mc_batch_normalize": (ctypes.c_int, [c_p, c_p, c_p, c_p, c_p]),
    "mc_batch_lanczos_graph": (ctypes.c_int, [c_p, c_i32, c_p, c_p, c_p, c_p, c_p, c_p,
                                              ctypes.POINTER(c_p)]),
    "mc_graph_launch": (ctypes.c_int, [c_p, c_p]),
    "mc_graph_destroy": (ctypes.c_int, [c_p]),
})


class MCError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = _lib
        text = lib.mc_strerror(status).decode() if lib is not None else "?"
        hip = lib.mc_last_hip_error() if lib is not None else 0
        super().__init__(f"{where}: {text} (status {status}, last HIP error {hip})")
        self.status = status


_lock = threading.Lock()
_lib = None


def load():
    """Loads libmc.so once and declares every exported symbol."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        # MC_LIBRARY: another build of the same sources (the sanitizer build)
        path = os.environ.get("MC_LIBRARY") or LIB_PATH
        if not os.path.exists(path):
            raise RuntimeError(
                f"{path} is not built; run `python -m paper_2005_13679_amd.build`")
        lib = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
        return lib


def check(status: int, where: str) -> None:
    if status != MC_OK:
        raise MCError(status, where)
