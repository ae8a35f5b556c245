"""ctypes wrapper around the plain-C oracle ``mc_oracle.c`` (test infrastructure only).

``build()`` compiles ``mc_oracle.c`` with gcc into ``oracle/_build/``; the
functions below load it on first use.  All complex arrays are complex128.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mc_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB = os.path.join(_BUILD, "libmc_oracle.so")

_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle (gcc -O2 -fopenmp).  Returns the library path."""
    os.makedirs(_BUILD, exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            # MC_ORACLE_LIBRARY: another build of mc_oracle.c (the sanitizer build)
            path = os.environ.get("MC_ORACLE_LIBRARY")
            if not path:
                build(force=False)
                path = _LIB
            lib = ctypes.CDLL(path)
            i32, i64, p = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
            lib.orc_nc.argtypes = [i64, i64]
            lib.orc_nc.restype = i64
            lib.orc_hash.argtypes = [i32, i32, p]
            lib.orc_hash.restype = i64
            lib.orc_unhash.argtypes = [i32, i32, i64, p]
            lib.orc_unhash.restype = ctypes.c_int
            lib.orc_apply_h_rows.argtypes = [i32, i32, p, p, p, p, i64, p]
            lib.orc_rho1.argtypes = [i32, i32, p, p]
            lib.orc_rho2.argtypes = [i32, i32, p, p]
            lib.orc_rho2_elements.argtypes = [i32, i32, p, p, i64, p]
            lib.orc_occ_rows.argtypes = [i32, i32, p, i64, p]
            lib.orc_t1_rows.argtypes = [i32, i32, p, i64, p]
            lib.orc_t2_row_lengths.argtypes = [i32, i32, p, i64, p]
            lib.orc_t2_rows.argtypes = [i32, i32, p, i64, p, p]
            lib.orc_t2r_row_lengths.argtypes = [i32, i32, p, i64, p]
            lib.orc_t2r_rows.argtypes = [i32, i32, p, i64, p, p]
            lib.orc_hash_rows.argtypes = [i32, i32, p, i64, p]
            _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.complex128)


def _rows(rows, D):
    if rows is None:
        return np.arange(D, dtype=np.int64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    if rows.size and (rows.min() < 0 or rows.max() >= D):
        raise ValueError("row index out of range")
    return rows


def nc(n: int, m: int) -> int:
    return int(_load().orc_nc(n, m))


def dim(N: int, M: int) -> int:
    return nc(N, M)


def hash_occ(occ, N: int) -> int:
    occ = np.ascontiguousarray(occ, dtype=np.int32)
    return int(_load().orc_hash(N, occ.size, _ptr(occ)))


def hash_rows(occ: np.ndarray, N: int) -> np.ndarray:
    occ = np.ascontiguousarray(occ, dtype=np.int32)
    out = np.empty(occ.shape[0], dtype=np.int64)
    _load().orc_hash_rows(N, occ.shape[1], _ptr(occ), occ.shape[0], _ptr(out))
    return out


def unhash(beta: int, N: int, M: int) -> np.ndarray:
    out = np.empty(M, dtype=np.int32)
    if _load().orc_unhash(N, M, beta, _ptr(out)) != 0:
        raise ValueError("index out of range")
    return out


def occ_rows(N: int, M: int, rows=None) -> np.ndarray:
    rows = _rows(rows, dim(N, M))
    out = np.empty((rows.size, M), dtype=np.int32)
    _load().orc_occ_rows(N, M, _ptr(rows), rows.size, _ptr(out))
    return out


def t1_rows(N: int, M: int, rows=None) -> np.ndarray:
    """Single-jump map rows, shape (len(rows), M, M), int32, -1 = empty k."""
    rows = _rows(rows, dim(N, M))
    out = np.empty((rows.size, M, M), dtype=np.int32)
    _load().orc_t1_rows(N, M, _ptr(rows), rows.size, _ptr(out))
    return out


def t2_row_lengths(N: int, M: int, rows=None) -> np.ndarray:
    rows = _rows(rows, dim(N, M))
    out = np.empty(rows.size, dtype=np.int64)
    _load().orc_t2_row_lengths(N, M, _ptr(rows), rows.size, _ptr(out))
    return out


def t2_rows(N: int, M: int, rows=None):
    """Double-jump map rows in the paper's variable-length layout.

    Returns (offsets[len(rows)+1] int64, entries int32)."""
    rows = _rows(rows, dim(N, M))
    lens = t2_row_lengths(N, M, rows)
    off = np.zeros(rows.size + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    ent = np.empty(int(off[-1]), dtype=np.int32)
    _load().orc_t2_rows(N, M, _ptr(rows), rows.size, _ptr(off), _ptr(ent))
    return off, ent


def t2r_row_lengths(N: int, M: int, rows=None) -> np.ndarray:
    rows = _rows(rows, dim(N, M))
    out = np.empty(rows.size, dtype=np.int64)
    _load().orc_t2r_row_lengths(N, M, _ptr(rows), rows.size, _ptr(out))
    return out


def t2r_rows(N: int, M: int, rows=None):
    """Reduced double-jump map rows (true double jumps only: creation pairs
    q <= l outside the removal pair).  Returns (offsets int64, entries int32)."""
    rows = _rows(rows, dim(N, M))
    lens = t2r_row_lengths(N, M, rows)
    off = np.zeros(rows.size + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    ent = np.empty(int(off[-1]), dtype=np.int32)
    _load().orc_t2r_rows(N, M, _ptr(rows), rows.size, _ptr(off), _ptr(ent))
    return off, ent


def apply_h(N: int, M: int, h, g, C, rows=None) -> np.ndarray:
    """(H C) for the given rows (all rows if None), by operator algebra."""
    D = dim(N, M)
    C = _c128(C)
    if C.size != D:
        raise ValueError("coefficient vector has the wrong length")
    h = _c128(h).reshape(M, M)
    g = _c128(g).reshape(M, M, M, M)
    rows = _rows(rows, D)
    out = np.empty(rows.size, dtype=np.complex128)
    _load().orc_apply_h_rows(N, M, _ptr(h), _ptr(g), _ptr(C), _ptr(rows), rows.size, _ptr(out))
    return out


def rho1(N: int, M: int, C) -> np.ndarray:
    C = _c128(C)
    if C.size != dim(N, M):
        raise ValueError("coefficient vector has the wrong length")
    out = np.empty((M, M), dtype=np.complex128)
    _load().orc_rho1(N, M, _ptr(C), _ptr(out))
    return out


def rho2(N: int, M: int, C) -> np.ndarray:
    C = _c128(C)
    if C.size != dim(N, M):
        raise ValueError("coefficient vector has the wrong length")
    out = np.empty((M, M, M, M), dtype=np.complex128)
    _load().orc_rho2(N, M, _ptr(C), _ptr(out))
    return out


def rho2_elements(N: int, M: int, C, flat_idx) -> np.ndarray:
    C = _c128(C)
    if C.size != dim(N, M):
        raise ValueError("coefficient vector has the wrong length")
    idx = np.ascontiguousarray(flat_idx, dtype=np.int64)
    out = np.empty(idx.size, dtype=np.complex128)
    _load().orc_rho2_elements(N, M, _ptr(C), _ptr(idx), idx.size, _ptr(out))
    return out
