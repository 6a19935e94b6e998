"""ctypes front-end of the plain-C FP64 oracle (ndf_oracle.c).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Columns follow Sec. 3: the local sample e(p) of a vertex p is the vector of its N
member values.  Blocks of query columns are member-major ``[N][nq]`` float32.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "ndf_oracle.c"
_LIB = _HERE / "liboracle.so"

_f32p = ctypes.POINTER(ctypes.c_float)
_f64p = ctypes.POINTER(ctypes.c_double)
_i32p = ctypes.POINTER(ctypes.c_int32)


def build(force: bool = True) -> Path:
    """Compile the oracle with gcc (OpenMP, no FP contraction, no fast-math)."""
    if force or not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
        tmp = _LIB.with_suffix(".so.tmp")
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off",
                               "-fno-fast-math", "-shared", "-fPIC", str(_SRC), "-o",
                               str(tmp), "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(str(_LIB))
        L.ndf_oracle_pearson.restype = ctypes.c_double
        L.ndf_oracle_pearson.argtypes = [_f32p, ctypes.c_int64, _f32p, ctypes.c_int64,
                                         ctypes.c_int64]
        L.ndf_oracle_pearson_field.restype = None
        L.ndf_oracle_pearson_field.argtypes = [_f32p, ctypes.c_int64, _f32p, ctypes.c_int64,
                                               ctypes.c_int64, _f64p]
        L.ndf_oracle_moments.restype = None
        L.ndf_oracle_moments.argtypes = [_f32p, ctypes.c_int64, ctypes.c_int64, _f64p, _f64p]
        L.ndf_oracle_ksg_codes.restype = ctypes.c_int
        L.ndf_oracle_ksg_codes.argtypes = [_f32p, ctypes.c_int64, ctypes.c_int64, _i32p]
        L.ndf_oracle_ksg.restype = ctypes.c_double
        L.ndf_oracle_ksg.argtypes = [_i32p, _i32p, ctypes.c_int64, ctypes.c_int, _i32p, _i32p]
        L.ndf_oracle_ksg_field.restype = None
        L.ndf_oracle_ksg_field.argtypes = [_f32p, ctypes.c_int64, _f32p, ctypes.c_int64,
                                           ctypes.c_int64, ctypes.c_int, _f64p, _i32p, _i32p]
        L.ndf_oracle_pearson_pairs.restype = None
        L.ndf_oracle_pearson_pairs.argtypes = [_f32p, _f32p, ctypes.c_int64, ctypes.c_int64,
                                               _f64p]
        L.ndf_oracle_ksg_pairs.restype = None
        L.ndf_oracle_ksg_pairs.argtypes = [_f32p, _f32p, ctypes.c_int64, ctypes.c_int64,
                                           ctypes.c_int, _f64p]
        L.ndf_oracle_set_threads.restype = None
        L.ndf_oracle_set_threads.argtypes = [ctypes.c_int]
        L.ndf_oracle_max_threads.restype = ctypes.c_int
        L.ndf_oracle_max_threads.argtypes = []
        _lib = L
    return _lib


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _ptr(a, t):
    return a.ctypes.data_as(t)


def pearson(a, b) -> float:
    """Eq. (1) for two sample vectors."""
    a = _f32(a)
    b = _f32(b)
    assert a.shape == b.shape and a.ndim == 1
    return lib().ndf_oracle_pearson(_ptr(a, _f32p), 1, _ptr(b, _f32p), 1, a.shape[0])


def pearson_field(ref_col, q) -> np.ndarray:
    """r(ref, q[:, v]) for every column of the member-major block q[N][nq]."""
    ref_col = _f32(ref_col)
    q = _f32(q)
    n, nq = q.shape
    assert ref_col.shape == (n,)
    out = np.empty(nq, dtype=np.float64)
    lib().ndf_oracle_pearson_field(_ptr(ref_col, _f32p), 1, _ptr(q, _f32p), nq, n,
                                   _ptr(out, _f64p))
    return out


def moments(col):
    col = _f32(col)
    m = ctypes.c_double()
    s = ctypes.c_double()
    lib().ndf_oracle_moments(_ptr(col, _f32p), 1, col.shape[0], ctypes.byref(m),
                             ctypes.byref(s))
    return m.value, s.value


def ksg_codes(col):
    """Min-max integer codes in [0, 2^23]; returns (codes int32, flat)."""
    col = _f32(col)
    code = np.empty(col.shape[0], dtype=np.int32)
    flat = lib().ndf_oracle_ksg_codes(_ptr(col, _f32p), 1, col.shape[0], _ptr(code, _i32p))
    return code, bool(flat)


def ksg(xc, yc, k):
    """KSG estimate (nats) and neighbour counts for integer samples xc, yc."""
    xc = np.ascontiguousarray(xc, dtype=np.int32)
    yc = np.ascontiguousarray(yc, dtype=np.int32)
    n = xc.shape[0]
    nx = np.empty(n, dtype=np.int32)
    ny = np.empty(n, dtype=np.int32)
    mi = lib().ndf_oracle_ksg(_ptr(xc, _i32p), _ptr(yc, _i32p), n, int(k), _ptr(nx, _i32p),
                              _ptr(ny, _i32p))
    return mi, nx, ny


def ksg_field(ref_col, q, k, counts=False):
    """KSG MI(ref, q[:, v]) for every column of q[N][nq]; optional counts [nq][N]."""
    ref_col = _f32(ref_col)
    q = _f32(q)
    n, nq = q.shape
    out = np.empty(nq, dtype=np.float64)
    if counts:
        nx = np.empty((nq, n), dtype=np.int32)
        ny = np.empty((nq, n), dtype=np.int32)
        px, py = _ptr(nx, _i32p), _ptr(ny, _i32p)
    else:
        nx = ny = None
        px = py = None
    lib().ndf_oracle_ksg_field(_ptr(ref_col, _f32p), 1, _ptr(q, _f32p), nq, n, int(k),
                               _ptr(out, _f64p), px, py)
    if counts:
        return out, nx, ny
    return out


def pearson_pairs(a, b) -> np.ndarray:
    """r(a[:, p], b[:, p]) for the columns p of two member-major blocks [N][np]."""
    a = _f32(a)
    b = _f32(b)
    assert a.shape == b.shape and a.ndim == 2
    n, npairs = a.shape
    out = np.empty(npairs, dtype=np.float64)
    lib().ndf_oracle_pearson_pairs(_ptr(a, _f32p), _ptr(b, _f32p), npairs, n, _ptr(out, _f64p))
    return out


def ksg_pairs(a, b, k) -> np.ndarray:
    """KSG MI(a[:, p], b[:, p]) (nats) for the columns p of two blocks [N][np]."""
    a = _f32(a)
    b = _f32(b)
    assert a.shape == b.shape and a.ndim == 2
    n, npairs = a.shape
    out = np.empty(npairs, dtype=np.float64)
    lib().ndf_oracle_ksg_pairs(_ptr(a, _f32p), _ptr(b, _f32p), npairs, n, int(k),
                               _ptr(out, _f64p))
    return out


def set_threads(n: int) -> None:
    lib().ndf_oracle_set_threads(int(n))


def max_threads() -> int:
    return int(lib().ndf_oracle_max_threads())
