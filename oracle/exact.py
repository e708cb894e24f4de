"""Correctly rounded sums, dot products and sparse products in FP64.

Every sum the oracle forms is the FP64 number nearest the exact real sum of
its terms, so its value does not depend on the order of summation. A dot
product sums the exact products a_i * b_i: each product is split without
error into p + e and all the p and e terms are added exactly.

Two interchangeable implementations compute the same values: plain C
(exact_sum.c, compiled with gcc into _exact.so next to it) for speed, and
pure Python (``math.fsum``, Shewchuk's exactly rounded summation, over
products split with Dekker's method). The Python one is used when the C
library cannot be built; a CPU test checks that both agree bit for bit.
"""

from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "exact_sum.c")
_LIB = os.path.join(_HERE, "_exact.so")
_clib = None


def build_c(force: bool = False) -> bool:
    """Compile exact_sum.c with gcc; True on success."""
    if os.path.exists(_LIB) and not force and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return True
    tmp = f"{_LIB}.{os.getpid()}.tmp"
    try:
        subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
                        "-o", tmp, _SRC, "-lm"], check=True, capture_output=True)
        os.replace(tmp, _LIB)
        return True
    except (OSError, subprocess.CalledProcessError):
        return False


def _load():
    global _clib
    if _clib is not None:
        return _clib or None
    if not build_c():
        _clib = False
        return None
    lib = ctypes.CDLL(_LIB)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int64)
    lib.exact_sum.restype = ctypes.c_double
    lib.exact_sum.argtypes = [ctypes.c_int64, dp]
    lib.exact_dot.restype = ctypes.c_double
    lib.exact_dot.argtypes = [ctypes.c_int64, dp, dp]
    lib.exact_spmv.restype = None
    lib.exact_spmv.argtypes = [ctypes.c_int64, ip, ip, dp, dp, dp]
    lib.exact_row_sums.restype = None
    lib.exact_row_sums.argtypes = [ctypes.c_int64, ip, dp, dp]
    _clib = lib
    return lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))

_SPLIT = 134217729.0  # 2**27 + 1


def _split(a: np.ndarray):
    t = _SPLIT * a
    hi = t - (t - a)
    return hi, a - hi


def two_prod(a: np.ndarray, b: np.ndarray):
    """p, e with p = fl(a * b) and p + e == a * b exactly."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    p = a * b
    ah, al = _split(a)
    bh, bl = _split(b)
    e = ((ah * bh - p) + ah * bl + al * bh) + al * bl
    return p, e


def py_exact_sum(v) -> float:
    return math.fsum(np.asarray(v, dtype=np.float64).tolist())


def py_exact_dot(a, b) -> float:
    p, e = two_prod(a, b)
    return math.fsum(p.tolist() + e.tolist())


def exact_sum(v) -> float:
    """FP64 value nearest the exact sum of v."""
    lib = _load()
    if lib is None:
        return py_exact_sum(v)
    v = _f64(v)
    return float(lib.exact_sum(v.size, _dp(v)))


def exact_dot(a, b) -> float:
    """FP64 value nearest the exact sum of a_i * b_i."""
    lib = _load()
    if lib is None:
        return py_exact_dot(a, b)
    a = _f64(a)
    b = _f64(b)
    assert a.shape == b.shape
    return float(lib.exact_dot(a.size, _dp(a), _dp(b)))


def exact_norm(a) -> float:
    return math.sqrt(exact_dot(a, a))


def exact_spmv(row_ptr, col_idx, val, x) -> np.ndarray:
    """CSR product with every row sum correctly rounded."""
    lib = _load()
    if lib is not None:
        rp = _i64(row_ptr)
        ci = _i64(col_idx)
        va = _f64(val)
        xv = _f64(x)
        out = np.zeros(rp.size - 1)
        lib.exact_spmv(rp.size - 1, _ip(rp), _ip(ci), _dp(va), _dp(xv), _dp(out))
        return out
    return py_exact_spmv(row_ptr, col_idx, val, x)


def py_exact_spmv(row_ptr, col_idx, val, x) -> np.ndarray:
    row_ptr = np.asarray(row_ptr)
    m = row_ptr.size - 1
    out = np.zeros(m)
    if m == 0 or row_ptr[-1] == 0:
        return out
    p, e = two_prod(val, np.asarray(x, dtype=np.float64)[col_idx])
    pl = p.tolist()
    el = e.tolist()
    rp = row_ptr.tolist()
    fsum = math.fsum
    for i in range(m):
        s, t = rp[i], rp[i + 1]
        if t > s:
            out[i] = fsum(pl[s:t] + el[s:t])
    return out


def exact_row_sums(row_ptr, v) -> np.ndarray:
    """Correctly rounded sum of each CSR row's entries of v."""
    lib = _load()
    if lib is not None:
        rp = _i64(row_ptr)
        vv = _f64(v)
        out = np.zeros(rp.size - 1)
        lib.exact_row_sums(rp.size - 1, _ip(rp), _dp(vv), _dp(out))
        return out
    return py_exact_row_sums(row_ptr, v)


def py_exact_row_sums(row_ptr, v) -> np.ndarray:
    row_ptr = np.asarray(row_ptr)
    m = row_ptr.size - 1
    out = np.zeros(m)
    vl = np.asarray(v, dtype=np.float64).tolist()
    rp = row_ptr.tolist()
    for i in range(m):
        s, t = rp[i], rp[i + 1]
        if t > s:
            out[i] = math.fsum(vl[s:t])
    return out
