"""Builds and loads the oracle's plain-C direct sums (test infrastructure)."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrc", "oracle_direct.c")
_LIB = os.path.join(_HERE, "csrc", "liboracle_direct.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle's C sums with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
                               "-ffp-contract=off", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        d = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.POINTER(ctypes.c_int64)
        L.oracle_near_traction.argtypes = [ctypes.c_int64, d, d, d, d, ctypes.c_int64, d, d, d, d,
                                           ctypes.c_int32, d, d, i64, d, d]
        L.oracle_near_traction.restype = None
        L.oracle_stokeslet_velocity.argtypes = [ctypes.c_int64, d, d, ctypes.c_int64, d, d, d, d,
                                                ctypes.c_int32, d, d, ctypes.c_double, d, d, d]
        L.oracle_stokeslet_velocity.restype = None
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def near_traction(x, n, y, f, shifts, self_idx=None):
    """T[i] = sum_j sum_s G^t(x_i - s, y_j; n_i) f_j (self pair skipped at s = 0)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    n = np.ascontiguousarray(n, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    f = np.ascontiguousarray(f, dtype=np.float64)
    shifts = np.ascontiguousarray(shifts, dtype=np.float64)
    x1, x2 = np.ascontiguousarray(x[:, 0]), np.ascontiguousarray(x[:, 1])
    n1, n2 = np.ascontiguousarray(n[:, 0]), np.ascontiguousarray(n[:, 1])
    y1, y2 = np.ascontiguousarray(y[:, 0]), np.ascontiguousarray(y[:, 1])
    f1, f2 = np.ascontiguousarray(f[:, 0]), np.ascontiguousarray(f[:, 1])
    s1, s2 = np.ascontiguousarray(shifts[:, 0]), np.ascontiguousarray(shifts[:, 1])
    t1 = np.zeros(len(x1))
    t2 = np.zeros(len(x1))
    si = None
    if self_idx is not None:
        si = np.ascontiguousarray(self_idx, dtype=np.int64)
    lib().oracle_near_traction(len(x1), _p(x1), _p(x2), _p(n1), _p(n2), len(y1), _p(y1), _p(y2),
                               _p(f1), _p(f2), len(s1), _p(s1), _p(s2),
                               None if si is None else si.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                               _p(t1), _p(t2))
    return np.stack([t1, t2], axis=1)


def stokeslet_velocity(x, y, f, shifts, mu):
    """u(x_i) = sum_j sum_s G(x_i - s, y_j) f_j and the vorticity of that field."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    f = np.ascontiguousarray(f, dtype=np.float64)
    shifts = np.ascontiguousarray(shifts, dtype=np.float64)
    x1, x2 = np.ascontiguousarray(x[:, 0]), np.ascontiguousarray(x[:, 1])
    y1, y2 = np.ascontiguousarray(y[:, 0]), np.ascontiguousarray(y[:, 1])
    f1, f2 = np.ascontiguousarray(f[:, 0]), np.ascontiguousarray(f[:, 1])
    s1, s2 = np.ascontiguousarray(shifts[:, 0]), np.ascontiguousarray(shifts[:, 1])
    u1 = np.zeros(len(x1))
    u2 = np.zeros(len(x1))
    w = np.zeros(len(x1))
    lib().oracle_stokeslet_velocity(len(x1), _p(x1), _p(x2), len(y1), _p(y1), _p(y2), _p(f1), _p(f2),
                                    len(s1), _p(s1), _p(s2), float(mu), _p(u1), _p(u2), _p(w))
    return np.stack([u1, u2], axis=1), w
