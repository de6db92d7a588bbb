"""Build and load the oracle's C Slater-Condon kernels (test infrastructure).

``build()`` compiles ``sc.c`` with gcc (OpenMP) into ``_sc.so`` next to it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sc.c")
_LIB = os.path.join(_HERE, "_sc.so")
_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        d, i64, u64p, dp = ctypes.c_double, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p
        L.sc_element.restype = d
        L.sc_element.argtypes = [ctypes.c_int, dp, dp, ctypes.c_uint64, ctypes.c_uint64,
                                 ctypes.c_uint64, ctypes.c_uint64]
        L.sc_hmat.restype = None
        L.sc_hmat.argtypes = [ctypes.c_int, dp, dp, d, i64, u64p, i64, u64p, dp]
        L.sc_matvec.restype = None
        L.sc_matvec.argtypes = [ctypes.c_int, dp, dp, d, i64, u64p, i64, u64p,
                                ctypes.c_uint64, dp, dp]
        L.sc_rdm12.restype = None
        L.sc_rdm12.argtypes = [ctypes.c_int, i64, u64p, i64, u64p, dp, dp, dp]
        _lib = L
    return _lib


def ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)
