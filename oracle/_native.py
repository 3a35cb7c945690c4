"""Oracle (test infrastructure only): builds and loads the plain-C quadrature
in ``fd_quad.c`` with gcc.  Only tests, the smoke check and the CPU baseline
load it; the product library never does.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fd_quad.c")
_LIB = os.path.join(_HERE, "_fd_quad.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile fd_quad.c -> _fd_quad.so (gcc, OpenMP).  Returns the path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
               "-ffp-contract=off", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            path = build()
            L = ctypes.CDLL(path)
            dp = ctypes.POINTER(ctypes.c_double)
            L.oracle_fd_eval.argtypes = [ctypes.c_ssize_t, dp, ctypes.c_int, dp, dp, dp, dp, dp]
            L.oracle_fd_eval.restype = None
            _lib = L
    return _lib


def as_ptr(a: np.ndarray | None):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
