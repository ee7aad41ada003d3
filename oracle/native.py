"""ctypes front end of oracle/core.c (test infrastructure only).

The shared object is built with gcc, -O2, -ffp-contract=off and OpenMP; no
-ffast-math, so the compensated sums stay compensated.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "core.c")
_LIB = os.path.join(_HERE, "_oracle_core.so")
_FSRC = os.path.join(_HERE, "factored.c")
_FLIB = os.path.join(_HERE, "_oracle_factored.so")
_lib = None
_flib = None


def _gcc(src, lib, force, opt):
    if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(src):
        tmp = lib + ".tmp%d" % os.getpid()
        cmd = ["gcc", opt, "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", src, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, lib)
    return lib


def build_native(force: bool = False) -> str:
    """Compile core.c into oracle/_oracle_core.so and factored.c into
    oracle/_oracle_factored.so (gcc, no GPU involved)."""
    _gcc(_FSRC, _FLIB, force, "-O3")
    return _gcc(_SRC, _LIB, force, "-O2")


def _get():
    global _lib
    if _lib is None:
        build_native()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_rhs_direct.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                          ctypes.POINTER(dp), dp, dp, dp]
        lib.oracle_rhs_conv.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                        ctypes.POINTER(dp), dp, ctypes.c_int, dp, dp]
        _lib = lib
    return _lib


def _marshal(D, N, kernel):
    R = (ctypes.c_int * (D + 1))()
    F = (ctypes.POINTER(ctypes.c_double) * (D + 1))()
    keep = []
    for d in range(2, D + 1):
        U = kernel.get(d)
        if U is None or U.shape[1] == 0:
            R[d] = 0
            continue
        U = np.ascontiguousarray(U, dtype=np.float64)
        assert U.shape == (d, U.shape[1], N), (U.shape, d, N)
        keep.append(U)
        R[d] = U.shape[1]
        F[d] = U.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return R, F, keep


def rhs_direct(D: int, N: int, kernel: dict, n: np.ndarray):
    """Literal sums; returns (p, q) as (D+1, N) arrays (rows 0, 1 are zero)."""
    lib = _get()
    n = np.ascontiguousarray(n, dtype=np.float64)
    R, F, keep = _marshal(D, N, kernel)
    p = np.zeros((D + 1, N))
    q = np.zeros((D + 1, N))
    dp = ctypes.POINTER(ctypes.c_double)
    rc = lib.oracle_rhs_direct(D, N, R, F, n.ctypes.data_as(dp), p.ctypes.data_as(dp),
                               q.ctypes.data_as(dp))
    if rc != 0:
        raise ValueError("oracle_rhs_direct rejected its arguments")
    del keep
    return p, q


def rhs_conv(D: int, N: int, kernel: dict, n: np.ndarray, kmax: int = 0):
    """Per-rank direct convolutions; gain outputs beyond kmax are NaN."""
    lib = _get()
    n = np.ascontiguousarray(n, dtype=np.float64)
    R, F, keep = _marshal(D, N, kernel)
    p = np.zeros((D + 1, N))
    q = np.zeros((D + 1, N))
    dp = ctypes.POINTER(ctypes.c_double)
    rc = lib.oracle_rhs_conv(D, N, R, F, n.ctypes.data_as(dp), int(kmax), p.ctypes.data_as(dp),
                             q.ctypes.data_as(dp))
    if rc != 0:
        raise ValueError("oracle_rhs_conv rejected its arguments")
    del keep
    return p, q


def _get_factored():
    global _flib
    if _flib is None:
        build_native()
        lib = ctypes.CDLL(_FLIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.factored_rhs.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                     ctypes.POINTER(dp), dp, dp, ctypes.POINTER(ctypes.c_int)]
        _flib = lib
    return _flib


def rhs_factored(D: int, N: int, kernel: dict, n: np.ndarray):
    """The factored CPU evaluation (factored.c, OpenMP): returns (f, threads)
    with f[k-1] = sum_d (p_k^(d) + q_k^(d))."""
    lib = _get_factored()
    n = np.ascontiguousarray(n, dtype=np.float64)
    R, F, keep = _marshal(D, N, kernel)
    f = np.zeros(N)
    th = ctypes.c_int(0)
    dp = ctypes.POINTER(ctypes.c_double)
    rc = lib.factored_rhs(D, N, R, F, n.ctypes.data_as(dp), f.ctypes.data_as(dp), ctypes.byref(th))
    if rc != 0:
        raise ValueError(f"factored_rhs failed ({rc})")
    del keep
    return f, th.value
