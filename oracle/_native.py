"""Loader for the oracle's C eigensolver (test infrastructure only).

Compiles ``eigsolve.c`` with the host C compiler into ``liboracle_eig.so`` next
to this file and exposes thin numpy wrappers.  Nothing in the product library
links or calls this code.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "eigsolve.c")
_LIB = os.path.join(_HERE, "liboracle_eig.so")
_lib = None


def build():
    """Compile the oracle's C code (always recompiles)."""
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.orc_syev.argtypes = [ctypes.c_int, dp, dp, dp]
    lib.orc_jacobi.argtypes = [ctypes.c_int, dp, dp, dp, ctypes.c_int]
    lib.orc_tridiag_eigvals.argtypes = [ctypes.c_int, dp, dp, dp]
    lib.orc_tridiagonalize.argtypes = [ctypes.c_int, dp, dp, dp, dp]
    for f in (lib.orc_syev, lib.orc_jacobi, lib.orc_tridiag_eigvals, lib.orc_tridiagonalize):
        f.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def syev(a, vectors=False):
    """Eigen-decomposition of a dense symmetric matrix by Householder + implicit QL.

    Returns ascending eigenvalues (and the row-major eigenvector matrix whose
    column j belongs to eigenvalue j when ``vectors``)."""
    a = np.array(a, dtype=np.float64, order="C", copy=True)
    n = a.shape[0]
    assert a.shape == (n, n)
    w = np.empty(n)
    z = np.empty((n, n)) if vectors else None
    rc = _load().orc_syev(n, _ptr(a), _ptr(w), _ptr(z))
    if rc != 0:
        raise RuntimeError("oracle syev failed to converge")
    return (w, z) if vectors else w


def jacobi(a, vectors=False, max_sweeps=100):
    """Eigen-decomposition by cyclic Jacobi (independent algorithm)."""
    a = np.array(a, dtype=np.float64, order="C", copy=True)
    n = a.shape[0]
    w = np.empty(n)
    v = np.empty((n, n)) if vectors else None
    _load().orc_jacobi(n, _ptr(a), _ptr(w), _ptr(v), max_sweeps)
    return (w, v) if vectors else w


def tridiag_eigvals(d, e):
    """Eigenvalues (ascending) of the symmetric tridiagonal with diagonal d and
    off-diagonal e (len(e) == len(d) - 1) by implicit QL."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    n = d.shape[0]
    ee = np.zeros(n)
    ee[: n - 1] = e
    w = np.empty(n)
    rc = _load().orc_tridiag_eigvals(n, _ptr(d), _ptr(ee), _ptr(w))
    if rc != 0:
        raise RuntimeError("oracle tridiagonal QL failed to converge")
    return w
