"""Python driver of the FP64 direct stencil stepper in direct.c.

Test infrastructure only.  ``build()`` compiles direct.c with gcc
(-O3 -ffp-contract=off -fopenmp) into oracle/_build/liboracle_direct.so;
``run`` steps a float64 copy of the grid; ``run_binary16`` is the same
definition with the state and coefficients held in binary16.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "direct.c")
_OUT_DIR = os.path.join(_HERE, "_build")
_LIB = os.path.join(_OUT_DIR, "liboracle_direct.so")
_lib = None


def build(force: bool = True) -> str:
    os.makedirs(_OUT_DIR, exist_ok=True)
    if force or not os.path.exists(_LIB):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O3", "-ffp-contract=off", "-fopenmp", "-fPIC",
                               "-shared", "-std=c99", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        lib.oracle_direct_run.restype = ctypes.c_int
        lib.oracle_direct_run.argtypes = [
            ctypes.c_int, ctypes.POINTER(ctypes.c_int64), ctypes.c_int,
            ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_int64,
            ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), ctypes.c_int]
        lib.oracle_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def threads() -> int:
    return int(_load().oracle_threads())


def run(x, w, steps: int, periodic: bool = False, nthreads: int = 0) -> np.ndarray:
    """Return the grid after ``steps`` sweeps of the stencil w (float64).

    x: 1-, 2- or 3-D array (any float type, converted exactly to float64);
    w: (2r+1)^ndim coefficients in correlation orientation."""
    lib = _load()
    a = np.ascontiguousarray(x, dtype=np.float64).copy()
    wv = np.ascontiguousarray(w, dtype=np.float64)
    ndim = a.ndim
    k = wv.shape[0]
    if wv.shape != (k,) * ndim or k % 2 == 0:
        raise ValueError("coefficient array must be (2r+1)^ndim")
    dims = (ctypes.c_int64 * ndim)(*a.shape)
    scratch = np.empty_like(a)
    rc = lib.oracle_direct_run(
        ndim, dims, (k - 1) // 2, wv.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
        1 if periodic else 0, int(steps), a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
        scratch.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_direct_run rejected its arguments")
    return a


def run_binary16(x, w, steps: int, periodic: bool = False) -> np.ndarray:
    """The plain binary16 computation (the paper's FP16 setting, Section 4.1):
    coefficients and state rounded to binary16 (nearest even), each sweep's
    sum of products formed exactly in FP64 by ``run`` and rounded to binary16.
    Returns the binary16 grid after ``steps`` sweeps as float64."""
    w16 = np.asarray(w, dtype=np.float64).astype(np.float16).astype(np.float64)
    a = np.asarray(x, dtype=np.float64).astype(np.float16)
    for _ in range(int(steps)):
        a = run(a.astype(np.float64), w16, 1, periodic=periodic).astype(np.float16)
    return a.astype(np.float64)
