"""Multi-core CPU comparison point for the resample + redistribute path
(OpenMP, ``omp_resample.c``).  The benchmark times it beside the GPU path;
the library and the parity tests do not use it."""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_DIR = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_DIR, "omp_resample.c")
_LIB = os.path.join(_DIR, "libsmc_omp.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile with gcc and OpenMP (no contraction, no fast-math; the
    deterministic exponential's fused multiply-adds are written out)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call([
            "gcc", "-O3", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
            "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            raise RuntimeError("baseline/libsmc_omp.so is not built (run __graft_entry__.build())")
        lib = C.CDLL(_LIB)
        lib.omp_threads.restype = C.c_int
        lib.omp_resample_redistribute.restype = C.c_int
        lib.omp_resample_redistribute.argtypes = [
            C.c_void_p, C.c_int64, C.c_uint64, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
            C.c_void_p, C.c_void_p, C.c_void_p]
        lib.omp_logreg_loglik.restype = C.c_int
        lib.omp_logreg_loglik.argtypes = [C.c_void_p, C.c_int64, C.c_int, C.c_void_p, C.c_void_p,
                                          C.c_int64, C.c_void_p]
        _lib = lib
    return _lib


def threads() -> int:
    return load().omp_threads()


class Workspace:
    """Output and scratch arrays for repeated calls at one (n, row_bytes)."""

    def __init__(self, n: int, row_shape, dtype):
        self.n = n
        self.x_out = np.empty((n,) + tuple(row_shape), dtype=dtype)
        self.ncopies = np.empty(n, dtype=np.int64)
        self.q = np.empty(n, dtype=np.uint64)
        self.res = np.zeros(5, dtype=np.uint64)
        self.zres = np.zeros(3, dtype=np.float64)


def resample_redistribute(lw: np.ndarray, r: int, x: np.ndarray, ws: Workspace | None = None):
    """Forced systematic resampling of log-weights lw and the redistribute of
    the rows of x.  Returns (ncopies, x_out, info)."""
    lw = np.ascontiguousarray(lw, dtype=np.float64)
    x = np.ascontiguousarray(x)
    n = lw.shape[0]
    if x.shape[0] != n:
        raise ValueError("x must have one row per log-weight")
    if ws is None:
        ws = Workspace(n, x.shape[1:], x.dtype)
    row_bytes = x.strides[0] if x.ndim > 1 else x.itemsize
    st = load().omp_resample_redistribute(
        lw.ctypes.data, n, r & (2**64 - 1), x.ctypes.data, row_bytes, ws.x_out.ctypes.data,
        ws.ncopies.ctypes.data, ws.q.ctypes.data, ws.res.ctypes.data, ws.zres.ctypes.data)
    if st != 0:
        raise ValueError("omp_resample_redistribute failed with status %d" % st)
    info = {"S": int(ws.res[0]), "U": int(ws.res[1]), "Q2_hi": int(ws.res[2]),
            "Q2_lo": int(ws.res[3]), "K": int(ws.res[4]), "Z": float(ws.zres[0]),
            "Z2": float(ws.zres[1]), "m": float(ws.zres[2])}
    return ws.ncopies, ws.x_out, info


def logreg_loglik(theta: np.ndarray, X: np.ndarray, y: np.ndarray) -> np.ndarray:
    """sum_r y_r z - softplus(z), z = X_r . theta_i, for every row theta_i."""
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    X = np.ascontiguousarray(X, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    n, d = theta.shape
    if X.shape[1] != d or y.shape[0] != X.shape[0]:
        raise ValueError("shapes of theta, X and y do not match")
    out = np.empty(n, dtype=np.float64)
    if load().omp_logreg_loglik(theta.ctypes.data, n, d, X.ctypes.data, y.ctypes.data,
                                X.shape[0], out.ctypes.data) != 0:
        raise MemoryError("omp_logreg_loglik: no memory for the transposed X")
    return out
