"""CPU FP64 oracle for the SBR symmetric eigensolver -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library in
``paper_1604_03703_amd``) never does, and the two share no code.

* ``liboracle.so`` (built from ``oracle.c`` with gcc + OpenMP): Householder
  tridiagonalisation + Sturm bisection, i.e. the eigenvalues of a dense
  symmetric matrix by a route independent of successive band reduction.
* ``sbr_model``: a NumPy transcription of the paper's algorithms
  (rect-QR, Householder reconstruction, full-to-band, band-to-band) used to
  settle the readings of the paper and to give per-stage expectations.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build()
            lib = ctypes.CDLL(_LIB)
            i64, dp = ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
            lib.oracle_tridiagonalize.argtypes = [i64, dp, i64, dp, dp]
            lib.oracle_tridiagonalize.restype = ctypes.c_int
            lib.oracle_sturm_count.argtypes = [i64, dp, dp, ctypes.c_double, ctypes.c_double]
            lib.oracle_sturm_count.restype = i64
            lib.oracle_pivmin.argtypes = [i64, dp]
            lib.oracle_pivmin.restype = ctypes.c_double
            lib.oracle_bisect_setup.argtypes = [i64, dp, dp, dp, dp, dp, ctypes.POINTER(ctypes.c_int)]
            lib.oracle_bisect_setup.restype = ctypes.c_int
            lib.oracle_bisect_all.argtypes = [i64, dp, dp, dp]
            lib.oracle_bisect_all.restype = ctypes.c_int
            lib.oracle_eigvalsh.argtypes = [i64, dp, i64, dp, dp]
            lib.oracle_eigvalsh.restype = ctypes.c_int
            lib.oracle_num_threads.argtypes = []
            lib.oracle_num_threads.restype = ctypes.c_int
            _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def tridiagonalize(A):
    """(d, e) of the Householder tridiagonal form of the symmetric matrix A."""
    lib = _load()
    A = np.array(A, dtype=np.float64, order="F", copy=True)
    n = A.shape[0]
    d = np.zeros(n)
    e = np.zeros(max(n - 1, 1))
    rc = lib.oracle_tridiagonalize(n, _ptr(A), max(n, 1), _ptr(d), _ptr(e))
    if rc:
        raise RuntimeError("oracle_tridiagonalize failed: %d" % rc)
    return d, e[: max(n - 1, 0)]


def pivmin(e, n=None) -> float:
    e = _f64(e)
    n = len(e) + 1 if n is None else n
    if e.size == 0:
        e = np.zeros(1)
    return float(_load().oracle_pivmin(n, _ptr(e)))


def sturm_count(d, e, x: float, piv: float | None = None) -> int:
    d = _f64(d)
    n = d.shape[0]
    e = _f64(e) if n > 1 else np.zeros(1)
    if piv is None:
        piv = pivmin(e, n)
    return int(_load().oracle_sturm_count(n, _ptr(d), _ptr(e), float(x), float(piv)))


def bisect_setup(d, e):
    d = _f64(d)
    n = d.shape[0]
    e = _f64(e) if n > 1 else np.zeros(1)
    lo, hi, pv = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    it = ctypes.c_int()
    _load().oracle_bisect_setup(n, _ptr(d), _ptr(e), ctypes.byref(lo), ctypes.byref(hi),
                                ctypes.byref(pv), ctypes.byref(it))
    return lo.value, hi.value, pv.value, it.value


def tridiag_eigvals(d, e) -> np.ndarray:
    """All eigenvalues of tridiag(e, d, e), ascending, by Sturm bisection."""
    d = _f64(d)
    n = d.shape[0]
    e = _f64(e) if n > 1 else np.zeros(1)
    w = np.zeros(n)
    rc = _load().oracle_bisect_all(n, _ptr(d), _ptr(e), _ptr(w))
    if rc:
        raise RuntimeError("oracle_bisect_all failed: %d" % rc)
    return w


def eigvalsh(A, return_seconds: bool = False):
    """Ascending eigenvalues of the dense symmetric A (lower triangle read)."""
    A = np.array(A, dtype=np.float64, order="F")
    n = A.shape[0]
    w = np.zeros(n)
    sec = np.zeros(2)
    rc = _load().oracle_eigvalsh(n, _ptr(A), max(n, 1), _ptr(w), _ptr(sec))
    if rc:
        raise RuntimeError("oracle_eigvalsh failed: %d" % rc)
    return (w, (float(sec[0]), float(sec[1]))) if return_seconds else w


def band_eigvalsh(band: np.ndarray, n: int) -> np.ndarray:
    """Eigenvalues of a symmetric band matrix given in lower band storage
    band[d, j] = B[j + d, j] (d = 0 .. rows-1)."""
    A = np.zeros((n, n))
    for dd in range(band.shape[0]):
        idx = np.arange(n - dd)
        A[idx + dd, idx] = band[dd, : n - dd]
    return eigvalsh(A)


def qr_r(A) -> np.ndarray:
    """R factor of A = QR (LAPACK via numpy), rows normalised to a positive diagonal."""
    R = np.linalg.qr(np.asarray(A, dtype=np.float64), mode="r")
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return s[:, None] * R
