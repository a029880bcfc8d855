"""FP64 CPU oracle for the orthonormal 2D DCT (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
import this package.  The product library never does, and this package never
imports the product library: the two share nothing but the seeded input
generators (``workloads``), which hold no transform arithmetic.

The arithmetic lives in ``dct_oracle.c`` (plain C, double precision, the
direct definition of the paper's Section 2.1 eq. 1-2 evaluated as two matrix
products; the spectral filter of Prop. 1 / eq. 4 as forward, multiply, inverse).  This module builds it with gcc on first use, wraps it with ctypes
and adds the acceptance metric of Section 6 eq. 5.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dct_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_dct.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile dct_oracle.c into liboracle_dct.so (gcc, -O2, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-pthread", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class Oracle:
    """ctypes handle on one build of dct_oracle.c (the default one, or a test variant)."""

    def __init__(self, path: str):
        lib = ctypes.CDLL(path)
        i64, i32 = ctypes.c_int64, ctypes.c_int32
        vp = ctypes.c_void_p
        for name in ("oracle_forward", "oracle_inverse", "oracle_roundtrip",
                     "oracle_forward_d", "oracle_inverse_d"):
            fn = getattr(lib, name)
            fn.argtypes = [vp, vp, i64, i32, i32, i64, i32]
            fn.restype = ctypes.c_int
        lib.oracle_filter.argtypes = [vp, vp, i64, i32, i32, i64, vp, i64, i32]
        lib.oracle_filter.restype = ctypes.c_int
        lib.oracle_qmatrix.argtypes = [i32, vp]
        lib.oracle_qmatrix.restype = ctypes.c_int
        self.lib = lib
        self.path = path

    def qmatrix(self, n: int) -> np.ndarray:
        """Q_n of eq. 1 in double precision."""
        q = np.empty((n, n), dtype=np.float64)
        rc = self.lib.oracle_qmatrix(int(n), q.ctypes.data)
        if rc != 0:
            raise ValueError("oracle_qmatrix(%d) failed: %d" % (n, rc))
        return q

    def _run(self, name: str, x: np.ndarray, threads: int | None) -> np.ndarray:
        squeeze = x.ndim == 2
        xb = x[None] if squeeze else x
        if xb.ndim != 3:
            raise ValueError("expected (batch, rows, cols) or (rows, cols)")
        xb = np.ascontiguousarray(xb)
        b, h, w = xb.shape
        if xb.dtype == np.float32:
            fn = getattr(self.lib, name)
        elif xb.dtype == np.float64:
            if name == "oracle_roundtrip":
                raise TypeError("roundtrip takes float32 input")
            fn = getattr(self.lib, name + "_d")
        else:
            raise TypeError("oracle input must be float32 or float64, got %s" % xb.dtype)
        y = np.empty((b, h, w), dtype=np.float64)
        rc = fn(xb.ctypes.data, y.ctypes.data, b, h, w, h * w, threads or default_threads())
        if rc != 0:
            raise RuntimeError("%s failed with %d" % (name, rc))
        return y[0] if squeeze else y

    def forward(self, x: np.ndarray, threads: int | None = None) -> np.ndarray:
        """Y = Q_h X Q_w^T (eq. 2) for every array in x; double output."""
        return self._run("oracle_forward", x, threads)

    def inverse(self, y: np.ndarray, threads: int | None = None) -> np.ndarray:
        """X = Q_h^T Y Q_w (eq. 2) for every array in y; double output."""
        return self._run("oracle_inverse", y, threads)

    def roundtrip(self, x: np.ndarray, threads: int | None = None) -> np.ndarray:
        """inverse(forward(X)) computed in double (exact result: X itself)."""
        return self._run("oracle_roundtrip", x, threads)

    def filter(self, x: np.ndarray, lam: np.ndarray, threads: int | None = None) -> np.ndarray:
        """Q_h^T (L o (Q_h X Q_w^T)) Q_w per array (Prop. 1, eq. 4), in double.

        x: float32 (batch, rows, cols) or (rows, cols).  lam: (rows, cols) for one
        operator shared by every array, or (batch, rows, cols) for one per array;
        promoted to double exactly.
        """
        squeeze = x.ndim == 2
        xb = np.ascontiguousarray(x[None] if squeeze else x)
        if xb.dtype != np.float32 or xb.ndim != 3:
            raise TypeError("filter takes float32 (batch, rows, cols) input")
        b, h, w = xb.shape
        lm = np.ascontiguousarray(lam, dtype=np.float64)
        if lm.shape == (h, w):
            lam_stride = 0
        elif lm.shape == (b, h, w):
            lam_stride = h * w
        else:
            raise ValueError("lam must be (rows, cols) or (batch, rows, cols)")
        y = np.empty((b, h, w), dtype=np.float64)
        rc = self.lib.oracle_filter(xb.ctypes.data, y.ctypes.data, b, h, w, h * w, lm.ctypes.data,
                                    lam_stride, threads or default_threads())
        if rc != 0:
            raise RuntimeError("oracle_filter failed with %d" % rc)
        return y[0] if squeeze else y


def _default() -> Oracle:
    global _lib
    with _lock:
        if _lib is None:
            _lib = Oracle(build())
    return _lib


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def qmatrix(n: int) -> np.ndarray:
    """Q_n of eq. 1 in double precision."""
    return _default().qmatrix(n)


def forward(x: np.ndarray, threads: int | None = None) -> np.ndarray:
    """Y = Q_h X Q_w^T (eq. 2) for every array in x; double output."""
    return _default().forward(x, threads)


def inverse(y: np.ndarray, threads: int | None = None) -> np.ndarray:
    """X = Q_h^T Y Q_w (eq. 2) for every array in y; double output."""
    return _default().inverse(y, threads)


def roundtrip(x: np.ndarray, threads: int | None = None) -> np.ndarray:
    """inverse(forward(X)) computed in double (exact result: X itself)."""
    return _default().roundtrip(x, threads)


def filter(x: np.ndarray, lam: np.ndarray, threads: int | None = None) -> np.ndarray:
    """Q_h^T (L o (Q_h X Q_w^T)) Q_w per array (Prop. 1, eq. 4), in double."""
    return _default().filter(x, lam, threads)


def e_rel(yhat: np.ndarray, y: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Per-array acceptance metric of Section 6 eq. 5.

    e_rel = ||Yhat - Y||_F / ||X||_F with X the input of that transform.  For a
    zero input the absolute error ||Yhat - Y||_F is returned instead (the paper
    checks zero inputs absolutely; no denominator floor is applied otherwise).
    """
    yhat = np.asarray(yhat, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    if yhat.ndim == 2:
        yhat, y, x = yhat[None], y[None], x[None]
    num = np.sqrt(np.sum((yhat - y) ** 2, axis=(1, 2)))
    den = np.sqrt(np.sum(x * x, axis=(1, 2)))
    out = np.where(den > 0, num / np.where(den > 0, den, 1.0), num)
    return out


def weak_component_error(yhat: np.ndarray, y: np.ndarray, k: int, l: int) -> float:
    """Relative error on one spectral coefficient (Section 6: weak-component loss)."""
    ref = float(y[k, l])
    return abs(float(yhat[k, l]) - ref) / abs(ref) if ref != 0 else abs(float(yhat[k, l]))
