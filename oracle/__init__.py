"""Plain FP64 CPU oracle for sliding-window cumulant tensors (arXiv:1701.06446).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code
with the HIP library: its arithmetic lives in ``orc.c`` (compiled with gcc) and in
the numpy helpers of ``full.py`` that work on full n^k tensors for tiny n.

What it computes (the plain definition that the sliding method reaches exactly):
for the current window of t rows, the raw moments of Eq. (mom) in the block
("hyper-pyramid") layout of Sec. 2.3, updated per Eq. (momupdate); cumulants by
Alg. 3/4 (all set partitions, singletons included, Sec. 2.6); Frobenius norms by
Alg. 5 and the estimator nu_k of Eq. (mef).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "orc.c")
_LIB = os.path.join(_HERE, "liborc.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile ``orc.c`` into ``liborc.so`` with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        i64, i32, dbl = ctypes.c_int64, ctypes.c_int, ctypes.c_double
        pd = ctypes.POINTER(ctypes.c_double)
        lib.orc_count_tuples.restype = i64
        lib.orc_count_tuples.argtypes = [i32, i32]
        lib.orc_tuples.restype = None
        lib.orc_tuples.argtypes = [i32, i32, ctypes.POINTER(ctypes.c_int)]
        lib.orc_sums_add.restype = None
        lib.orc_sums_add.argtypes = [pd, i64, i32, i32, i32, dbl, pd, pd]
        lib.orc_count_partitions.restype = i64
        lib.orc_count_partitions.argtypes = [i32, i32]
        lib.orc_moms2cums.restype = i32
        lib.orc_moms2cums.argtypes = [i32, i32, i32, ctypes.POINTER(pd), ctypes.POINTER(pd)]
        lib.orc_block_norm.restype = dbl
        lib.orc_block_norm.argtypes = [i32, i32, i32, pd]
        lib.orc_norms.restype = None
        lib.orc_norms.argtypes = [i32, i32, i32, ctypes.POINTER(pd), pd, pd]
        lib.orc_num_threads.restype = i32
        lib.orc_num_threads.argtypes = []
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def nblocks(n: int, b: int, k: int) -> int:
    """Stored blocks of an order-k tensor, counted by walking the tuples."""
    return int(_load().orc_count_tuples((n + b - 1) // b, k))


def tuples(n: int, b: int, k: int) -> np.ndarray:
    """Non-decreasing block tuples of order k in lexicographic order."""
    nbar = (n + b - 1) // b
    cnt = int(_load().orc_count_tuples(nbar, k))
    out = np.zeros((cnt, k), dtype=np.int32)
    _load().orc_tuples(nbar, k, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    return out


def num_threads() -> int:
    """Threads the oracle's OpenMP loops use."""
    return int(_load().orc_num_threads())


def count_partitions(s: int, sigma: int) -> int:
    return int(_load().orc_count_partitions(s, sigma))


def pyramid_size(n: int, b: int, k: int) -> int:
    return nblocks(n, b, k) * b ** k


def _as_rows(X) -> np.ndarray:
    X = np.ascontiguousarray(np.asarray(X, dtype=np.float64))
    assert X.ndim == 2
    return X


class SlidingOracle:
    """The sliding-window state of Alg. 1 in FP64: compensated sums S_k for
    k = 1..d, the window length t, and the combine/norm steps on demand."""

    def __init__(self, X, n: int, d: int, b: int):
        X = _as_rows(X)
        assert X.shape[1] == n and 1 <= d <= 6 and b >= 1
        self.n, self.d, self.b, self.t = n, d, b, X.shape[0]
        self.S = [np.zeros(pyramid_size(n, b, k)) for k in range(1, d + 1)]
        self.c = [np.zeros_like(s) for s in self.S]
        self._add(X, +1.0)

    def _add(self, X, sign):
        lib = _load()
        for k in range(1, self.d + 1):
            lib.orc_sums_add(_ptr(X), X.shape[0], self.n, self.b, k, sign,
                             _ptr(self.S[k - 1]), _ptr(self.c[k - 1]))

    def update(self, X_new, X_old):
        """Eq. (momupdate): the window drops X_old (its oldest rows) and gains X_new."""
        X_new, X_old = _as_rows(X_new), _as_rows(X_old)
        assert X_new.shape == X_old.shape and X_new.shape[1] == self.n
        self._add(X_new, +1.0)
        self._add(X_old, -1.0)

    def sums(self):
        return [s + c for s, c in zip(self.S, self.c)]

    def moments(self):
        """M_k = S_k / t (Eq. (mom))."""
        return [s / self.t for s in self.sums()]

    def cumulants(self):
        return moms2cums(self.moments(), self.n, self.b)

    def norms(self):
        return norms(self.cumulants(), self.n, self.b)


def moments_of(X, n: int, d: int, b: int):
    """Moments of a whole window computed from scratch (the recomputation)."""
    return SlidingOracle(X, n, d, b).moments()


def moms2cums(M, n: int, b: int):
    """Alg. 3/4 on pyramid-form moments M[0..d-1] (FP64)."""
    lib = _load()
    d = len(M)
    M = [np.ascontiguousarray(m, dtype=np.float64) for m in M]
    C = [np.zeros_like(m) for m in M]
    Mp = (ctypes.POINTER(ctypes.c_double) * d)(*[_ptr(m) for m in M])
    Cp = (ctypes.POINTER(ctypes.c_double) * d)(*[_ptr(c) for c in C])
    rc = lib.orc_moms2cums(n, b, d, Mp, Cp)
    if rc != 0:
        raise MemoryError("oracle combine failed")
    return C


def block_norm(A, n: int, b: int, k: int) -> float:
    """Alg. 5 with exponent 2 on one order-k pyramid."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    return float(_load().orc_block_norm(n, b, k, _ptr(A)))


def norms(C, n: int, b: int):
    """Returns (fro, nu): fro[k] = ||C_k||_F for k = 1..d, nu[k] per Eq. (mef)
    for k >= 3 (NaN elsewhere)."""
    lib = _load()
    d = len(C)
    C = [np.ascontiguousarray(c, dtype=np.float64) for c in C]
    fro = np.zeros(d + 1)
    nu = np.zeros(d + 1)
    Cp = (ctypes.POINTER(ctypes.c_double) * d)(*[_ptr(c) for c in C])
    lib.orc_norms(n, b, d, Cp, _ptr(fro), _ptr(nu))
    return fro, nu
