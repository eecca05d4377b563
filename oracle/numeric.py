"""Python side of the oracle's numeric core (test infrastructure only).

Loads ``oracle/numeric.c`` (built with gcc into ``oracle/_numeric.so``) and
exposes the no-pivot right-looking LU on S, the solves and their transposes.
See ``numeric.c`` for the storage layout and the paper passages it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import ordering as _ord

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "numeric.c")
_LIB = os.path.join(_HERE, "_numeric.so")
_lib = None


def build(force=True):
    """Compile the oracle's C core with gcc (IEEE fp64, no contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math",
                               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        i64, p = ctypes.c_int64, ctypes.c_void_p
        lib.oracle_scatter.argtypes = [i64, p, p, p, p, p, p, p, p]
        lib.oracle_scatter.restype = ctypes.c_int
        lib.oracle_factor.argtypes = [i64, i64, p, p, p, p]
        lib.oracle_factor.restype = i64
        lib.oracle_solve.argtypes = [i64, p, p, p, p, p, i64, i64, ctypes.c_int]
        lib.oracle_solve.restype = None
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class ZeroPivot(RuntimeError):
    def __init__(self, col):
        super().__init__("zero or non-finite pivot at permuted column %d" % col)
        self.col = col


class Factors:
    """L and U of A[perm][:, perm] on S (see numeric.c for the layout)."""

    def __init__(self, n, perm, colptr, rowidx, lval, uval):
        self.n = n
        self.perm = np.asarray(perm, dtype=np.int32)
        self.colptr = colptr
        self.rowidx = rowidx
        self.lval = lval
        self.uval = uval

    def diag(self):
        return self.lval[self.colptr[:-1]]

    def dense(self):
        """Dense (L, U) for small n."""
        n = self.n
        L = np.eye(n)
        U = np.zeros((n, n))
        cols = np.repeat(np.arange(n), np.diff(self.colptr))
        r = self.rowidx.astype(np.int64)
        low = r > cols
        L[r[low], cols[low]] = self.lval[low]
        U[cols[low], r[low]] = self.uval[low]
        U[cols[~low], cols[~low]] = self.lval[~low]
        return L, U


def scatter(n, rowptr, colidx, values, perm, colptr, rowidx):
    """Values of A[perm][:, perm] placed on S (lval, uval)."""
    lib = _load()
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    colidx = np.ascontiguousarray(colidx, dtype=np.int32)
    values = np.ascontiguousarray(values, dtype=np.float64)
    inv = np.ascontiguousarray(_ord.inverse(perm), dtype=np.int32)
    colptr = np.ascontiguousarray(colptr, dtype=np.int64)
    rowidx = np.ascontiguousarray(rowidx, dtype=np.int32)
    lval = np.zeros(int(colptr[-1]))
    uval = np.zeros(int(colptr[-1]))
    rc = lib.oracle_scatter(n, _ptr(rowptr), _ptr(colidx), _ptr(values), _ptr(inv),
                            _ptr(colptr), _ptr(rowidx), _ptr(lval), _ptr(uval))
    if rc != 0:
        raise ValueError("an entry of A is not in the symbolic pattern")
    return lval, uval


def factor(n, rowptr, colidx, values, perm, colptr, rowidx, kmax=None):
    """No-pivot right-looking LU of A[perm][:, perm] on S.

    ``kmax`` limits the elimination to the first kmax columns (a partial
    factorization: the trailing part then holds the Schur complement).
    """
    lval, uval = scatter(n, rowptr, colidx, values, perm, colptr, rowidx)
    colptr = np.ascontiguousarray(colptr, dtype=np.int64)
    rowidx = np.ascontiguousarray(rowidx, dtype=np.int32)
    km = n if kmax is None else int(kmax)
    rc = _load().oracle_factor(n, km, _ptr(colptr), _ptr(rowidx), _ptr(lval), _ptr(uval))
    if rc == -2:
        raise ValueError("pattern is not closed under fill")
    if rc < 0:
        raise MemoryError("oracle_factor")
    if rc > 0:
        raise ZeroPivot(int(rc) - 1)
    return Factors(n, perm, colptr, rowidx, lval, uval)


def solve(F, B, transpose=False):
    """X = A^{-1} B (or A^{-T} B) using the factors of A[perm][:, perm].

    A = P^T L U P with (P v) = v[perm]; so x = P^T U^{-1} L^{-1} P b and
    x = P^T L^{-T} U^{-T} P b for the transpose.
    """
    B = np.asarray(B, dtype=np.float64)
    vec = B.ndim == 1
    Bm = B[:, None] if vec else B
    W = np.asfortranarray(Bm[F.perm, :])
    _load().oracle_solve(F.n, _ptr(F.colptr), _ptr(F.rowidx), _ptr(F.lval), _ptr(F.uval),
                         _ptr(W), W.shape[1], F.n, 1 if transpose else 0)
    X = np.empty_like(W)
    X[F.perm, :] = W
    return X[:, 0] if vec else X
