"""Flop count and backward error for the oracle (test infrastructure only).

* ``flops``: the work of the no-pivot LU on S.  The paper's tables quote
  "FLOPs" without a definition (Table 3); the reading used is the algorithmic
  count on S, identical for every blocking:
      F = sum_k [ (c_k - 1) + 2 (c_k - 1)(r_k - 1) ],
  c_k = |S(k:n, k)|, r_k = |S(k, k:n)| (one division per sub-diagonal entry,
  one multiply-add per update).  S is symmetric, so c_k = r_k.
* ``backward_error``: the normwise (Rigal-Gaches) backward error per
  right-hand side, eta = ||b - A x||_inf / (||A||_inf ||x||_inf + ||b||_inf),
  on the original, unpermuted A, in fp64.
"""
from __future__ import annotations

import numpy as np


def flops(colptr, kmax=None):
    c = np.diff(np.asarray(colptr, dtype=np.int64))   # c_k (diagonal included)
    if kmax is not None:
        c = c[: int(kmax)]
    l = c - 1
    return int(np.sum(l + 2 * l * l))


def residual(n, rowptr, colidx, values, X, B):
    """R = B - A X in fp64 (X and B of shape (n,) or (n, k)), one row
    reduction per row of A."""
    X = np.asarray(X, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    vec = X.ndim == 1
    Xm = X[:, None] if vec else X
    Bm = B[:, None] if vec else B
    rp = np.asarray(rowptr, dtype=np.int64)
    prod = np.asarray(values)[:, None] * Xm[np.asarray(colidx, dtype=np.int64)]
    AX = np.zeros_like(Bm, dtype=np.float64)
    ne = np.diff(rp) > 0
    if prod.shape[0]:
        AX[ne] = np.add.reduceat(prod, rp[:-1][ne], axis=0)
    R = Bm - AX
    return R[:, 0] if vec else R


def norm_inf_matrix(n, rowptr, values):
    rp = np.asarray(rowptr, dtype=np.int64)
    a = np.abs(np.asarray(values, dtype=np.float64))
    ne = np.diff(rp) > 0
    s = np.zeros(n)
    if a.shape[0]:
        s[ne] = np.add.reduceat(a, rp[:-1][ne])
    return float(s.max()) if n else 0.0


def backward_error(n, rowptr, colidx, values, X, B, transpose=False):
    """Normwise backward error per right-hand side (array of length nrhs).

    With ``transpose`` the system is A^T x = b: the residual uses A^T and the
    norm ||A^T||_inf = ||A||_1.
    """
    X = np.asarray(X, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    Xm = X[:, None] if X.ndim == 1 else X
    Bm = B[:, None] if B.ndim == 1 else B
    rp = np.asarray(rowptr, dtype=np.int64)
    ci = np.asarray(colidx, dtype=np.int64)
    v = np.asarray(values, dtype=np.float64)
    if transpose:
        rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
        order = np.lexsort((rows, ci))
        tptr = np.zeros(n + 1, dtype=np.int64)
        np.add.at(tptr, ci + 1, 1)
        tptr = np.cumsum(tptr)
        rp, ci, v = tptr, rows[order], v[order]
    R = residual(n, rp, ci, v, Xm, Bm)
    na = norm_inf_matrix(n, rp, v)
    nx = np.abs(Xm).max(axis=0) if n else np.zeros(Xm.shape[1])
    nb = np.abs(Bm).max(axis=0) if n else np.zeros(Bm.shape[1])
    nr = np.abs(R).max(axis=0) if n else np.zeros(Bm.shape[1])
    den = na * nx + nb
    with np.errstate(invalid="ignore", divide="ignore"):
        eta = np.where(den > 0, nr / np.where(den > 0, den, 1.0), 0.0)
    return eta
