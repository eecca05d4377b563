"""Adjoint of the solve x = A^{-1} b (test infrastructure only).

For a scalar loss with dloss/dx = w, the gradient with respect to b is
g = A^{-T} w and, since dx = -A^{-1} (dA) x, the gradient with respect to an
entry a_ij of A is -g_i x_j; only entries in A's pattern are variables.
Written from that definition with the oracle's own factorization and solves
(``numeric``); it shares nothing with the HIP path.
"""
from __future__ import annotations

import numpy as np

from . import numeric, symbolic


def solve_gradients(n, rowptr, colidx, values, perm, B, W):
    """(X, grad_B, grad_values) for loss = sum(W * X), X = A^{-1} B.

    B, W: (n,) or (n, k).  grad_values follows A's CSR order."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colidx = np.asarray(colidx, dtype=np.int64)
    cp, ri = symbolic.symbolic(n, rowptr, colidx, perm)
    F = numeric.factor(n, rowptr, colidx, values, perm, cp, ri)
    X = numeric.solve(F, B)
    G = numeric.solve(F, W, transpose=True)
    X2 = X.reshape(n, -1)
    G2 = G.reshape(n, -1)
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    grad_values = -np.sum(G2[rows] * X2[colidx], axis=1)
    return X, G, grad_values
