"""Symbolic factorization for the oracle (test infrastructure only).

The paper's symbolic phase predicts the nonzero pattern of L and U before the
numeric phase (Section 1, Section 2.1) and treats the result as structurally
symmetric (Section 4.2).  The reading used here: S is the fill of the
symmetrised, permuted pattern

    P0 = pattern(A) | pattern(A^T) | diag,   B = P0[perm][:, perm],

under elimination in the order 0..n-1.  By the fill-path theorem, (i, j) is
in S iff i and j are joined in the graph of B by a path whose interior
vertices are all numbered below min(i, j).  It is computed column by column
with the elimination-tree recurrence

    Struct(L[:, k]) = Adj_{>k}(k)  union  (union over children c of k of
                      Struct(L[:, c]) minus {k}),

where the parent of c is the smallest row of Struct(L[:, c]).

S is returned as its lower triangle in CSC form, diagonal included, rows
sorted inside every column: ``colptr`` int64[n+1], ``rowidx`` int32.
Since S is symmetric, the upper triangle is the transpose of this pattern.
"""
from __future__ import annotations

import numpy as np


def symmetric_pattern(n, rowptr, colidx):
    """CSR pattern of A + A^T + I (sorted, no duplicates)."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colidx = np.asarray(colidx, dtype=np.int64)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr))
    diag = np.arange(n, dtype=np.int64)
    r = np.concatenate([rows, colidx, diag])
    c = np.concatenate([colidx, rows, diag])
    key = np.unique(r * np.int64(n) + c)
    r = key // n
    c = key % n
    ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(ptr, r + 1, 1)
    return np.cumsum(ptr), c.astype(np.int32)


def permute_symmetric(n, ptr, idx, perm):
    """Pattern of P0[perm][:, perm] for a symmetric CSR pattern P0."""
    perm = np.asarray(perm, dtype=np.int64)
    inv = np.empty(n, dtype=np.int64)
    inv[perm] = np.arange(n, dtype=np.int64)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(ptr))
    r = inv[rows]
    c = inv[np.asarray(idx, dtype=np.int64)]
    key = np.sort(r * np.int64(n) + c)
    r = key // n
    c = key % n
    nptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(nptr, r + 1, 1)
    return np.cumsum(nptr), c.astype(np.int32)


def etree(n, ptr, idx):
    """Elimination tree of a symmetric pattern (Liu's algorithm, path compression).

    parent[j] = -1 for a root.
    """
    parent = np.full(n, -1, dtype=np.int64)
    anc = np.full(n, -1, dtype=np.int64)
    idx = np.asarray(idx, dtype=np.int64)
    for j in range(n):
        for i in idx[ptr[j]:ptr[j + 1]].tolist():
            if i >= j:
                continue
            while True:
                a = anc[i]
                if a == j:
                    break
                anc[i] = j
                if a == -1:
                    parent[i] = j
                    break
                i = a
    return parent


def fill_lower(n, ptr, idx):
    """Lower-CSC pattern (diagonal included) of the fill of a symmetric pattern.

    ``ptr``/``idx`` describe a symmetric pattern in CSR (equal to its CSC).
    """
    idx = np.asarray(idx, dtype=np.int64)
    pending = [[] for _ in range(n)]
    cols = []
    counts = np.zeros(n, dtype=np.int64)
    for k in range(n):
        a = idx[ptr[k]:ptr[k + 1]]
        parts = [a[a > k]]
        parts.extend(pending[k])
        pending[k] = None
        s = np.unique(np.concatenate(parts)) if len(parts) > 1 else parts[0]
        # children structures carry k itself; it is not strictly below k
        s = s[s > k]
        if s.shape[0]:
            pending[int(s[0])].append(s[1:])
        cols.append(np.concatenate([[k], s]))
        counts[k] = s.shape[0] + 1
    colptr = np.zeros(n + 1, dtype=np.int64)
    colptr[1:] = np.cumsum(counts)
    rowidx = np.concatenate(cols).astype(np.int32) if n else np.zeros(0, np.int32)
    return colptr, rowidx


def symbolic(n, rowptr, colidx, perm):
    """S for matrix A (CSR pattern) under ordering ``perm`` (new -> old)."""
    ptr, idx = symmetric_pattern(n, rowptr, colidx)
    pptr, pidx = permute_symmetric(n, ptr, idx, perm)
    return fill_lower(n, pptr, pidx)


def fill_dense_bruteforce(mask):
    """Fill of a dense boolean symmetric pattern by explicit elimination.

    For k = 0..n-1 every pair of neighbours of k numbered above k becomes
    adjacent.  Returns the filled boolean matrix (symmetric, diagonal set).
    """
    m = np.array(mask, dtype=bool, copy=True)
    n = m.shape[0]
    np.fill_diagonal(m, True)
    for k in range(n):
        nb = np.nonzero(m[k + 1:, k])[0] + k + 1
        if nb.shape[0]:
            m[np.ix_(nb, nb)] = True
    return m


def lower_to_dense(n, colptr, rowidx):
    """Dense symmetric boolean matrix of a lower-CSC pattern."""
    m = np.zeros((n, n), dtype=bool)
    cols = np.repeat(np.arange(n), np.diff(colptr))
    m[rowidx, cols] = True
    m[cols, rowidx] = True
    return m
