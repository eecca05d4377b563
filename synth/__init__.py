"""Seeded synthetic sparse matrices for the blocked sparse LU workloads.

This module only builds input data: CSR patterns and values of the test
matrices, and seeded right-hand sides.  It contains none of the solver's
arithmetic (no ordering, no fill, no blocking, no factorization), so both the
oracle and the GPU path can consume its output without sharing method code.

All matrices are returned as ``(n, rowptr, colidx, values)`` with

* ``rowptr``: int64[n+1], monotone, ``rowptr[0] == 0``;
* ``colidx``: int32[nnz], strictly increasing inside every row;
* ``values``: float64[nnz], in the same (row-major) order.

Grid points are numbered ``x + nx*(y + ny*z)``; boundaries are Dirichlet,
i.e. a neighbour outside the grid is simply dropped.

The paper measures on SuiteSparse matrices that are not available here; these
generators are synthetic stand-ins with the structural premise the paper relies
on (after a fill-reducing ordering the factor's nonzeros gather in the
bottom-right, a bordered-block-diagonal shape; Section 2.1 and Section 1).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "grid_laplacian",
    "laplacian_2d",
    "laplacian_3d",
    "convection_diffusion_3d",
    "bbd_circuit",
    "batch_system",
    "random_x",
    "csr_matvec",
    "coo_to_csr",
]


def coo_to_csr(n, rows, cols, vals=None):
    """Sort (row, col) pairs into CSR; duplicate pairs keep their first value."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    key = rows * np.int64(n) + cols
    order = np.argsort(key, kind="stable")
    key = key[order]
    keep = np.ones(key.shape[0], dtype=bool)
    keep[1:] = key[1:] != key[:-1]
    sel = order[keep]
    r = rows[sel]
    c = cols[sel]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, r + 1, 1)
    rowptr = np.cumsum(rowptr).astype(np.int64)
    out_vals = None if vals is None else np.asarray(vals, dtype=np.float64)[sel]
    return rowptr, c.astype(np.int32), out_vals


def _grid_stencil(dims, diag, lower, upper):
    """7-point (or 5-point when nz == 1) stencil on an nx*ny*nz grid.

    ``lower[d]`` is the coefficient of the neighbour at -1 along axis d,
    ``upper[d]`` the one at +1.  Returns CSR.
    """
    nx, ny, nz = dims
    n = nx * ny * nz
    idx = np.arange(n, dtype=np.int64)
    x = idx % nx
    y = (idx // nx) % ny
    z = idx // (nx * ny)
    coord = (x, y, z)
    stride = (1, nx, nx * ny)
    rows = [idx]
    cols = [idx]
    vals = [np.full(n, float(diag))]
    for d in range(3):
        ext = dims[d]
        if ext <= 1:
            continue
        m = coord[d] > 0
        rows.append(idx[m]); cols.append(idx[m] - stride[d])
        vals.append(np.full(int(m.sum()), float(lower[d])))
        m = coord[d] < ext - 1
        rows.append(idx[m]); cols.append(idx[m] + stride[d])
        vals.append(np.full(int(m.sum()), float(upper[d])))
    rows = np.concatenate(rows); cols = np.concatenate(cols); vals = np.concatenate(vals)
    rowptr, colidx, values = coo_to_csr(n, rows, cols, vals)
    return n, rowptr, colidx, values


def grid_laplacian(dims):
    """Plain Laplacian on a 2D (nz == 1) or 3D grid: diagonal 2*dim, neighbours -1."""
    dims = tuple(int(v) for v in dims) + (1,) * (3 - len(dims))
    ndim = sum(1 for v in dims if v > 1)
    return _grid_stencil(dims, 2.0 * ndim, (-1.0,) * 3, (-1.0,) * 3)


def laplacian_2d(k):
    """2D 5-point Laplacian on a k x k grid (diagonal 4, neighbours -1)."""
    return _grid_stencil((k, k, 1), 4.0, (-1.0,) * 3, (-1.0,) * 3)


def laplacian_3d(k):
    """3D 7-point Laplacian on a k^3 grid (diagonal 6, neighbours -1)."""
    return _grid_stencil((k, k, k), 6.0, (-1.0,) * 3, (-1.0,) * 3)


def convection_diffusion_3d(k, beta=(10.0, 10.0, 10.0)):
    """-Laplace(u) + beta . grad(u) on the unit cube, first-order upwind.

    k interior points per axis, h = 1/(k+1), scaled by h^2: the diagonal is
    6 + h*sum(beta), the upwind neighbour (at -1 for beta_d > 0) is
    -1 - h*beta_d and the downwind neighbour is -1.  The values are
    unsymmetric while the pattern is symmetric.
    """
    h = 1.0 / (k + 1)
    diag = 6.0 + h * float(sum(abs(b) for b in beta))
    lower = [(-1.0 - h * b) if b >= 0 else -1.0 for b in beta]
    upper = [-1.0 if b >= 0 else (-1.0 + h * b) for b in beta]
    return _grid_stencil((k, k, k), diag, lower, upper)


def bbd_circuit(n=200_000, nblocks=64, border=2_000, per_row=4,
                border_nnz=400_000, seed=0):
    """Bordered-block-diagonal circuit-like matrix.

    Rows ``0 .. n-border-1`` are split into ``nblocks`` diagonal blocks of
    near-equal size; every such row holds its diagonal plus ``per_row``
    uniformly drawn in-block columns.  The last ``border`` rows and columns
    each receive ``border_nnz`` uniformly placed entries.  Off-diagonal values
    are U[-1, 1]; the diagonal is the row's absolute off-diagonal sum plus 1,
    so the matrix is strictly row diagonally dominant.
    """
    rng = np.random.default_rng(seed)
    inner = n - border
    sizes = np.full(nblocks, inner // nblocks, dtype=np.int64)
    sizes[: inner % nblocks] += 1
    starts = np.concatenate([[0], np.cumsum(sizes)])
    rows = []
    cols = []
    for b in range(nblocks):
        lo, hi = starts[b], starts[b + 1]
        r = np.repeat(np.arange(lo, hi, dtype=np.int64), per_row)
        c = rng.integers(lo, hi, size=r.shape[0], dtype=np.int64)
        rows.append(r); cols.append(c)
    # border rows x all columns, all rows x border columns
    rows.append(rng.integers(inner, n, size=border_nnz, dtype=np.int64))
    cols.append(rng.integers(0, n, size=border_nnz, dtype=np.int64))
    rows.append(rng.integers(0, n, size=border_nnz, dtype=np.int64))
    cols.append(rng.integers(inner, n, size=border_nnz, dtype=np.int64))
    rows = np.concatenate(rows); cols = np.concatenate(cols)
    off = rows != cols
    rows = rows[off]; cols = cols[off]
    rowptr, colidx, _ = coo_to_csr(n, rows, cols)
    offvals = rng.uniform(-1.0, 1.0, size=colidx.shape[0])
    absrow = np.add.reduceat(np.abs(offvals), rowptr[:-1]) if colidx.shape[0] else np.zeros(n)
    absrow = np.where(np.diff(rowptr) > 0, absrow, 0.0)
    # insert the diagonal
    r_all = np.concatenate([np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr)),
                            np.arange(n, dtype=np.int64)])
    c_all = np.concatenate([colidx.astype(np.int64), np.arange(n, dtype=np.int64)])
    v_all = np.concatenate([offvals, absrow + 1.0])
    rowptr, colidx, values = coo_to_csr(n, r_all, c_all, v_all)
    return n, rowptr, colidx, values


def batch_system(s):
    """System ``s`` (0..255) of the batch workload.

    ``n_target`` ~ U{2000..20000} from ``default_rng(s)``.  Systems 0..127 are
    2D 5-point grids with k = round(sqrt(n_target)); systems 128..255 are 3D
    7-point grids with k = round(cbrt(n_target)).  The diagonal is scaled by
    d_i ~ U[1, 2] and every off-diagonal is -1 + delta, delta ~ U[-0.1, 0.1].
    """
    rng = np.random.default_rng(s)
    n_target = int(rng.integers(2000, 20000, endpoint=True))
    if s < 128:
        k = int(round(n_target ** 0.5))
        n, rowptr, colidx, values = laplacian_2d(k)
        dims = (k, k, 1)
    else:
        k = int(round(n_target ** (1.0 / 3.0)))
        n, rowptr, colidx, values = laplacian_3d(k)
        dims = (k, k, k)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr))
    isdiag = rows == colidx
    d = rng.uniform(1.0, 2.0, size=n)
    values = values.copy()
    values[isdiag] *= d
    noff = int((~isdiag).sum())
    values[~isdiag] = -1.0 + rng.uniform(-0.1, 0.1, size=noff)
    return n, rowptr, colidx, values, dims


def random_x(n, nrhs=1, seed=0):
    """Seeded solution block X ~ U[-1, 1], column-major (n, nrhs) float64."""
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.uniform(-1.0, 1.0, size=(nrhs, n)).T)


def csr_matvec(n, rowptr, colidx, values, x):
    """B = A @ X for X of shape (n,) or (n, k), float64 (input preparation)."""
    x = np.asarray(x, dtype=np.float64)
    vec = x.ndim == 1
    xm = x[:, None] if vec else x
    prod = values[:, None] * xm[colidx]
    out = np.zeros((n, xm.shape[1]))
    nonempty = np.diff(rowptr) > 0
    if prod.shape[0]:
        sums = np.add.reduceat(prod, rowptr[:-1][nonempty], axis=0)
        out[nonempty] = sums
    return out[:, 0] if vec else np.asfortranarray(out)
