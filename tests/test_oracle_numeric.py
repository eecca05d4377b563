"""Pins of the oracle's numeric part (no-pivot LU on S, solves, flops, eta).

Independent references: a dense Doolittle elimination written out here,
scipy's SuperLU with natural ordering and no pivoting, closed forms of the
tridiagonal (-1, 2, -1) factors, the LDL^T relation for symmetric matrices,
and exact solutions."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synth
from oracle import metrics, ordering, symbolic


def _dense(n, rp, ci, v):
    A = np.zeros((n, n))
    rows = np.repeat(np.arange(n), np.diff(rp))
    A[rows, ci] = v
    return A


def _doolittle(A):
    """Textbook dense LU without pivoting (unit lower L)."""
    n = A.shape[0]
    U = np.zeros_like(A)
    L = np.eye(n)
    for i in range(n):
        for j in range(i, n):
            U[i, j] = A[i, j] - L[i, :i] @ U[:i, j]
        for j in range(i + 1, n):
            L[j, i] = (A[j, i] - L[j, :i] @ U[:i, i]) / U[i, i]
    return L, U


def _random_dd(n, dens, rng):
    m = rng.random((n, n)) < dens
    A = np.where(m, rng.uniform(-1, 1, (n, n)), 0.0)
    np.fill_diagonal(A, 0.0)
    np.fill_diagonal(A, np.abs(A).sum(axis=1) + 1.0)
    rows, cols = np.nonzero(A)
    rp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rp, rows + 1, 1)
    return np.cumsum(rp), cols.astype(np.int32), A[rows, cols], A


@pytest.mark.parametrize("seed", range(8))
def test_factor_matches_doolittle(oracle_lib, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 48))
    rp, ci, v, A = _random_dd(n, 0.12, rng)
    perm = rng.permutation(n).astype(np.int32)
    cp, ri = symbolic.symbolic(n, rp, ci, perm)
    F = oracle_lib.factor(n, rp, ci, v, perm, cp, ri)
    L, U = F.dense()
    Ld, Ud = _doolittle(A[np.ix_(perm, perm)])
    np.testing.assert_allclose(L, Ld, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(U, Ud, rtol=1e-12, atol=1e-14)
    # entries outside S are exactly zero in the dense reference too
    S = symbolic.lower_to_dense(n, cp, ri)
    assert np.all(Ld[~S] == 0.0) and np.all(Ud[~S] == 0.0)


def test_tridiagonal_closed_form(oracle_lib):
    n = 30
    rows, cols, vals = [], [], []
    for i in range(n):
        for j, a in ((i - 1, -1.0), (i, 2.0), (i + 1, -1.0)):
            if 0 <= j < n:
                rows.append(i); cols.append(j); vals.append(a)
    rp, ci, v = synth.coo_to_csr(n, rows, cols, vals)
    perm = np.arange(n, dtype=np.int32)
    cp, ri = symbolic.symbolic(n, rp, ci, perm)
    F = oracle_lib.factor(n, rp, ci, v, perm, cp, ri)
    L, U = F.dense()
    k = np.arange(1, n + 1, dtype=np.float64)      # 1-based
    np.testing.assert_allclose(np.diag(U), (k + 1) / k, rtol=1e-15)
    np.testing.assert_allclose(np.diag(L, -1), -k[:-1] / (k[:-1] + 1), rtol=1e-15)
    np.testing.assert_allclose(np.diag(U, 1), -1.0, rtol=0)
    assert abs(np.prod(np.diag(U)) - (n + 1)) < 1e-10


def test_symmetric_ldlt_relation(oracle_lib):
    # A symmetric: U = diag(U) L^T
    n, rp, ci, v = synth.laplacian_2d(16)
    perm = ordering.nd_grid((16, 16))
    cp, ri = symbolic.symbolic(n, rp, ci, perm)
    F = oracle_lib.factor(n, rp, ci, v, perm, cp, ri)
    d = F.diag()
    cols = np.repeat(np.arange(n), np.diff(cp))
    low = ri > cols
    np.testing.assert_allclose(F.uval[low], d[cols[low]] * F.lval[low], rtol=1e-13, atol=1e-15)


def test_matches_scipy_superlu_natural(oracle_lib):
    n, rp, ci, v, dims = synth.batch_system(130)     # 3D, unsymmetric values
    assert dims[2] > 1 and n > 3000
    perm = ordering.nd_grid(dims)
    cp, ri = symbolic.symbolic(n, rp, ci, perm)
    F = oracle_lib.factor(n, rp, ci, v, perm, cp, ri)
    A = sp.csr_matrix((v, ci, rp), shape=(n, n))
    Ap = A[perm][:, perm].tocsc()
    lu = spla.splu(Ap, permc_spec="NATURAL", diag_pivot_thresh=0.0,
                   options=dict(SymmetricMode=True))
    assert np.all(lu.perm_r == np.arange(n)) and np.all(lu.perm_c == np.arange(n))
    cols = np.repeat(np.arange(n), np.diff(cp))
    r = ri.astype(np.int64)
    low = r > cols
    L = sp.csr_matrix((np.concatenate([F.lval[low], np.ones(n)]),
                       (np.concatenate([r[low], np.arange(n)]), np.concatenate([cols[low], np.arange(n)]))),
                      shape=(n, n))
    U = sp.csr_matrix((np.concatenate([F.uval[low], F.diag()]),
                       (np.concatenate([cols[low], np.arange(n)]), np.concatenate([r[low], np.arange(n)]))),
                      shape=(n, n))
    dl = abs(L - lu.L).max()
    du = abs(U - lu.U).max()
    assert dl <= 1e-12 * abs(L).max() and du <= 1e-12 * abs(U).max()


@pytest.mark.parametrize("case", ["lap2d", "lap3d", "convdiff", "batch"])
def test_solve_and_backward_error(oracle_lib, case):
    if case == "lap2d":
        n, rp, ci, v = synth.laplacian_2d(40); dims = (40, 40, 1)
    elif case == "lap3d":
        n, rp, ci, v = synth.laplacian_3d(12); dims = (12, 12, 12)
    elif case == "convdiff":
        n, rp, ci, v = synth.convection_diffusion_3d(12); dims = (12, 12, 12)
    else:
        n, rp, ci, v, dims = synth.batch_system(5)
    perm = ordering.nd_grid(dims)
    cp, ri = symbolic.symbolic(n, rp, ci, perm)
    F = oracle_lib.factor(n, rp, ci, v, perm, cp, ri)
    xt = synth.random_x(n, 3, seed=1)
    b = synth.csr_matvec(n, rp, ci, v, xt)
    x = oracle_lib.solve(F, b)
    eta = metrics.backward_error(n, rp, ci, v, x, b)
    assert np.all(eta <= 1e-14)
    assert np.max(np.abs(x - xt)) < 1e-11
    # transpose solve
    A = _dense(n, rp, ci, v) if n <= 2000 else None
    bt = synth.csr_matvec(n, rp, ci, v, np.ones(n))
    xtr = oracle_lib.solve(F, bt, transpose=True)
    eta_t = metrics.backward_error(n, rp, ci, v, xtr, bt, transpose=True)
    assert np.all(eta_t <= 1e-14)
    if A is not None:
        np.testing.assert_allclose(A.T @ xtr, bt, rtol=0, atol=1e-12)


def test_ones_solution_exact(oracle_lib):
    n, rp, ci, v = synth.laplacian_2d(64)
    perm = ordering.nd_grid((64, 64))
    cp, ri = symbolic.symbolic(n, rp, ci, perm)
    F = oracle_lib.factor(n, rp, ci, v, perm, cp, ri)
    b = synth.csr_matvec(n, rp, ci, v, np.ones(n))
    x = oracle_lib.solve(F, b)
    assert np.max(np.abs(x - 1.0)) < 1e-12


def test_zero_pivot_reported(oracle_lib):
    # [[0, 1], [1, 0]] has a zero leading pivot without row exchanges
    rp = np.array([0, 1, 2], dtype=np.int64)
    ci = np.array([1, 0], dtype=np.int32)
    v = np.array([1.0, 1.0])
    perm = np.arange(2, dtype=np.int32)
    cp, ri = symbolic.symbolic(2, rp, ci, perm)
    with pytest.raises(oracle_lib.ZeroPivot) as e:
        oracle_lib.factor(2, rp, ci, v, perm, cp, ri)
    assert e.value.col == 0
    # a pivot that becomes zero after an update: [[1, 1], [1, 1]]
    rp = np.array([0, 2, 4], dtype=np.int64)
    ci = np.array([0, 1, 0, 1], dtype=np.int32)
    cp, ri = symbolic.symbolic(2, rp, ci, perm)
    with pytest.raises(oracle_lib.ZeroPivot) as e:
        oracle_lib.factor(2, rp, ci, np.ones(4), perm, cp, ri)
    assert e.value.col == 1
    # non-finite values
    with pytest.raises(oracle_lib.ZeroPivot):
        oracle_lib.factor(2, rp, ci, np.array([np.nan, 1, 1, 3.0]), perm, cp, ri)


def test_partial_factor_is_schur_complement(oracle_lib):
    rng = np.random.default_rng(7)
    n = 30
    rp, ci, v, A = _random_dd(n, 0.15, rng)
    perm = np.arange(n, dtype=np.int32)
    cp, ri = symbolic.symbolic(n, rp, ci, perm)
    kmax = 12
    F = oracle_lib.factor(n, rp, ci, v, perm, cp, ri, kmax=kmax)
    L, U = F.dense()
    A11, A12, A21, A22 = A[:kmax, :kmax], A[:kmax, kmax:], A[kmax:, :kmax], A[kmax:, kmax:]
    schur = A22 - A21 @ np.linalg.solve(A11, A12)
    # trailing part of the stored arrays holds the Schur complement
    T = np.tril(L[kmax:, kmax:], -1) + U[kmax:, kmax:]
    np.testing.assert_allclose(T, schur, rtol=1e-11, atol=1e-12)


def test_flops_closed_forms():
    n = 25
    # dense: every column has n-k-1 sub-diagonal entries
    cp = np.concatenate([[0], np.cumsum(np.arange(n, 0, -1))])
    assert metrics.flops(cp) == n * (n - 1) // 2 + (n - 1) * n * (2 * n - 1) // 3
    # tridiagonal: one sub-diagonal entry per column but the last
    cp = np.concatenate([[0], np.cumsum([2] * (n - 1) + [1])])
    assert metrics.flops(cp) == 3 * (n - 1)


def test_backward_error_known_values():
    n = 3
    A = np.array([[2.0, 0, 0], [0, 4.0, 0], [1.0, 0, 1.0]])
    rows, cols = np.nonzero(A)
    rp = np.array([0, 1, 2, 4], dtype=np.int64)
    ci = cols.astype(np.int32)
    v = A[rows, cols]
    x = np.array([1.0, 1.0, 1.0])
    b = A @ x
    assert metrics.backward_error(n, rp, ci, v, x, b)[0] == 0.0
    # ||A||_inf = 4, ||x|| = 1, ||b2||_inf = 4, residual 0.5 on one entry
    b2 = b.copy(); b2[0] += 0.5
    eta = metrics.backward_error(n, rp, ci, v, x, b2)[0]
    assert abs(eta - 0.5 / (4 * 1 + 4)) < 1e-16
    # transpose: ||A^T||_inf = ||A||_1 = 4
    bt = A.T @ x
    assert metrics.backward_error(n, rp, ci, v, x, bt, transpose=True)[0] == 0.0
