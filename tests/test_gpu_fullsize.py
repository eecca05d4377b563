"""Parity at full size: the 3D 7-point Laplacian on 48^3 (n = 110,592) in
the launch configuration the benchmark times (grid nested dissection,
irregular blocking of Algorithm 3, wave schedule, FP64).

The oracle cannot factor the whole matrix in seconds, so the factors are
checked by what holds at any size, each independent of the HIP path:

* the pattern and the ordering equal the oracle's;
* the oracle's right-looking LU stopped after the first kmax pivots has the
  final values of L's first kmax columns and U's first kmax rows: those
  entries are compared one by one (same tolerance as the small cases);
* A is symmetric, so the unique no-pivot LU has U = diag(U) L^T (every entry);
* A' = L U on randomly sampled entries of S, within the rounding bound of
  Gaussian elimination;
* solves reach a backward error <= 1e-12, recomputed on the host;
* irregular and regular (b = 500) blocking give the same factors to rounding.
"""
import numpy as np
import pytest

import synth
from gpu_common import ETA_MAX, announce, factor_close
from oracle import metrics, numeric, ordering, symbolic

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

K = 48
DIMS = (K, K, K)
ORACLE_FLOPS = 3e9       # work of the oracle's leading pivots (a few seconds)


@pytest.fixture(scope="module")
def big():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2512_04389_amd as slu
    n, rp, ci, v = synth.laplacian_3d(K)
    announce("lap3d-48 full size: analyze + factor (irregular, waves)")
    h = slu.SparseLU(n, rp, ci, ordering="grid_nd", grid_dims=DIMS).bind()
    vals = torch.from_numpy(v).cuda()
    h.factor(vals)
    lv, uv = h.factors()
    cp, ri = h.pattern()
    yield dict(h=h, n=n, rp=rp, ci=ci, v=v, vals=vals, lv=lv, uv=uv, cp=cp, ri=ri)
    h.close()


def test_fullsize_ordering_and_pattern(big):
    n = big["n"]
    perm = ordering.nd_grid(DIMS)
    assert np.array_equal(big["h"].perm(), perm)
    cp, ri = symbolic.symbolic(n, big["rp"], big["ci"], perm)
    assert np.array_equal(big["cp"], cp) and np.array_equal(big["ri"], ri)


def test_fullsize_leading_pivots_match_oracle(big):
    n, cp, ri = big["n"], big["cp"], big["ri"]
    perm = ordering.nd_grid(DIMS)
    c = np.diff(cp) - 1
    kmax = int(np.searchsorted(np.cumsum(c + 2 * c * c), ORACLE_FLOPS))
    assert kmax > 1000
    announce("oracle: first %d pivots" % kmax)
    F = numeric.factor(n, big["rp"], big["ci"], big["v"], perm, cp, ri, kmax=kmax)
    cols = np.repeat(np.arange(n), np.diff(cp))
    fin = cols < kmax                      # L columns and U rows < kmax are final
    okl, nbl, rl = factor_close(big["lv"][fin], F.lval[fin])
    oku, nbu, ru = factor_close(big["uv"][fin & (ri > cols)], F.uval[fin & (ri > cols)])
    assert okl, "L / diag(U) differ: %d entries (max rel %.3e)" % (nbl, rl)
    assert oku, "U differs: %d entries (max rel %.3e)" % (nbu, ru)


def test_fullsize_symmetric_ldlt_relation(big):
    # symmetric A: U(k, r) = U(k, k) L(r, k) for every entry below the diagonal
    n, cp, ri, lv, uv = big["n"], big["cp"], big["ri"], big["lv"], big["uv"]
    cols = np.repeat(np.arange(n), np.diff(cp))
    low = ri.astype(np.int64) > cols
    d = lv[cp[:-1]]
    pred = d[cols[low]] * lv[low]
    ok, nb, rel = factor_close(uv[low], pred)
    assert ok, "U != diag(U) L^T at %d entries (max rel %.3e)" % (nb, rel)


def _csr(rowptr, colidx, vals, n):
    import scipy.sparse as sp
    return sp.csr_matrix((vals, colidx, rowptr), shape=(n, n))


def test_fullsize_sampled_residual(big):
    import scipy.sparse as sp
    n, cp, ri, lv, uv = big["n"], big["cp"], big["ri"], big["lv"], big["uv"]
    perm = ordering.nd_grid(DIMS)
    A = _csr(big["rp"], big["ci"], big["v"], n)
    Ap = A[perm][:, perm].tocsr()
    cols = np.repeat(np.arange(n), np.diff(cp))
    strict = ri.astype(np.int64) > cols
    # L (unit lower) by rows; U^T (lower, U's diagonal) by rows = U by columns
    Lc = sp.csc_matrix((np.where(strict, lv, 1.0), ri, cp), shape=(n, n)).tocsr()
    Ut = sp.csc_matrix((np.where(strict, uv, lv), ri, cp), shape=(n, n)).tocsr()
    rng = np.random.default_rng(7)
    q = rng.integers(0, len(ri), 4000)
    amax = float(np.max(np.abs(big["v"])))
    worst = 0.0
    for k in q:
        r, c = int(ri[k]), int(cols[k])
        for (i, j) in ((r, c), (c, r)):          # the entry and its mirror in U
            li, lvv = Lc.indices[Lc.indptr[i]:Lc.indptr[i + 1]], Lc.data[Lc.indptr[i]:Lc.indptr[i + 1]]
            uj, uvv = Ut.indices[Ut.indptr[j]:Ut.indptr[j + 1]], Ut.data[Ut.indptr[j]:Ut.indptr[j + 1]]
            common, ia, ib = np.intersect1d(li, uj, assume_unique=True, return_indices=True)
            s = float(np.dot(lvv[ia], uvv[ib]))
            sabs = float(np.dot(np.abs(lvv[ia]), np.abs(uvv[ib])))
            a = float(Ap[i, j])
            err = abs(s - a)
            bound = 1e-12 * sabs + 1e-14 * amax
            worst = max(worst, err / bound)
            assert err <= bound, "A' - LU at (%d, %d): %.3e > %.3e" % (i, j, err, bound)
    announce("sampled residual: worst err/bound %.3e" % worst)


def test_fullsize_solves(big):
    n, rp, ci, v = big["n"], big["rp"], big["ci"], big["v"]
    h = big["h"]
    xt = synth.random_x(n, 2, seed=0)
    b = synth.csr_matvec(n, rp, ci, v, xt)
    B = torch.from_numpy(np.ascontiguousarray(b)).cuda()
    x = h.solve(B).cpu().numpy()
    eta = metrics.backward_error(n, rp, ci, v, x, b)
    assert np.all(eta <= ETA_MAX), "eta %s" % eta
    xT = h.solve_transpose(B).cpu().numpy()
    etaT = metrics.backward_error(n, rp, ci, v, xT, b, transpose=True)
    assert np.all(etaT <= ETA_MAX), "eta^T %s" % etaT
    assert np.max(np.abs(x - xt)) < 1e-8


def test_fullsize_blocking_invariance(big):
    import paper_2512_04389_amd as slu
    n = big["n"]
    announce("regular b=500 at full size")
    hr = slu.SparseLU(n, big["rp"], big["ci"], ordering="grid_nd", grid_dims=DIMS, blocking="regular",
                      block_size=500).bind()
    hr.factor(big["vals"])
    lr, ur = hr.factors()
    hr.close()
    cols = np.repeat(np.arange(n), np.diff(big["cp"]))
    low = big["ri"].astype(np.int64) > cols
    okl, nbl, rl = factor_close(big["lv"], lr)
    oku, nbu, ru = factor_close(big["uv"][low], ur[low])
    assert okl and oku, "irregular vs regular: L %d (%.3e), U %d (%.3e)" % (nbl, rl, nbu, ru)



def test_convdiff64_sixteen_rhs_and_adjoint():
    """3D convection-diffusion 64^3 (n = 262,144, unsymmetric): factor, solve
    16 right-hand sides and back-propagate a loss through the solve; every
    result is checked on the host against A itself."""
    import time

    import paper_2512_04389_amd as slu
    k = 64
    n, rp, ci, v = synth.convection_diffusion_3d(k)
    announce("convdiff-64 full size: factor + 16 RHS + adjoint")
    lu = slu.SparseLU(n, rp, ci, ordering="grid_nd", grid_dims=(k, k, k)).bind()
    rng = np.random.default_rng(0)
    xt = synth.random_x(n, 16, seed=0)
    b = synth.csr_matvec(n, rp, ci, v, xt)
    W = rng.uniform(-1, 1, (n, 16))
    vals = torch.from_numpy(v).cuda().requires_grad_(True)
    B = torch.from_numpy(np.ascontiguousarray(b)).cuda().requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    X = slu.solve(lu, vals, B)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    (X * torch.from_numpy(W).cuda()).sum().backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    info = lu.info()
    announce("factor+solve %.1f ms, adjoint %.1f ms, F %.3g, levels %d" %
             ((t1 - t0) * 1e3, (t2 - t1) * 1e3, info["flops"], info["nblocks"]))
    x = X.detach().cpu().numpy()
    eta = metrics.backward_error(n, rp, ci, v, x, b)
    assert np.all(eta <= ETA_MAX), "eta %s" % eta
    g = B.grad.cpu().numpy()
    etag = metrics.backward_error(n, rp, ci, v, g, W, transpose=True)
    assert np.all(etag <= ETA_MAX), "adjoint eta %s" % etag
    rows = np.repeat(np.arange(n), np.diff(rp))
    gv_host = -np.sum(g[rows] * x[ci], axis=1)
    got = vals.grad.cpu().numpy()
    assert np.all(np.abs(got - gv_host) <= 1e-12 * (np.abs(gv_host) + np.max(np.abs(gv_host))))
    lu.close()
