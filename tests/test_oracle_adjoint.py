"""Pins of oracle.adjoint: a dense numpy gradient (np.linalg) and central
finite differences of the loss on small unsymmetric systems."""
import numpy as np

import synth
from oracle import adjoint, ordering


def _case(k=4, seed=3):
    n, rp, ci, v = synth.convection_diffusion_3d(k)
    rng = np.random.default_rng(seed)
    v = v * (1.0 + 0.05 * rng.uniform(-1, 1, v.shape))
    return n, rp, ci, v


def _dense(n, rp, ci, v):
    A = np.zeros((n, n))
    rows = np.repeat(np.arange(n), np.diff(rp))
    A[rows, ci] = v
    return A


def test_adjoint_matches_dense_gradient():
    n, rp, ci, v = _case()
    rng = np.random.default_rng(5)
    B = rng.uniform(-1, 1, (n, 2))
    W = rng.uniform(-1, 1, (n, 2))
    perm = ordering.nd_grid((4, 4, 4))
    X, G, gv = adjoint.solve_gradients(n, rp, ci, v, perm, B, W)
    A = _dense(n, rp, ci, v)
    Xd = np.linalg.solve(A, B)
    Gd = np.linalg.solve(A.T, W)
    full = -Gd @ Xd.T                       # d loss / d A for every entry
    rows = np.repeat(np.arange(n), np.diff(rp))
    assert np.allclose(X, Xd, rtol=1e-12, atol=1e-14)
    assert np.allclose(G, Gd, rtol=1e-12, atol=1e-14)
    assert np.allclose(gv, full[rows, ci], rtol=1e-10, atol=1e-14)


def test_adjoint_matches_finite_differences():
    n, rp, ci, v = _case(k=3, seed=8)
    rng = np.random.default_rng(2)
    b = rng.uniform(-1, 1, n)
    w = rng.uniform(-1, 1, n)
    perm = ordering.natural(n)
    _, g, gv = adjoint.solve_gradients(n, rp, ci, v, perm, b, w)
    A = _dense(n, rp, ci, v)

    def loss(vals, bb):
        Ad = A.copy()
        rows = np.repeat(np.arange(n), np.diff(rp))
        Ad[rows, ci] = vals
        return float(w @ np.linalg.solve(Ad, bb))

    for q in rng.choice(len(v), 12, replace=False):
        h = 1e-6 * max(1.0, abs(v[q]))
        vp, vm = v.copy(), v.copy()
        vp[q] += h
        vm[q] -= h
        fd = (loss(vp, b) - loss(vm, b)) / (2 * h)
        assert abs(fd - gv[q]) <= 1e-6 * max(1.0, abs(fd)), (q, fd, gv[q])
    for i in rng.choice(n, 6, replace=False):
        bp, bm = b.copy(), b.copy()
        bp[i] += 1e-6
        bm[i] -= 1e-6
        fd = (loss(v, bp) - loss(v, bm)) / 2e-6
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd))
