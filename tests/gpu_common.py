"""Shared helpers of the GPU parity tests: run a case through the C ABI and
compare with the oracle computed independently on the host."""
import sys

import numpy as np

import synth
from oracle import metrics, numeric, ordering, symbolic

# FP64 factor parity: |f - f*| <= RTOL * (|f*| + FLOOR * max|F*|), per factor
RTOL = 1e-10
FLOOR = 1e-8
ETA_MAX = 1e-12


def announce(msg):
    print("[gpu case] " + msg, flush=True)
    sys.stdout.flush()


def oracle_perm(n, kw, h=None):
    o = kw.get("ordering", "natural")
    if o == "grid_nd":
        return ordering.nd_grid(kw["grid_dims"])
    if o == "user":
        return np.asarray(kw["perm"], dtype=np.int32)
    if o == "graph_nd":
        # the library's graph nested dissection: the oracle consumes the order
        perm = h.perm()
        assert ordering.is_permutation(perm, n)
        return perm
    return ordering.natural(n)


def factor_close(got, ref):
    scale = float(np.max(np.abs(ref))) if ref.size else 0.0
    err = np.abs(got - ref)
    bound = RTOL * (np.abs(ref) + FLOOR * scale)
    bad = err > bound
    rel = float(np.max(err / np.maximum(np.abs(ref), 1e-300))) if ref.size else 0.0
    return (not bad.any()), int(bad.sum()), rel


def check_factors(h, n, rp, ci, v, kw, oracle_factors=None):
    perm = oracle_perm(n, kw, h)
    cp, ri = symbolic.symbolic(n, rp, ci, perm)
    hcp, hri = h.pattern()
    assert np.array_equal(hcp, cp) and np.array_equal(hri, ri), "pattern differs from oracle"
    F = oracle_factors or numeric.factor(n, rp, ci, v, perm, cp, ri)
    lv, uv = h.factors()
    cols = np.repeat(np.arange(n), np.diff(cp))
    low = ri.astype(np.int64) > cols
    okl, nbl, rl = factor_close(lv[low], F.lval[low])
    oku, nbu, ru = factor_close(np.concatenate([uv[low], lv[~low]]), np.concatenate([F.uval[low], F.lval[~low]]))
    assert okl, "L differs: %d entries beyond tolerance (max rel %.3e)" % (nbl, rl)
    assert oku, "U differs: %d entries beyond tolerance (max rel %.3e)" % (nbu, ru)
    return F


def check_solves(h, n, rp, ci, v, values_dev, nrhs=1, seed=1):
    import torch
    xt = synth.random_x(n, nrhs, seed=seed)
    b = synth.csr_matvec(n, rp, ci, v, xt)
    B = torch.from_numpy(np.ascontiguousarray(b)).cuda()
    X = h.solve(B)
    x = X.cpu().numpy()
    eta = metrics.backward_error(n, rp, ci, v, x, b)
    assert np.all(eta <= ETA_MAX), "eta %s" % eta
    eta_dev = h.backward_error(values_dev, B, X)
    assert np.all(eta_dev <= ETA_MAX)
    # both are residuals at roundoff level, summed in different orders: they
    # agree in magnitude, not digit for digit
    assert np.allclose(eta_dev, eta, rtol=0.5, atol=1e-15), "eta device %s host %s" % (eta_dev, eta)
    # transpose
    Xt = h.solve_transpose(B)
    xt_ = Xt.cpu().numpy()
    eta_t = metrics.backward_error(n, rp, ci, v, xt_, b, transpose=True)
    assert np.all(eta_t <= ETA_MAX), "eta^T %s" % eta_t
    eta_t_dev = h.backward_error(values_dev, B, Xt, transpose=True)
    assert np.all(eta_t_dev <= ETA_MAX)
    return eta, eta_t


def run_case(name, n, rp, ci, v, nrhs=1, factors=True, **kw):
    import torch
    import paper_2512_04389_amd as slu
    announce("%s n=%d nnz=%d %s" % (name, n, len(ci), kw))
    h = slu.SparseLU(n, rp, ci, **kw).bind()
    vals = torch.from_numpy(np.ascontiguousarray(v, dtype=np.float64)).cuda()
    h.factor(vals)
    torch.cuda.synchronize()
    if factors:
        check_factors(h, n, rp, ci, v, kw)
    check_solves(h, n, rp, ci, v, vals, nrhs=nrhs)
    return h, vals
