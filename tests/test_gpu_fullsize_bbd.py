"""Parity at full size on the bordered block-diagonal circuit-like matrix
(n = 200,000; 64 systems of 3,094 / 3,093 rows, a 2,000-row border), natural
order, irregular blocking, in the launch configuration the benchmark times.

The oracle cannot factor the whole matrix in seconds; what it can do exactly:

* the pivots of one system depend only on that system and the border (no
  entry of S couples two systems, the border comes last), so the oracle's
  right-looking LU of the submatrix (system j + border), stopped after its
  first kmax pivots, fixes L's columns and U's rows of those pivots; they are
  compared entry by entry with the library's for the first system and a
  middle one (row sets identical, values within the 1e-10 tolerance);
* solves and transpose solves with 8 right-hand sides reach backward error
  <= 1e-12, recomputed on the host from the original A;
* FP32 factorization + FP64 refinement reaches the same 1e-12 on the same
  right-hand sides, with its factor error against FP64 stated;
* regular blocking (b = 500) and the one-launch / split chunked GETRF give
  the same factors as the default to the parity tolerance.
(The pattern, block pointer and block boundaries are compared bit for bit
with the oracle on the host by tests/test_analyze_fullsize.py.)"""
import numpy as np
import pytest

import synth
from gpu_common import ETA_MAX, announce, factor_close
from oracle import metrics, numeric, ordering, symbolic

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

NSYS, BORDER = 64, 2000
ORACLE_FLOPS = 1.2e10     # per system checked (about 10 s of the oracle)


@pytest.fixture(scope="module")
def big():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2512_04389_amd as slu
    n, rp, ci, v = synth.bbd_circuit()
    announce("bbd200k full size: analyze + factor (natural order, irregular, default GETRF)")
    h = slu.SparseLU(n, rp, ci).bind()
    vals = torch.from_numpy(v).cuda()
    h.factor(vals)
    lv, uv = h.factors()
    cp, ri = h.pattern()
    yield dict(h=h, n=n, rp=rp, ci=ci, v=v, vals=vals, lv=lv, uv=uv, cp=cp, ri=ri)
    h.close()


def _system_range(j, n):
    inner = n - BORDER
    sizes = [inner // NSYS + (1 if q < inner % NSYS else 0) for q in range(NSYS)]
    s0 = int(np.sum(sizes[:j]))
    return s0, s0 + sizes[j]


@pytest.mark.parametrize("j", [0, 37])
def test_bbd_system_pivots_match_oracle(big, j):
    import scipy.sparse as sp
    n, rp, ci, v = big["n"], big["rp"], big["ci"], big["v"]
    s0, s1 = _system_range(j, n)
    glob = np.concatenate([np.arange(s0, s1), np.arange(n - BORDER, n)])   # sub index -> global
    A = sp.csr_matrix((v, ci, rp), shape=(n, n))
    sub = A[glob][:, glob].tocsr()
    sub.sort_indices()
    ns = glob.shape[0]
    srp, sci, sv = sub.indptr.astype(np.int64), sub.indices.astype(np.int32), sub.data.astype(np.float64)
    perm = ordering.natural(ns)
    scp, sri = symbolic.symbolic(ns, srp, sci, perm)
    c = np.diff(scp) - 1
    kmax = int(np.searchsorted(np.cumsum(c + 2 * c * c), ORACLE_FLOPS))
    kmax = min(kmax, s1 - s0)
    assert kmax >= 100
    announce("oracle: system %d + border (n=%d), first %d pivots" % (j, ns, kmax))
    F = numeric.factor(ns, srp, sci, sv, perm, scp, sri, kmax=kmax)
    cp, ri, lv, uv = big["cp"], big["ri"], big["lv"], big["uv"]
    got_l, got_u, ref_l, ref_u = [], [], [], []
    for k in range(kmax):
        kg = s0 + k
        rows_ref = glob[sri[scp[k]:scp[k + 1]]]
        lo, hi = cp[kg], cp[kg + 1]
        assert np.array_equal(ri[lo:hi], rows_ref), "column %d: row sets differ" % kg
        got_l.append(lv[lo:hi])
        got_u.append(uv[lo + 1:hi])
        ref_l.append(F.lval[scp[k]:scp[k + 1]])
        ref_u.append(F.uval[scp[k] + 1:scp[k + 1]])
    okl, nbl, rl = factor_close(np.concatenate(got_l), np.concatenate(ref_l))
    oku, nbu, ru = factor_close(np.concatenate(got_u), np.concatenate(ref_u))
    announce("system %d: max rel L %.2e, U %.2e" % (j, rl, ru))
    assert okl, "L / diag(U) differ: %d entries (max rel %.3e)" % (nbl, rl)
    assert oku, "U differs: %d entries (max rel %.3e)" % (nbu, ru)


def _rhs(big, nrhs=8):
    xt = synth.random_x(big["n"], nrhs, seed=1)
    b = synth.csr_matvec(big["n"], big["rp"], big["ci"], big["v"], xt)
    return b, torch.from_numpy(np.ascontiguousarray(b)).cuda()


def test_bbd_solves_8_rhs(big):
    h = big["h"]
    b, B = _rhs(big)
    for trans in (False, True):
        X = (h.solve_transpose(B) if trans else h.solve(B)).cpu().numpy()
        eta = metrics.backward_error(big["n"], big["rp"], big["ci"], big["v"], X, b, transpose=trans)
        announce("solve%s: eta max %.2e" % (" (transpose)" if trans else "", float(np.max(eta))))
        assert np.all(eta <= ETA_MAX), eta


def test_bbd_fp32_refined_8_rhs(big):
    h = big["h"]
    b, B = _rhs(big)
    h.set_precision("fp32")
    try:
        h.factor(big["vals"])
        lv32, _ = h.factors()
        X, its, eta_dev, conv = h.solve_refined(big["vals"], B)
    finally:
        h.set_precision("fp64")
        h.factor(big["vals"])
    lv = big["lv"]
    sig = np.abs(lv) > 1e-6 * np.max(np.abs(lv))
    fdiff = float(np.max(np.abs(lv32[sig] - lv[sig]) / np.abs(lv[sig])))
    eta = metrics.backward_error(big["n"], big["rp"], big["ci"], big["v"], X.cpu().numpy(), b)
    announce("fp32 + refinement: %d corrections, eta max %.2e, factor rel diff vs fp64 %.2e"
             % (its, float(np.max(eta)), fdiff))
    assert conv and np.all(eta <= ETA_MAX), eta
    assert fdiff < 1e-3


def test_bbd_regular_blocking_same_factors(big):
    import paper_2512_04389_amd as slu
    announce("bbd200k regular blocking b=500")
    hr = slu.SparseLU(big["n"], big["rp"], big["ci"], blocking="regular", block_size=500).bind()
    hr.factor(big["vals"])
    lr, ur = hr.factors()
    hr.close()
    ok, nb, rel = factor_close(lr, big["lv"])
    assert ok, "regular vs irregular L: %d entries (max rel %.3e)" % (nb, rel)
    ok, nb, rel = factor_close(ur, big["uv"])
    assert ok, "regular vs irregular U: %d entries (max rel %.3e)" % (nb, rel)


def test_bbd_chunked_getrf_same_factors(big):
    h = big["h"]
    announce("bbd200k chunked (split) GETRF")
    h.set_getrf_tiled(0)
    try:
        h.factor(big["vals"])
        lc, uc = h.factors()
    finally:
        h.set_getrf_tiled(1)
        h.factor(big["vals"])
    ok, nb, rel = factor_close(lc, big["lv"])
    assert ok, "chunked vs tiled GETRF L: %d entries (max rel %.3e)" % (nb, rel)
    ok, nb, rel = factor_close(uc, big["uv"])
    assert ok, "chunked vs tiled GETRF U: %d entries (max rel %.3e)" % (nb, rel)
