"""FP32 factorization (Schur updates in FP32 on the matrix cores) won back by
FP64 iterative refinement: every case states the factor error against the
FP64 oracle and must reach a backward error <= 1e-12."""
import numpy as np
import pytest

import synth
from gpu_common import ETA_MAX, announce, oracle_perm
from oracle import metrics, numeric, symbolic

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _cases():
    return [
        ("lap3d-12", synth.laplacian_3d(12), dict(ordering="grid_nd", grid_dims=(12, 12, 12))),
        ("convdiff-16", synth.convection_diffusion_3d(16), dict(ordering="grid_nd", grid_dims=(16, 16, 16))),
        ("convdiff-14-regular-700", synth.convection_diffusion_3d(14),
         dict(ordering="grid_nd", grid_dims=(14, 14, 14), blocking="regular", block_size=700)),
        ("bbd-2400", synth.bbd_circuit(n=2400, nblocks=8, border=80, border_nnz=2000, seed=4), {}),
    ]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c[0])
def test_fp32_factor_with_refinement(case):
    import paper_2512_04389_amd as slu
    name, (n, rp, ci, v), kw = case
    h = slu.SparseLU(n, rp, ci, **kw).bind()
    vals = torch.from_numpy(v).cuda()
    h.set_precision("fp32")
    assert h.info()["precision"] == 1
    h.factor(vals)
    # factor error against the FP64 oracle
    perm = oracle_perm(n, kw)
    cp, ri = symbolic.symbolic(n, rp, ci, perm)
    F = numeric.factor(n, rp, ci, v, perm, cp, ri)
    lv, uv = h.factors()
    cols = np.repeat(np.arange(n), np.diff(cp))
    low = ri.astype(np.int64) > cols
    got = np.concatenate([lv, uv[low]])
    ref = np.concatenate([F.lval, F.uval[low]])
    big = np.abs(ref) > 1e-6 * np.max(np.abs(ref))
    rel = float(np.max(np.abs(got[big] - ref[big]) / np.abs(ref[big])))
    xt = synth.random_x(n, 8, seed=2)
    b = synth.csr_matvec(n, rp, ci, v, xt)
    B = torch.from_numpy(np.ascontiguousarray(b)).cuda()
    x1 = h.solve(B).cpu().numpy()
    eta1 = float(np.max(metrics.backward_error(n, rp, ci, v, x1, b)))
    X, iters, eta, ok = h.solve_refined(vals, B, tol=ETA_MAX, maxit=10)
    x = X.cpu().numpy()
    eta_host = metrics.backward_error(n, rp, ci, v, x, b)
    announce("[fp32] %s: max rel factor error vs FP64 oracle %.2e; one solve eta %.2e; refinement %d "
             "corrections, eta %.2e" % (name, rel, eta1, iters, float(np.max(eta_host))))
    assert rel < 1e-3, "FP32 factor error %.3e" % rel
    assert ok and np.all(eta <= ETA_MAX) and np.all(eta_host <= ETA_MAX)
    assert 1 <= iters <= 10
    # the FP64 mode needs no correction
    h.set_precision("fp64")
    h.factor(vals)
    X, iters, eta, ok = h.solve_refined(vals, B, tol=ETA_MAX, maxit=10)
    assert ok and iters == 0


def test_refinement_argument_checks():
    import paper_2512_04389_amd as slu
    n, rp, ci, v = synth.laplacian_2d(8)
    h = slu.SparseLU(n, rp, ci).bind()
    vals = torch.from_numpy(v).cuda()
    B = torch.ones(n, dtype=torch.float64, device="cuda")
    with pytest.raises(slu.SluError):
        h.solve_refined(vals, B)                 # not factored yet
    with pytest.raises(slu.SluError):
        slu._abi.check(slu.lib.slu_set_precision(h._h, 7), "slu_set_precision")
    with pytest.raises(KeyError):
        h.set_precision("fp16")
