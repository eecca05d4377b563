"""Tiled diagonal solves (slu_set_solve_tiled): waves whose blocks were
factored by the 32 x 32 tiled GETRF solve their diagonal blocks tile by tile
with the kept inverted tiles.  Solutions and transpose solutions reach
backward error <= 1e-12 (host) and agree with the one-workgroup-per-block
solve to rounding; the refined FP32 solve and the allocation-free solve take
the same path."""
import numpy as np
import pytest

import synth
from gpu_common import ETA_MAX, announce
from oracle import metrics

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _dense_dd(n, seed):
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1, 1, (n, n))
    a[np.arange(n), np.arange(n)] = np.abs(a).sum(1) + 1.0
    rp = np.arange(0, n * n + 1, n, dtype=np.int64)
    ci = np.tile(np.arange(n, dtype=np.int32), n)
    return n, rp, ci, a.reshape(-1).copy()


CASES = {
    "dense-913": lambda: (_dense_dd(913, 3), dict(blocking="regular", block_size=913)),
    "bbd-6000-regular-700": lambda: (synth.bbd_circuit(n=6000, nblocks=4, border=300, border_nnz=20000, seed=9),
                                     dict(blocking="regular", block_size=700)),
    "bbd-6000-irregular": lambda: (synth.bbd_circuit(n=6000, nblocks=4, border=300, border_nnz=20000, seed=9), {}),
    # sparse 700-row blocks: tiled only when sparse blocks are allowed
    "convdiff-14-regular-700": lambda: (synth.convection_diffusion_3d(14),
                                        dict(ordering="grid_nd", grid_dims=(14, 14, 14), blocking="regular",
                                             block_size=700)),
    "convdiff-14-regular-300": lambda: (synth.convection_diffusion_3d(14),
                                        dict(ordering="grid_nd", grid_dims=(14, 14, 14), blocking="regular",
                                             block_size=300)),
}
# blocks of one to four 32-row tiles (tiles are solved in pairs: a single
# tile, one pair, a pair and a single last tile, two pairs), several blocks
# per wave, ragged last blocks
for _b, _k in ((20, 24), (40, 24), (70, 24), (100, 30)):
    CASES["lap2d-%d-regular-%d" % (_k, _b)] = (
        lambda b=_b, k=_k: (synth.laplacian_2d(k), dict(ordering="grid_nd", grid_dims=(k, k, 1), blocking="regular",
                                                        block_size=b)))


@pytest.mark.parametrize("case", sorted(CASES))
def test_tiled_solve_matches(case):
    import paper_2512_04389_amd as slu
    (n, rp, ci, v), opts = CASES[case]()
    announce("tiled solve %s n=%d" % (case, n))
    h = slu.SparseLU(n, rp, ci, **opts).bind()
    vals = torch.from_numpy(v).cuda()
    h.factor(vals)
    xt = synth.random_x(n, 17, seed=4)
    b = synth.csr_matvec(n, rp, ci, v, xt)
    B = torch.from_numpy(np.ascontiguousarray(b)).cuda()
    out = {}
    for rows in (1, 0):
        # rows = 1: every wave factored by the tiled GETRF, any density
        h.set_solve_tiled(rows, 1)
        for trans in (False, True):
            X = (h.solve_transpose(B) if trans else h.solve(B)).cpu().numpy()
            eta = metrics.backward_error(n, rp, ci, v, X, b, transpose=trans)
            assert np.all(eta <= ETA_MAX), (rows, trans, eta)
            out[(rows, trans)] = X
    for trans in (False, True):
        d = np.max(np.abs(out[(1, trans)] - out[(0, trans)])) / np.max(np.abs(out[(0, trans)]))
        assert d < 1e-10, (trans, d)
    h.set_solve_tiled(1, 1)
    Xn = h.solve_noalloc(B).cpu().numpy()
    np.testing.assert_array_equal(Xn, out[(1, False)])
    h.set_precision("fp32")
    h.factor(vals)
    Xr, its, eta_dev, conv = h.solve_refined(vals, B)
    eta = metrics.backward_error(n, rp, ci, v, Xr.cpu().numpy(), b)
    assert conv and np.all(eta <= ETA_MAX), eta
    assert slu.lib.slu_set_solve_tiled(h._h, -1, 640) == slu._abi.SLU_ERR_ARG
    assert slu.lib.slu_set_solve_tiled(h._h, 256, -1) == slu._abi.SLU_ERR_ARG
