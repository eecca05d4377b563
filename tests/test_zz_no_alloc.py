"""slu_solve_noalloc: the solve with its work block in the library's fixed
device scratch instead of the workspace.  Its results must equal slu_solve's
(same kernels, same arithmetic: bit for bit) and meet the parity bar against
the oracle, on two calls in a row, the second with a smaller system; sizes
beyond the fixed scratch are rejected before any device call."""
import ctypes

import numpy as np
import pytest

import synth
from gpu_common import ETA_MAX, announce
from oracle import metrics

torch = pytest.importorskip("torch")
slu = pytest.importorskip("paper_2512_04389_amd")


def test_noalloc_rejects_beyond_fixed_scratch():
    # n = 4 Mi + 1 rows: one column of the work block no longer fits; the
    # size check comes before any device call (no GPU needed)
    n = (4 << 20) + 1
    h = slu.SparseLU(n, np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32),
                     blocking="regular", block_size=64)
    fake = ctypes.c_void_p(256)
    assert slu.lib.slu_solve_noalloc(h._h, fake, fake, 1, n, 0, None) == slu._abi.SLU_ERR_LIMIT
    assert slu.lib.slu_solve_noalloc(h._h, fake, fake, 1, n, 2, None) == slu._abi.SLU_ERR_ARG
    h.close()


def _case(name, n, rp, ci, v, nrhs, **kw):
    announce("noalloc solve %s n=%d nrhs=%d" % (name, n, nrhs))
    h = slu.SparseLU(n, rp, ci, **kw).bind()
    vals = torch.from_numpy(v).cuda()
    h.factor(vals)
    xt = synth.random_x(n, nrhs, seed=7)
    b = synth.csr_matvec(n, rp, ci, v, xt)
    B = torch.from_numpy(np.ascontiguousarray(b)).cuda()
    for trans in (False, True):
        ref = (h.solve_transpose(B) if trans else h.solve(B)).cpu().numpy()
        got = h.solve_noalloc(B, transpose=trans).cpu().numpy()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(got, ref)
        eta = metrics.backward_error(n, rp, ci, v, got, b, transpose=trans)
        assert np.all(eta <= ETA_MAX), "eta %s" % eta
    h.close()


@pytest.mark.gpu
def test_noalloc_matches_solve_twice():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    n, rp, ci, v = synth.laplacian_3d(12)
    _case("lap3d-12", n, rp, ci, v, 20, ordering="grid_nd", grid_dims=(12, 12, 12))
    n, rp, ci, v = synth.convection_diffusion_3d(6)
    _case("convdiff-6", n, rp, ci, v, 3, ordering="grid_nd", grid_dims=(6, 6, 6))
