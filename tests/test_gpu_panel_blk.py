"""The blocked panel solve (slu_set_panel_blocked): levels whose coupled
triangles have at least 256 columns solve their panels in 128-column blocks
with inverted diagonal blocks.  Factors must match the oracle (1e-10) and the
tile-by-tile solve, on wide dense triangles with ragged last blocks."""
import numpy as np
import pytest

import synth
from gpu_common import announce, check_factors, check_solves, factor_close

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
    "dense-900-regular-600": lambda: (_dense_dd(900, 5), dict(blocking="regular", block_size=600)),
    "dense-1100-regular-300": lambda: (_dense_dd(1100, 6), dict(blocking="regular", block_size=300)),
    # panel rows above 2000 in the first levels
    "dense-2600-regular-300": lambda: (_dense_dd(2600, 7), dict(blocking="regular", block_size=300)),
    "bbd-6000-regular-700": lambda: (synth.bbd_circuit(n=6000, nblocks=4, border=300, border_nnz=20000, seed=9),
                                     dict(blocking="regular", block_size=700)),
    "convdiff-16-regular-800": lambda: (synth.convection_diffusion_3d(16),
                                        dict(ordering="grid_nd", grid_dims=(16, 16, 16), blocking="regular",
                                             block_size=800)),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_blocked_panels_match_oracle_and_tilewise(case):
    import paper_2512_04389_amd as slu
    (n, rp, ci, v), opts = CASES[case]()
    announce("blocked panels %s n=%d" % (case, n))
    h = slu.SparseLU(n, rp, ci, **opts).bind()
    vals = torch.from_numpy(v).cuda()
    h.factor(vals)
    check_factors(h, n, rp, ci, v, opts)
    check_solves(h, n, rp, ci, v, vals, nrhs=2)
    lb, ub = h.factors()
    h.set_panel_blocked(False)
    h.factor(vals)
    lt, ut = h.factors()
    ok, nb, rel = factor_close(lb, lt)
    assert ok, "blocked vs tile-wise L: %d entries (max rel %.3e)" % (nb, rel)
    ok, nb, rel = factor_close(ub, ut)
    assert ok, "blocked vs tile-wise U: %d entries (max rel %.3e)" % (nb, rel)
    h.set_panel_blocked(True)
    h.set_graph(True)
    for _ in range(2):
        h.factor(vals)
        l2, u2 = h.factors()
        np.testing.assert_array_equal(l2, lb)
        np.testing.assert_array_equal(u2, ub)
    h.set_graph(False)
    assert slu.lib.slu_set_panel_blocked(h._h, 2) == slu._abi.SLU_ERR_ARG
