"""Lookahead of the Schur updates (slu_set_lookahead): the updates of a wave
that reach only later waves run on a second stream.  Every target receives
its updates in the same order as without lookahead, so the factors must be
identical bit for bit, launch by launch and under graph replay, in FP64 and
FP32, for single systems and a batch; with lookahead (the default) they
match the oracle."""
import numpy as np
import pytest

import synth
from gpu_common import announce, check_factors, check_solves

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


CASES = {
    "bbd-6000": lambda: (synth.bbd_circuit(n=6000, nblocks=4, border=300, border_nnz=20000, seed=9), {}),
    "bbd-6000-regular-300": lambda: (synth.bbd_circuit(n=6000, nblocks=4, border=300, border_nnz=20000, seed=9),
                                     dict(blocking="regular", block_size=300)),
    "convdiff-16-grid-nd": lambda: (synth.convection_diffusion_3d(16),
                                    dict(ordering="grid_nd", grid_dims=(16, 16, 16))),
    "lap2d-60-levels": lambda: (synth.laplacian_2d(60), dict(ordering="grid_nd", grid_dims=(60, 60),
                                                             schedule="levels")),
}


def _factors(h, vals):
    h.factor(vals)
    return h.factors()


@pytest.mark.parametrize("case", sorted(CASES))
def test_lookahead_bit_identical(case):
    import paper_2512_04389_amd as slu
    (n, rp, ci, v), opts = CASES[case]()
    announce("lookahead %s n=%d" % (case, n))
    h = slu.SparseLU(n, rp, ci, **opts).bind()
    vals = torch.from_numpy(np.ascontiguousarray(v, dtype=np.float64)).cuda()
    h.set_lookahead(True)
    l1, u1 = _factors(h, vals)
    check_factors(h, n, rp, ci, v, opts)
    check_solves(h, n, rp, ci, v, vals, nrhs=2)
    h.set_lookahead(False)
    l0, u0 = _factors(h, vals)
    np.testing.assert_array_equal(l1, l0)
    np.testing.assert_array_equal(u1, u0)
    # repeated: a race between the two streams would show as a changing result
    h.set_lookahead(True)
    for _ in range(4):
        l1, u1 = _factors(h, vals)
        np.testing.assert_array_equal(l1, l0)
        np.testing.assert_array_equal(u1, u0)
    # deferred launches of 8 workgroups (walking their tiles) and uncapped ones
    for groups in (8, 0):
        h.set_lookahead(True, groups)
        l1, u1 = _factors(h, vals)
        np.testing.assert_array_equal(l1, l0)
        np.testing.assert_array_equal(u1, u0)
    h.set_lookahead(True)
    # graph replay holds both streams' launches
    h.set_lookahead(True)
    h.set_graph(True)
    for _ in range(3):
        l2, u2 = _factors(h, vals)
        np.testing.assert_array_equal(l2, l0)
        np.testing.assert_array_equal(u2, u0)
    h.set_graph(False)
    # FP32 Schur updates: the same split, the same bits either way
    h.set_precision("fp32")
    h.set_lookahead(False)
    l4, u4 = _factors(h, vals)
    h.set_lookahead(True)
    for _ in range(3):
        l3, u3 = _factors(h, vals)
        np.testing.assert_array_equal(l3, l4)
        np.testing.assert_array_equal(u3, u4)
    assert slu.lib.slu_set_lookahead(h._h, 2, 256) == slu._abi.SLU_ERR_ARG
    assert slu.lib.slu_set_lookahead(h._h, 1, 100) == slu._abi.SLU_ERR_ARG
    assert slu.lib.slu_set_lookahead(h._h, 1, -8) == slu._abi.SLU_ERR_ARG


def test_lookahead_batch_bit_identical():
    import paper_2512_04389_amd as slu
    sy = [synth.laplacian_3d(12), synth.convection_diffusion_3d(10),
          synth.bbd_circuit(n=3000, nblocks=3, border=150, border_nnz=6000, seed=4)]
    announce("lookahead batch of %d systems" % len(sy))
    h = slu.SparseLU.batch([(x[0], x[1], x[2]) for x in sy]).bind()
    v = np.concatenate([x[3] for x in sy])
    vals = torch.from_numpy(np.ascontiguousarray(v, dtype=np.float64)).cuda()
    h.set_lookahead(False)
    l0, u0 = _factors(h, vals)
    h.set_lookahead(True)
    for _ in range(4):
        l1, u1 = _factors(h, vals)
        np.testing.assert_array_equal(l1, l0)
        np.testing.assert_array_equal(u1, u0)
    # every system solved to FP64 backward error with the lookahead factors
    h.set_lookahead(True)
    h.factor(vals)
    b = np.concatenate([synth.csr_matvec(x[0], x[1], x[2], x[3], synth.random_x(x[0], 1, seed=k))
                        for k, x in enumerate(sy)])
    B = torch.from_numpy(np.ascontiguousarray(b)).cuda()
    X = h.solve(B)
    eta = h.backward_error(vals, B, X)
    assert np.all(eta <= 1e-12), eta
