"""The autotuner (slu_autotune): it times every launch-shape setting it
knows on the handle's values, reports them, keeps the fastest, and leaves
the handle factored with it: the factors then match the oracle and the
solves reach backward error <= 1e-12, for a single system and a batch."""
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


def test_autotune_single_system():
    import paper_2512_04389_amd as slu
    n, rp, ci, v = synth.bbd_circuit(n=6000, nblocks=4, border=300, border_nnz=20000, seed=9)
    announce("autotune bbd-6000")
    h = slu.SparseLU(n, rp, ci).bind()
    vals = torch.from_numpy(v).cuda()
    table = h.autotune(vals, reps=2)
    assert len(table) == 9
    assert {r["lookahead"] for r in table} == {0, 1}
    assert all(r["ms"] > 0 for r in table)
    assert table[0]["ms"] == min(r["ms"] for r in table)
    assert h.info()["factored"] == 1
    check_factors(h, n, rp, ci, v, {})
    check_solves(h, n, rp, ci, v, vals, nrhs=3)
    h.factor(vals)                       # later factors keep the chosen setting
    check_factors(h, n, rp, ci, v, {})
    assert slu.lib.slu_autotune(h._h, slu._dptr(vals), 0, None, 0, None, slu._stream(None)) == slu._abi.SLU_ERR_ARG


def test_autotune_batch():
    import paper_2512_04389_amd as slu
    from oracle import metrics
    sy = [synth.batch_system(s) for s in (3, 140, 200)]
    announce("autotune batch of 3")
    h = slu.SparseLU.batch([(x[0], x[1], x[2]) for x in sy], ordering="grid_nd", grid_dims=[x[4] for x in sy]).bind()
    vals = torch.from_numpy(np.concatenate([x[3] for x in sy])).cuda()
    table = h.autotune(vals, reps=1)
    assert len(table) == 9
    xs = [synth.random_x(x[0], 1, seed=q) for q, x in enumerate(sy)]
    b = np.concatenate([synth.csr_matvec(x[0], x[1], x[2], x[3], xx) for x, xx in zip(sy, xs)])
    X = h.solve(torch.from_numpy(np.ascontiguousarray(b)).cuda()).cpu().numpy()
    off = 0
    for (n, rp, ci, v, _) in sy:
        eta = metrics.backward_error(n, rp, ci, v, X[off:off + n], b[off:off + n])
        assert np.all(eta <= 1e-12), eta
        off += n
