"""Batched factorization of independent systems (slu_analyze_batch): every
system's factors against its own oracle, host backward errors of the stacked
solve, shared launches; and the graph mode (capture once, replay) against
the launch-by-launch factorization, replay after replay."""
import numpy as np
import pytest

import synth
from gpu_common import ETA_MAX, announce, factor_close
from oracle import metrics, numeric, ordering, symbolic

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SEEDS = (11, 14, 23, 27, 221, 255)     # 2D and 3D members with n <= 9000


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _systems():
    out = []
    for s in SEEDS:
        n, rp, ci, v, dims = synth.batch_system(s)
        if n <= 9000:
            out.append((n, rp, ci, v, dims))
    return out


def test_batch_factors_and_solves():
    import paper_2512_04389_amd as slu
    sy = _systems()
    assert len(sy) >= 4
    announce("batch of %d systems, n = %s" % (len(sy), [x[0] for x in sy]))
    h = slu.SparseLU.batch([(x[0], x[1], x[2]) for x in sy], ordering="grid_nd",
                           grid_dims=[x[4] for x in sy]).bind()
    vals = torch.from_numpy(np.concatenate([x[3] for x in sy])).cuda()
    h.factor(vals)
    info = h.info()
    singles = [slu.SparseLU(x[0], x[1], x[2], ordering="grid_nd", grid_dims=x[4]).info() for x in sy]
    # levels of different systems share launches
    assert info["waves"] <= max(s["waves"] for s in singles)
    assert info["nblocks"] == sum(s["nblocks"] for s in singles)
    lv, uv = h.factors()
    cp, ri = h.pattern()
    xs = [synth.random_x(x[0], 2, seed=k) for k, x in enumerate(sy)]
    B = np.concatenate([synth.csr_matvec(x[0], x[1], x[2], x[3], xx) for x, xx in zip(sy, xs)])
    X = h.solve(torch.from_numpy(np.ascontiguousarray(B)).cuda()).cpu().numpy()
    off = 0
    for (n, rp, ci, v, dims) in sy:
        perm = ordering.nd_grid(dims)
        cp1, ri1 = symbolic.symbolic(n, rp, ci, perm)
        F = numeric.factor(n, rp, ci, v, perm, cp1, ri1)
        q0, q1 = cp[off], cp[off + n]
        cols = np.repeat(np.arange(n), np.diff(cp1))
        low = ri1.astype(np.int64) > cols
        okl, nbl, rl = factor_close(lv[q0:q1], F.lval)
        oku, nbu, ru = factor_close(uv[q0:q1][low], F.uval[low])
        assert okl and oku, "system n=%d: L %d (%.2e), U %d (%.2e)" % (n, nbl, rl, nbu, ru)
        eta = metrics.backward_error(n, rp, ci, v, X[off:off + n], B[off:off + n])
        assert np.all(eta <= ETA_MAX)
        off += n


def test_graph_replays_match_launch_by_launch():
    import paper_2512_04389_amd as slu
    n, rp, ci, v = synth.convection_diffusion_3d(16)
    kw = dict(ordering="grid_nd", grid_dims=(16, 16, 16))
    eager = slu.SparseLU(n, rp, ci, **kw).bind()
    graph = slu.SparseLU(n, rp, ci, **kw).bind()
    graph.set_graph(True)
    rng = np.random.default_rng(3)
    b = torch.from_numpy(rng.uniform(-1, 1, n)).cuda()
    for rep in range(4):
        vv = torch.from_numpy(v * (1.0 + 0.1 * rep)).cuda()
        announce("graph replay %d" % rep)
        eager.factor(vv)
        le, ue = eager.factors()
        graph.factor(vv)
        lg, ug = graph.factors()
        assert np.array_equal(le, lg) and np.array_equal(ue, ug), "replay %d differs" % rep
        # the program's own eager work between the replays
        x = graph.solve(b)
        torch.cuda.synchronize()
        assert float(graph.backward_error(vv, b, x)[0]) <= ETA_MAX
    # fp32 mode recaptures
    eager.set_precision("fp32")
    graph.set_precision("fp32")
    eager.factor(vv)
    graph.factor(vv)
    assert np.array_equal(eager.factors()[0], graph.factors()[0])
