"""The full 256-system batch (2D 5-point and 3D 7-point grids, n 2k-20k,
perturbed unsymmetric values) in one handle, in the configuration the
benchmark times: every system's solve reaches backward error <= 1e-12
(recomputed per system on the host), in FP64 and after FP32 factorization +
FP64 refinement; a seeded sample of systems, including the three largest 3D
ones, has its factors compared entry by entry with its own oracle; graph
replay gives the launch-by-launch factors bit for bit."""
import numpy as np
import pytest

import synth
from gpu_common import ETA_MAX, announce, factor_close
from oracle import metrics, numeric, ordering, symbolic

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

NSYS = 256


@pytest.fixture(scope="module")
def batch():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2512_04389_amd as slu
    sy = [synth.batch_system(s) for s in range(NSYS)]
    announce("batch of %d systems: analyze + factor" % NSYS)
    h = slu.SparseLU.batch([(x[0], x[1], x[2]) for x in sy], ordering="grid_nd", grid_dims=[x[4] for x in sy]).bind()
    vals = torch.from_numpy(np.concatenate([x[3] for x in sy])).cuda()
    h.factor(vals)
    offs = np.concatenate([[0], np.cumsum([x[0] for x in sy])]).astype(np.int64)
    xs = [synth.random_x(x[0], 2, seed=100 + q) for q, x in enumerate(sy)]
    b = np.concatenate([synth.csr_matvec(x[0], x[1], x[2], x[3], xx) for x, xx in zip(sy, xs)])
    yield dict(h=h, sy=sy, vals=vals, offs=offs, b=b, B=torch.from_numpy(np.ascontiguousarray(b)).cuda())
    h.close()


def _per_system_eta(batch, X):
    worst = 0.0
    for q, (n, rp, ci, v, _) in enumerate(batch["sy"]):
        o0, o1 = batch["offs"][q], batch["offs"][q + 1]
        eta = metrics.backward_error(n, rp, ci, v, X[o0:o1], batch["b"][o0:o1])
        assert np.all(eta <= ETA_MAX), "system %d: eta %s" % (q, eta)
        worst = max(worst, float(np.max(eta)))
    return worst


def test_batch256_every_system_solves(batch):
    X = batch["h"].solve(batch["B"]).cpu().numpy()
    announce("fp64: worst eta over %d systems %.2e" % (NSYS, _per_system_eta(batch, X)))


def test_batch256_sampled_systems_match_oracle(batch):
    sy, offs = batch["sy"], batch["offs"]
    h = batch["h"]
    lv, uv = h.factors()
    cp, ri = h.pattern()
    three_d = sorted(range(128, NSYS), key=lambda q: -sy[q][0])[:3]
    rng = np.random.default_rng(2024)
    others = [int(q) for q in rng.choice([q for q in range(NSYS) if q not in three_d], 6, replace=False)]
    for q in three_d + others:
        n, rp, ci, v, dims = sy[q]
        o = int(offs[q])
        perm = ordering.nd_grid(dims)
        cpq, riq = symbolic.symbolic(n, rp, ci, perm)
        e0, e1 = cp[o], cp[o + n]
        assert np.array_equal(cp[o:o + n + 1] - e0, cpq)
        assert np.array_equal(ri[e0:e1] - o, riq)
        F = numeric.factor(n, rp, ci, v, perm, cpq, riq)
        okl, nbl, rl = factor_close(lv[e0:e1], F.lval)
        cols = np.repeat(np.arange(n), np.diff(cpq))
        low = riq.astype(np.int64) > cols
        oku, nbu, ru = factor_close(uv[e0:e1][low], F.uval[low])
        announce("system %d (n=%d, %s): max rel L %.2e U %.2e" % (q, n, dims, rl, ru))
        assert okl and oku, "system %d: %d / %d entries beyond tolerance" % (q, nbl, nbu)


def test_batch256_graph_replay_and_fp32(batch):
    h = batch["h"]
    l0, u0 = h.factors()
    h.set_graph(True)
    try:
        for _ in range(2):
            h.factor(batch["vals"])
            l1, u1 = h.factors()
            np.testing.assert_array_equal(l1, l0)
            np.testing.assert_array_equal(u1, u0)
    finally:
        h.set_graph(False)
    h.set_precision("fp32")
    try:
        h.factor(batch["vals"])
        X, its, eta_dev, conv = h.solve_refined(batch["vals"], batch["B"])
    finally:
        h.set_precision("fp64")
        h.factor(batch["vals"])
    assert conv
    worst = _per_system_eta(batch, X.cpu().numpy())
    announce("fp32 + refinement: %d corrections, worst eta %.2e" % (its, worst))
