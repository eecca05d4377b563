"""Graph nested dissection (SLU_ORDER_GRAPH_ND), checked on the host.

The library computes the order; the oracle consumes it (pattern, Algorithm 2
and Algorithm 3 bit-exact with the oracle on that order) and pins its
defining properties independently: a permutation; dense vertices last (the
arrowhead of Fig. 2 then has no fill); independent systems of a bordered
block-diagonal matrix contiguous, with the border last and no fill between
systems; the top separator of a connected grid disconnects it; fill no worse
than the geometric nested dissection on grids; deterministic."""
import numpy as np
import pytest

import synth
from oracle import blocking, metrics, ordering, symbolic

slu = pytest.importorskip("paper_2512_04389_amd")


def _order(n, rp, ci, **kw):
    h = slu.SparseLU(n, rp, ci, ordering="graph_nd", **kw)
    p = h.perm()
    assert ordering.is_permutation(p, n)
    return h, p


def _adjacency(n, rp, ci):
    rows = np.repeat(np.arange(n), np.diff(rp))
    cols = np.asarray(ci, dtype=np.int64)
    off = rows != cols
    adj = [set() for _ in range(n)]
    for r, c in zip(rows[off].tolist(), cols[off].tolist()):
        adj[r].add(c)
        adj[c].add(r)
    return adj


def _components(vertices, adj):
    left = set(vertices)
    comps = []
    while left:
        s = min(left)
        stack, seen = [s], {s}
        while stack:
            v = stack.pop()
            for u in adj[v]:
                if u in left and u not in seen:
                    seen.add(u)
                    stack.append(u)
        comps.append(seen)
        left -= seen
    return comps


@pytest.mark.parametrize("case", ["lap2d-40", "lap3d-12", "convdiff-10", "random-500"])
def test_oracle_consumes_order(case):
    if case == "lap2d-40":
        n, rp, ci, _ = synth.laplacian_2d(40)
    elif case == "lap3d-12":
        n, rp, ci, _ = synth.laplacian_3d(12)
    elif case == "convdiff-10":
        n, rp, ci, _ = synth.convection_diffusion_3d(10)
    else:
        rng = np.random.default_rng(3)
        n = 500
        r = rng.integers(0, n, 1500)
        c = rng.integers(0, n, 1500)
        rp, ci, _ = synth.coo_to_csr(n, np.concatenate([r, np.arange(n)]), np.concatenate([c, np.arange(n)]))
    h, p = _order(n, rp, ci)
    cp, ri = symbolic.symbolic(n, rp, ci, p)
    hcp, hri = h.pattern()
    assert np.array_equal(hcp, cp) and np.array_equal(hri, ri)
    bp = blocking.diag_block_ptr(n, cp, ri)
    assert np.array_equal(h.blockptr(), bp)
    assert np.array_equal(h.blocking(), blocking.irregular_blocking(bp))
    assert h.info()["flops"] == float(metrics.flops(cp))
    # deterministic
    _, p2 = _order(n, rp, ci)
    assert np.array_equal(p, p2)


def test_arrowhead_hub_last():
    # Fig. 2: the hub eliminated first fills the whole matrix, last none
    n = 300
    rows = np.concatenate([np.zeros(n - 1, np.int64), np.arange(1, n), np.arange(n)])
    cols = np.concatenate([np.arange(1, n), np.zeros(n - 1, np.int64), np.arange(n)])
    rp, ci, _ = synth.coo_to_csr(n, rows, cols)
    h, p = _order(n, rp, ci)
    assert p[-1] == 0
    cp, ri = symbolic.symbolic(n, rp, ci, p)
    assert 2 * (int(cp[-1]) - n) + n == 3 * n - 2
    cp0, _ = symbolic.symbolic(n, rp, ci, ordering.natural(n))
    assert 2 * (int(cp0[-1]) - n) + n == n * n


def test_bordered_block_diagonal_border_last_systems_apart():
    nb, border = 6, 60
    n, rp, ci, _ = synth.bbd_circuit(n=1860, nblocks=nb, border=border, border_nnz=12000, seed=7)
    h, p = _order(n, rp, ci)
    inner = n - border
    # the border rows are exactly the last ones
    assert set(p[inner:].tolist()) == set(range(inner, n))
    # each system occupies one contiguous range of positions
    sizes = [inner // nb + (1 if q < inner % nb else 0) for q in range(nb)]
    starts = np.concatenate([[0], np.cumsum(sizes)])
    sys_of = np.searchsorted(starts, p[:inner], side="right") - 1
    changes = int(np.sum(sys_of[1:] != sys_of[:-1]))
    assert changes == nb - 1
    # no fill couples two systems: S restricted to the systems is block diagonal
    cp, ri = symbolic.symbolic(n, rp, ci, p)
    col = np.repeat(np.arange(n), np.diff(cp))
    r = ri.astype(np.int64)
    inside = (col < inner) & (r < inner)
    assert np.array_equal(sys_of[col[inside]], sys_of[r[inside]])


@pytest.mark.parametrize("dims", [(30, 30, 1), (9, 9, 9)])
def test_top_separator_disconnects(dims):
    n, rp, ci, _ = synth.grid_laplacian(dims)
    h, p = _order(n, rp, ci)
    cp, ri = symbolic.symbolic(n, rp, ci, p)
    # the top separator is the chain at the root of the elimination tree
    pptr, pidx = symbolic.permute_symmetric(n, *symbolic.symmetric_pattern(n, rp, ci), p)
    parent = symbolic.etree(n, pptr, pidx)
    children = [[] for _ in range(n)]
    for j in range(n):
        if parent[j] >= 0:
            children[int(parent[j])].append(j)
    roots = [j for j in range(n) if parent[j] < 0]
    assert len(roots) == 1
    chain, v = [], roots[0]
    while len(children[v]) == 1:
        chain.append(v)
        v = children[v][0]
    chain.append(v)
    assert len(children[v]) >= 2, "no branching below the top separator"
    sep = {int(p[k]) for k in chain}
    assert len(sep) < n // 4
    adj = _adjacency(n, rp, ci)
    comps = _components([u for u in range(n) if u not in sep], adj)
    assert len(comps) >= 2


@pytest.mark.parametrize("k", [32, 12])
def test_fill_against_geometric_nd(k):
    dims = (k, k, 1) if k == 32 else (k, k, k)
    n, rp, ci, _ = synth.grid_laplacian(dims)
    h, p = _order(n, rp, ci)
    cp, _ = symbolic.symbolic(n, rp, ci, p)
    cg, _ = symbolic.symbolic(n, rp, ci, ordering.nd_grid(dims))
    cn, _ = symbolic.symbolic(n, rp, ci, ordering.natural(n))
    assert cp[-1] <= 1.25 * cg[-1]
    assert cp[-1] < 0.8 * cn[-1]


def test_batch_with_graph_nd():
    systems = [synth.batch_system(s)[:3] for s in (0, 130)]
    h = slu.SparseLU.batch(systems, ordering="graph_nd")
    p = h.perm()
    n0 = systems[0][0]
    for q, (n, rp, ci) in enumerate(systems):
        off = 0 if q == 0 else n0
        hs = slu.SparseLU(n, rp, ci, ordering="graph_nd")
        assert np.array_equal(p[off:off + n] - off, hs.perm())
