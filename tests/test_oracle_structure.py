"""Pins of the oracle's structural part: ordering, symbolic fill, Algorithm 2,
sampling and Algorithm 3.  Each check is against something other than the
oracle itself: hand-derived cases, brute force, closed forms, invariants."""
import numpy as np
import pytest

import synth
from oracle import blocking, ordering, symbolic


# ----------------------------------------------------------------- ordering
def test_nd_1d_hand_derived():
    # 20 points on a line: cut at 10, then at 5 and 15; leaves have <= 8 points
    perm = ordering.nd_grid((20, 1, 1))
    expect = [0, 1, 2, 3, 4, 6, 7, 8, 9, 5, 11, 12, 13, 14, 16, 17, 18, 19, 15, 10]
    assert perm.tolist() == expect


def test_nd_2d_hand_derived():
    # 5 x 5: cut x at 2 (tie between axes -> x); each half cut along y at 2
    perm = ordering.nd_grid((5, 5))
    expect = [0, 1, 5, 6, 15, 16, 20, 21, 10, 11,
              3, 4, 8, 9, 18, 19, 23, 24, 13, 14,
              2, 7, 12, 17, 22]
    assert perm.tolist() == expect


@pytest.mark.parametrize("dims", [(64, 64, 1), (13, 7, 1), (9, 10, 11), (16, 16, 16), (1, 1, 1), (3, 1, 1)])
def test_nd_is_permutation_and_separator_last(dims):
    perm = ordering.nd_grid(dims)
    n = dims[0] * dims[1] * dims[2]
    assert ordering.is_permutation(perm, n)
    if max(dims) > 2 and n > 8:
        # the last block of the order is the top separator plane
        d = int(np.argmax(dims))
        m = dims[d] // 2
        nsep = n // dims[d]
        last = perm[-nsep:].astype(np.int64)
        coords = [last % dims[0], (last // dims[0]) % dims[1], last // (dims[0] * dims[1])]
        assert np.all(coords[d] == m)


# ----------------------------------------------------------------- symbolic
def _random_sym_pattern(n, density, rng):
    m = rng.random((n, n)) < density
    m = m | m.T
    np.fill_diagonal(m, True)
    return m


def _dense_to_csr(m):
    n = m.shape[0]
    rows, cols = np.nonzero(m)
    rp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rp, rows + 1, 1)
    return np.cumsum(rp), cols.astype(np.int32)


@pytest.mark.parametrize("seed", range(12))
def test_fill_matches_bruteforce(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 60))
    dens = float(rng.choice([0.02, 0.05, 0.1, 0.3]))
    m = rng.random((n, n)) < dens          # unsymmetric pattern
    np.fill_diagonal(m, rng.random(n) < 0.5)  # diagonal sometimes missing
    rp, ci = _dense_to_csr(m)
    perm = rng.permutation(n).astype(np.int32)
    cp, ri = symbolic.symbolic(n, rp, ci, perm)
    # brute force on the symmetrised permuted pattern
    ms = m | m.T
    np.fill_diagonal(ms, True)
    mp = ms[np.ix_(perm, perm)]
    expect = symbolic.fill_dense_bruteforce(mp)
    got = symbolic.lower_to_dense(n, cp, ri)
    assert np.array_equal(got, expect)
    # rows sorted, diagonal first in every column
    for k in range(n):
        col = ri[cp[k]:cp[k + 1]]
        assert col[0] == k and np.all(np.diff(col) > 0)


@pytest.mark.parametrize("seed", range(6))
def test_fill_path_theorem(seed):
    # (i, j) in S iff a path joins i and j through vertices < min(i, j)
    rng = np.random.default_rng(100 + seed)
    n = 25
    m = _random_sym_pattern(n, 0.08, rng)
    rp, ci = _dense_to_csr(m)
    cp, ri = symbolic.symbolic(n, rp, ci, np.arange(n, dtype=np.int32))
    got = symbolic.lower_to_dense(n, cp, ri)
    for i in range(n):
        for j in range(i):
            lim = j
            # BFS from i to j through vertices < lim
            seen = {i}
            stack = [i]
            found = False
            while stack and not found:
                v = stack.pop()
                for w in np.nonzero(m[v])[0]:
                    w = int(w)
                    if w == j:
                        found = True
                        break
                    if w < lim and w not in seen:
                        seen.add(w)
                        stack.append(w)
            assert got[i, j] == found, (i, j)


def test_etree_parent_is_first_subdiagonal_row():
    n, rp, ci, _ = synth.laplacian_2d(12)
    perm = ordering.nd_grid((12, 12))
    ptr, idx = symbolic.symmetric_pattern(n, rp, ci)
    pptr, pidx = symbolic.permute_symmetric(n, ptr, idx, perm)
    parent = symbolic.etree(n, pptr, pidx)
    cp, ri = symbolic.fill_lower(n, pptr, pidx)
    for k in range(n):
        below = ri[cp[k] + 1:cp[k + 1]]
        assert parent[k] == (below[0] if below.shape[0] else -1)


def test_tridiagonal_no_fill():
    n = 50
    m = np.eye(n, dtype=bool) | np.eye(n, k=1, dtype=bool) | np.eye(n, k=-1, dtype=bool)
    rp, ci = _dense_to_csr(m)
    cp, ri = symbolic.symbolic(n, rp, ci, np.arange(n, dtype=np.int32))
    assert 2 * (int(cp[-1]) - n) + n == 3 * n - 2


def test_arrowhead_hub_first_and_last():
    # Fig. 2: the same graph fills completely or not at all depending on order
    n = 30
    m = np.eye(n, dtype=bool)
    m[0, :] = True
    m[:, 0] = True
    rp, ci = _dense_to_csr(m)
    cp, _ = symbolic.symbolic(n, rp, ci, np.arange(n, dtype=np.int32))
    assert 2 * (int(cp[-1]) - n) + n == n * n
    hub_last = np.concatenate([np.arange(1, n), [0]]).astype(np.int32)
    cp, _ = symbolic.symbolic(n, rp, ci, hub_last)
    assert 2 * (int(cp[-1]) - n) + n == 3 * n - 2


# --------------------------------------------------------------- Algorithm 2
@pytest.mark.parametrize("seed", range(6))
def test_blockptr_bruteforce(seed):
    rng = np.random.default_rng(200 + seed)
    n = int(rng.integers(1, 50))
    m = rng.random((n, n)) < 0.1
    rp, ci = _dense_to_csr(m)
    cp, ri = symbolic.symbolic(n, rp, ci, rng.permutation(n).astype(np.int32))
    S = symbolic.lower_to_dense(n, cp, ri)
    bp = blocking.diag_block_ptr(n, cp, ri)
    for i in range(n + 1):
        assert bp[i] == int(S[:i, :i].sum())
    # the full symmetric CSC gives the same pointer (only lower entries count)
    rows, cols = np.nonzero(S.T)   # CSC of S: column-major scan
    fcp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(fcp, rows + 1, 1)
    fcp = np.cumsum(fcp)
    assert np.array_equal(blocking.diag_block_ptr(n, fcp, cols), bp)
    assert bp[n] == int(S.sum())
    assert np.all(np.diff(bp) % 2 == 1)


def test_blockptr_closed_forms():
    n = 40
    tri = np.eye(n, dtype=bool) | np.eye(n, k=1, dtype=bool) | np.eye(n, k=-1, dtype=bool)
    rp, ci = _dense_to_csr(tri)
    cp, ri = symbolic.symbolic(n, rp, ci, np.arange(n, dtype=np.int32))
    bp = blocking.diag_block_ptr(n, cp, ri)
    assert bp[0] == 0 and all(bp[i] == 3 * i - 2 for i in range(1, n + 1))
    dense = np.ones((n, n), dtype=bool)
    rp, ci = _dense_to_csr(dense)
    cp, ri = symbolic.symbolic(n, rp, ci, np.arange(n, dtype=np.int32))
    bp = blocking.diag_block_ptr(n, cp, ri)
    assert all(bp[i] == i * i for i in range(n + 1))


# --------------------------------------------------------------- Algorithm 3
def _tri_bp(N):
    bp = np.zeros(N + 1, dtype=np.int64)
    bp[1:] = 3 * np.arange(1, N + 1) - 2
    return bp


def _dense_bp(N):
    return (np.arange(N + 1, dtype=np.int64)) ** 2


def test_alg3_tridiagonal_1000():
    ptr = blocking.irregular_blocking(_tri_bp(1000))
    # first window: 4*1000 < 2*2998 (skip); every later window: 6000 >= 5996
    assert ptr.tolist() == [0] + list(range(3, 1001))
    assert len(ptr) - 1 == 998


def test_alg3_dense_1000():
    ptr = blocking.irregular_blocking(_dense_bp(1000))
    # window i passes iff (4i + 4) * 1000 >= 2 * 10^6, i.e. i >= 499;
    # before that the skip counter forces a boundary every 4 samples
    expect = [0] + list(range(5, 498, 4)) + [501] + list(range(502, 1001))
    assert ptr.tolist() == expect
    sizes = np.diff(ptr)
    assert len(sizes) == 624
    assert sizes[0] == 5 and np.sum(sizes == 4) == 124 and np.sum(sizes == 1) == 499


def test_alg3_dense_16():
    ptr = blocking.irregular_blocking(_dense_bp(16))
    assert ptr.tolist() == [0, 5, 9, 10, 11, 12, 13, 14, 15, 16]


def test_alg3_advance_step():
    ptr = blocking.irregular_blocking(_tri_bp(1000), advance=2)
    assert ptr.tolist() == [0] + list(range(4, 1001, 2))
    ptr = blocking.irregular_blocking(_dense_bp(1000), advance=2)
    assert set(np.diff(ptr).tolist()) == {8, 6, 2}


@pytest.mark.parametrize("N", [1, 2, 3, 7, 999, 1000, 1001, 4096, 12345])
def test_alg3_invariants(N):
    rng = np.random.default_rng(N)
    inc = 2 * rng.integers(0, 6, size=N) + 1          # odd increments
    bp = np.concatenate([[0], np.cumsum(inc)]).astype(np.int64)
    ptr = blocking.irregular_blocking(bp)
    assert ptr[0] == 0 and ptr[-1] == N
    assert np.all(np.diff(ptr) > 0)
    pos, sp = blocking.sample_rows(N)
    # every interior boundary is a sample row; sizes are 1..4 basic intervals
    assert set(ptr[1:-1].tolist()) <= set(pos.tolist())
    idx = np.searchsorted(pos, ptr[1:-1])
    if idx.shape[0] > 1:
        assert np.all(np.diff(idx) >= 1) and np.all(np.diff(idx) <= 4)
    if idx.shape[0]:
        assert 2 <= idx[0] <= 5


def test_alg3_dense_tail_gets_fine_blocks():
    # a matrix sparse top-left and dense bottom-right (Section 1, Fig. 11):
    # coarse blocks first, single basic intervals at the end
    N = 2000
    inc = np.ones(N, dtype=np.int64)
    inc[1500:] = 2 * 600 + 1
    bp = np.concatenate([[0], np.cumsum(inc)])
    sizes = np.diff(blocking.irregular_blocking(bp))
    assert sizes[:10].min() >= 8 and sizes[-10:].max() == 2


def test_regular_blocking():
    assert blocking.regular_blocking(10, 3).tolist() == [0, 3, 6, 9, 10]
    assert blocking.regular_blocking(9, 3).tolist() == [0, 3, 6, 9]
    assert blocking.regular_blocking(2, 5).tolist() == [0, 2]


def test_nonempty_blocks_bruteforce():
    n, rp, ci, _ = synth.laplacian_2d(9)
    perm = ordering.nd_grid((9, 9))
    cp, ri = symbolic.symbolic(n, rp, ci, perm)
    ptr = np.array([0, 10, 25, 40, 60, 81])
    bi, bj, cnt = blocking.nonempty_blocks(n, cp, ri, ptr)
    S = symbolic.lower_to_dense(n, cp, ri)
    expect = {}
    for a in range(5):
        for b in range(5):
            c = int(S[ptr[a]:ptr[a + 1], ptr[b]:ptr[b + 1]].sum())
            if c:
                expect[(a, b)] = c
    got = {(int(a), int(b)): int(c) for a, b, c in zip(bi, bj, cnt)}
    assert got == expect
