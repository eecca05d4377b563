"""GPU parity of slu_factor / slu_solve / slu_solve_transpose with the oracle
(element-wise factors within 1e-10 relative, backward error <= 1e-12)."""
import numpy as np
import pytest

import synth
from gpu_common import announce, check_factors, run_case

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _dd_random(n, dens, seed, sym_pattern=False):
    rng = np.random.default_rng(seed)
    nnz = max(1, int(dens * n * n))
    r = rng.integers(0, n, nnz)
    c = rng.integers(0, n, nnz)
    if sym_pattern:
        r, c = np.concatenate([r, c]), np.concatenate([c, r])
    off = r != c
    r, c = r[off], c[off]
    rp, ci, _ = synth.coo_to_csr(n, r, c)
    vals = rng.uniform(-1, 1, len(ci))
    rows = np.repeat(np.arange(n), np.diff(rp))
    diag = np.bincount(rows, weights=np.abs(vals), minlength=n) + 1.0
    rp, ci, v = synth.coo_to_csr(n, np.concatenate([rows, np.arange(n)]),
                                 np.concatenate([ci, np.arange(n)]), np.concatenate([vals, diag]))
    return n, rp, ci, v


@pytest.mark.parametrize("k", [3, 8, 64])
def test_laplacian_2d(k):
    n, rp, ci, v = synth.laplacian_2d(k)
    run_case("lap2d-%d" % k, n, rp, ci, v, ordering="grid_nd", grid_dims=(k, k, 1))


@pytest.mark.parametrize("k", [6, 12])
def test_laplacian_3d(k):
    n, rp, ci, v = synth.laplacian_3d(k)
    run_case("lap3d-%d" % k, n, rp, ci, v, nrhs=3, ordering="grid_nd", grid_dims=(k, k, k))


def test_convection_diffusion_16():
    n, rp, ci, v = synth.convection_diffusion_3d(16)
    run_case("convdiff-16", n, rp, ci, v, nrhs=17, ordering="grid_nd", grid_dims=(16, 16, 16))


def test_strict_level_schedule():
    n, rp, ci, v = synth.convection_diffusion_3d(14)
    run_case("convdiff-14-levels", n, rp, ci, v, ordering="grid_nd", grid_dims=(14, 14, 14),
             schedule="levels")
    run_case("convdiff-14-regular-300-levels", n, rp, ci, v, ordering="grid_nd", grid_dims=(14, 14, 14),
             blocking="regular", block_size=300, schedule="levels")


@pytest.mark.parametrize("b", [37, 200, 700])
def test_regular_blocking_chunked_getrf(b):
    # b > 128 exercises the chunked GETRF path; 37 leaves a ragged last block
    n, rp, ci, v = synth.convection_diffusion_3d(14)
    run_case("convdiff-14-regular-%d" % b, n, rp, ci, v, ordering="grid_nd", grid_dims=(14, 14, 14),
             blocking="regular", block_size=b)


def test_solve_chunks_split_beyond_staging_budget():
    # natural order on a 600 x 4 grid has bandwidth 600: the 16-column chunks
    # of 1200-row blocks couple about 600 rows, more than one LDS batch holds
    n, rp, ci, v = synth.grid_laplacian((600, 4, 1))
    run_case("band-600x4-regular-1200", n, rp, ci, v, nrhs=3, blocking="regular", block_size=1200)


def test_random_unsymmetric_natural():
    n, rp, ci, v = _dd_random(600, 0.01, seed=5)
    run_case("random-600", n, rp, ci, v, nrhs=2)
    run_case("random-600-regular-160", n, rp, ci, v, blocking="regular", block_size=160)


@pytest.mark.parametrize("case", ["lap3d-12", "convdiff-16", "bbd-2400", "random-600"])
def test_graph_nested_dissection(case):
    if case == "lap3d-12":
        n, rp, ci, v = synth.laplacian_3d(12)
    elif case == "convdiff-16":
        n, rp, ci, v = synth.convection_diffusion_3d(16)
    elif case == "bbd-2400":
        n, rp, ci, v = synth.bbd_circuit(n=2400, nblocks=8, border=80, border_nnz=12000, seed=4)
    else:
        n, rp, ci, v = _dd_random(600, 0.01, seed=5)
    run_case("graph-nd-" + case, n, rp, ci, v, nrhs=2, ordering="graph_nd")


def test_random_user_perm():
    n, rp, ci, v = _dd_random(400, 0.02, seed=6, sym_pattern=True)
    perm = np.random.default_rng(1).permutation(n).astype(np.int32)
    run_case("random-400-user", n, rp, ci, v, ordering="user", perm=perm)


def test_bbd_small():
    n, rp, ci, v = synth.bbd_circuit(n=2400, nblocks=8, border=80, border_nnz=2000, seed=4)
    run_case("bbd-2400", n, rp, ci, v, nrhs=8)


@pytest.mark.parametrize("s", [0, 200])
def test_batch_member(s):
    n, rp, ci, v, dims = synth.batch_system(s)
    run_case("batch-%d" % s, n, rp, ci, v, ordering="grid_nd", grid_dims=dims)


def test_tiny_and_degenerate():
    run_case("n1", 1, np.array([0, 1]), np.array([0], np.int32), np.array([4.0]))
    run_case("n2", 2, np.array([0, 2, 4]), np.array([0, 1, 0, 1], np.int32), np.array([2.0, 1.0, 1.0, 3.0]))
    # structurally missing diagonal is filled in S with a zero that receives fill
    run_case("tridiag-natural", *synth.grid_laplacian((50, 1, 1)))


def test_zero_pivot_and_nonfinite():
    import paper_2512_04389_amd as slu
    announce("zero pivot")
    h = slu.SparseLU(2, np.array([0, 1, 2]), np.array([1, 0], np.int32)).bind()
    with pytest.raises(slu.ZeroPivot) as e:
        h.factor(torch.tensor([1.0, 1.0], dtype=torch.float64, device="cuda"))
    assert e.value.col == 0
    assert h.info()["factored"] == 0
    with pytest.raises(slu.SluError):
        h.solve(torch.ones(2, dtype=torch.float64, device="cuda"))
    announce("pivot cancels to zero")
    h = slu.SparseLU(2, np.array([0, 2, 4]), np.array([0, 1, 0, 1], np.int32)).bind()
    with pytest.raises(slu.ZeroPivot) as e:
        h.factor(torch.ones(4, dtype=torch.float64, device="cuda"))
    assert e.value.col == 1
    announce("nan value")
    with pytest.raises(slu.ZeroPivot):
        h.factor(torch.tensor([float("nan"), 1.0, 1.0, 3.0], dtype=torch.float64, device="cuda"))
    # a good factorization afterwards works
    h.factor(torch.tensor([2.0, 1.0, 1.0, 3.0], dtype=torch.float64, device="cuda"))
    assert h.info()["factored"] == 1


@pytest.mark.parametrize("case", ["convdiff-14-regular-200", "convdiff-14-regular-700", "band-600x4-regular-1200",
                                  "bbd-2400-regular-300"])
def test_split_getrf_matches_one_launch(case):
    # slu_set_getrf_split(0): every wave with a chunked block (b > 128) takes
    # the panel + chip-wide trailing-tile launches per chunk; the factors
    # must equal the one-launch GETRF's bit for bit (also under graph replay),
    # and the oracle's within the parity tolerance
    import paper_2512_04389_amd as slu
    if case.startswith("convdiff"):
        n, rp, ci, v = synth.convection_diffusion_3d(14)
        opts = dict(ordering="grid_nd", grid_dims=(14, 14, 14), blocking="regular",
                    block_size=int(case.rsplit("-", 1)[1]))
    elif case.startswith("band"):
        n, rp, ci, v = synth.grid_laplacian((600, 4, 1))
        opts = dict(blocking="regular", block_size=1200)
    else:
        n, rp, ci, v = synth.bbd_circuit(n=2400, nblocks=8, border=80, border_nnz=2000, seed=4)
        opts = dict(blocking="regular", block_size=300)
    announce("split GETRF " + case)
    h = slu.SparseLU(n, rp, ci, **opts).bind()
    h.set_getrf_tiled(0)
    assert max(np.diff(h.blocking())) > 128
    vals = torch.from_numpy(v).cuda()
    h.factor(vals)
    l0, u0 = h.factors()
    h.set_getrf_split(0)
    h.factor(vals)
    l1, u1 = h.factors()
    np.testing.assert_array_equal(l1, l0)
    np.testing.assert_array_equal(u1, u0)
    h.set_graph(True)
    for _ in range(2):
        h.factor(vals)
        l2, u2 = h.factors()
        np.testing.assert_array_equal(l2, l0)
        np.testing.assert_array_equal(u2, u0)
    h.set_graph(False)
    check_factors(h, n, rp, ci, v, opts)
    with pytest.raises(slu.SluError):
        h.set_getrf_split(-1.0)


@pytest.mark.parametrize("case", ["lap3d-12", "convdiff-14-regular-200", "bbd-2400"])
def test_chunked_getrf_paths(case):
    # slu_set_getrf_tiled(0): the one-launch GETRF (dense blocks of at most
    # 128 rows in LDS, chunked above) on every wave
    import paper_2512_04389_amd as slu
    if case == "lap3d-12":
        n, rp, ci, v = synth.laplacian_3d(12)
        opts = dict(ordering="grid_nd", grid_dims=(12, 12, 12))
    elif case.startswith("convdiff"):
        n, rp, ci, v = synth.convection_diffusion_3d(14)
        opts = dict(ordering="grid_nd", grid_dims=(14, 14, 14), blocking="regular", block_size=200)
    else:
        n, rp, ci, v = synth.bbd_circuit(n=2400, nblocks=8, border=80, border_nnz=2000, seed=4)
        opts = {}
    announce("chunked GETRF " + case)
    h = slu.SparseLU(n, rp, ci, **opts).bind()
    h.set_getrf_tiled(0)
    vals = torch.from_numpy(v).cuda()
    h.factor(vals)
    check_factors(h, n, rp, ci, v, opts)


def test_determinism_and_refactor():
    import paper_2512_04389_amd as slu
    n, rp, ci, v = synth.laplacian_3d(12)
    announce("determinism lap3d-12")
    h = slu.SparseLU(n, rp, ci, ordering="grid_nd", grid_dims=(12, 12, 12)).bind()
    vals = torch.from_numpy(v).cuda()
    h.factor(vals)
    l1, u1 = h.factors()
    # refactor with other values on the same pattern, then the first again
    h.factor(vals * 2.0)
    l2, u2 = h.factors()
    cp, ri = h.pattern()
    low = ri.astype(np.int64) > np.repeat(np.arange(n), np.diff(cp))
    np.testing.assert_array_equal(l2[low], l1[low])  # L is invariant under A -> 2A
    np.testing.assert_array_equal(u2[low], 2.0 * u1[low])
    np.testing.assert_array_equal(l2[~low], 2.0 * l1[~low])  # diagonal of U
    h.factor(vals)
    l3, u3 = h.factors()
    assert np.array_equal(l1, l3) and np.array_equal(u1, u3)
    check_factors(h, n, rp, ci, v, dict(ordering="grid_nd", grid_dims=(12, 12, 12)))
