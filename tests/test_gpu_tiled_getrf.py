"""GPU parity of the tiled GETRF (slu_set_getrf_tiled): every wave whose
largest diagonal block reaches the threshold factors its blocks in 16 x 16
tiles; the factors must match the oracle element-wise (1e-10 relative) and
the solves reach backward error <= 1e-12, on ragged, sparse and dense
diagonal blocks up to a 1000-row dense block."""
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


def _dense_dd(n, seed):
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1, 1, (n, n))
    a[np.arange(n), np.arange(n)] = np.abs(a).sum(1) + 1.0
    rp = np.arange(0, n * n + 1, n, dtype=np.int64)
    ci = np.tile(np.arange(n, dtype=np.int32), n)
    return n, rp, ci, a.reshape(-1).copy()


TILES = (32, 16)


def _run_tiled(name, n, rp, ci, v, min_rows=1, nrhs=1, tile=32, **kw):
    import paper_2512_04389_amd as slu
    announce("tiled GETRF (tile %d) %s n=%d min_rows=%d %s" % (tile, name, n, min_rows, kw))
    h = slu.SparseLU(n, rp, ci, **kw).bind()
    h.set_getrf_tiled(min_rows)
    h.set_getrf_tile(tile)
    vals = torch.from_numpy(np.ascontiguousarray(v, dtype=np.float64)).cuda()
    h.factor(vals)
    torch.cuda.synchronize()
    check_factors(h, n, rp, ci, v, kw)
    check_solves(h, n, rp, ci, v, vals, nrhs=nrhs)
    return h, vals


@pytest.mark.parametrize("tile", TILES)
def test_tiled_grids(tile):
    n, rp, ci, v = synth.laplacian_2d(64)
    _run_tiled("lap2d-64", n, rp, ci, v, tile=tile, ordering="grid_nd", grid_dims=(64, 64, 1))
    n, rp, ci, v = synth.laplacian_3d(12)
    _run_tiled("lap3d-12", n, rp, ci, v, nrhs=3, tile=tile, ordering="grid_nd", grid_dims=(12, 12, 12))
    n, rp, ci, v = synth.convection_diffusion_3d(16)
    _run_tiled("convdiff-16", n, rp, ci, v, nrhs=2, tile=tile, ordering="grid_nd", grid_dims=(16, 16, 16))


@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("b", [37, 200, 700])
def test_tiled_regular_blocks(b, tile):
    n, rp, ci, v = synth.convection_diffusion_3d(14)
    _run_tiled("convdiff-14-regular-%d" % b, n, rp, ci, v, tile=tile, ordering="grid_nd", grid_dims=(14, 14, 14),
               blocking="regular", block_size=b)


def test_tiled_only_large_waves():
    # threshold 129: waves of small blocks keep the one-launch GETRF
    n, rp, ci, v = synth.convection_diffusion_3d(14)
    _run_tiled("convdiff-14-irregular-129", n, rp, ci, v, min_rows=129, ordering="grid_nd",
               grid_dims=(14, 14, 14))


@pytest.mark.parametrize("tile", TILES)
def test_tiled_bbd_and_random(tile):
    n, rp, ci, v = synth.bbd_circuit(n=2400, nblocks=8, border=80, border_nnz=2000, seed=4)
    _run_tiled("bbd-2400", n, rp, ci, v, nrhs=8, tile=tile)
    _run_tiled("bbd-2400-regular-300", n, rp, ci, v, tile=tile, blocking="regular", block_size=300)
    n, rp, ci, v = synth.grid_laplacian((600, 4, 1))
    _run_tiled("band-600x4-regular-1200", n, rp, ci, v, tile=tile, blocking="regular", block_size=1200)


@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("n", [1000, 913, 47])
def test_tiled_dense_block(n, tile):
    # one dense diagonal block of n rows (913, 47: ragged last tiles)
    n, rp, ci, v = _dense_dd(n, seed=n)
    _run_tiled("dense-%d" % n, n, rp, ci, v, nrhs=2, tile=tile, blocking="regular", block_size=n)


@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("zc", [21, 9, 37])
def test_tiled_tiny_and_zero_pivot(tile, zc):
    import paper_2512_04389_amd as slu
    _run_tiled("n1", 1, np.array([0, 1]), np.array([0], np.int32), np.array([4.0]), tile=tile)
    _run_tiled("n2", 2, np.array([0, 2, 4]), np.array([0, 1, 0, 1], np.int32), np.array([2.0, 1.0, 1.0, 3.0]),
               tile=tile)
    _run_tiled("tridiag-natural", *synth.grid_laplacian((50, 1, 1)), tile=tile)
    announce("tiled GETRF (tile %d) zero pivot in a 40-row dense block, column %d" % (tile, zc))
    n, rp, ci, v = _dense_dd(40, seed=3)
    a = v.reshape(n, n).copy()
    # row zc zero up to its diagonal: no multiplier reaches it, so pivot zc
    # is exactly zero
    a[zc, :zc + 1] = 0.0
    h = slu.SparseLU(n, rp, ci, blocking="regular", block_size=n).bind()
    h.set_getrf_tiled(1)
    h.set_getrf_tile(tile)
    with pytest.raises(slu.ZeroPivot) as e:
        h.factor(torch.from_numpy(a.reshape(-1).copy()).cuda())
    assert e.value.col == zc
    h.factor(torch.from_numpy(v).cuda())
    assert h.info()["factored"] == 1
    with pytest.raises(slu.SluError):
        h.set_getrf_tiled(-1)
    with pytest.raises(slu.SluError):
        h.set_getrf_tile(8)


@pytest.mark.parametrize("tile", TILES)
def test_tiled_graph_replay_bit_identical(tile):
    import paper_2512_04389_amd as slu
    n, rp, ci, v = synth.convection_diffusion_3d(14)
    announce("tiled GETRF (tile %d) graph replay convdiff-14 regular 300" % tile)
    h = slu.SparseLU(n, rp, ci, ordering="grid_nd", grid_dims=(14, 14, 14), blocking="regular",
                     block_size=300).bind()
    h.set_getrf_tiled(1)
    h.set_getrf_tile(tile)
    vals = torch.from_numpy(v).cuda()
    h.factor(vals)
    l0, u0 = h.factors()
    h.set_graph(True)
    for _ in range(3):
        h.factor(vals)
        torch.cuda.synchronize()
        l1, u1 = h.factors()
        np.testing.assert_array_equal(l1, l0)
        np.testing.assert_array_equal(u1, u0)
    h.set_graph(False)
