"""Host parity of the analysis at the benchmark configurations, no GPU: the
ordering, the filled pattern S, Algorithm 2's block pointer and Algorithm 3's
block boundaries of the library equal the oracle's bit for bit on the 3D
Laplacian 48^3, the convection-diffusion 64^3 (geometric nested dissection)
and the bordered block-diagonal 200k matrix (natural order), and so do the
flop count and the number of non-empty blocks.  The library's handle is
released before the oracle runs, to bound the memory held at once."""
import gc

import numpy as np
import pytest

import synth
from oracle import blocking, metrics, ordering, symbolic

slu = pytest.importorskip("paper_2512_04389_amd")


def _library(n, rp, ci, **kw):
    h = slu.SparseLU(n, rp, ci, **kw)
    out = dict(perm=h.perm(), pattern=h.pattern(), blockptr=h.blockptr(), ptr=h.blocking(), info=h.info())
    h.close()
    del h
    gc.collect()
    return out


@pytest.mark.parametrize("case", ["lap3d48", "convdiff64", "bbd200k"])
def test_bench_configuration_structure_bit_exact(case):
    if case == "lap3d48":
        n, rp, ci, _ = synth.laplacian_3d(48)
        kw = dict(ordering="grid_nd", grid_dims=(48, 48, 48))
        perm = ordering.nd_grid((48, 48, 48))
    elif case == "convdiff64":
        n, rp, ci, _ = synth.convection_diffusion_3d(64)
        kw = dict(ordering="grid_nd", grid_dims=(64, 64, 64))
        perm = ordering.nd_grid((64, 64, 64))
    else:
        n, rp, ci, _ = synth.bbd_circuit()
        kw = dict(ordering="natural")
        perm = ordering.natural(n)
    lib = _library(n, rp, ci, **kw)
    assert np.array_equal(lib["perm"], perm)
    cp, ri = symbolic.symbolic(n, rp, ci, perm)
    hcp, hri = lib.pop("pattern")
    assert np.array_equal(hcp, cp)
    assert np.array_equal(hri, ri)
    del hcp, hri
    bp = blocking.diag_block_ptr(n, cp, ri)
    assert np.array_equal(lib["blockptr"], bp)
    ptr = blocking.irregular_blocking(bp)
    assert np.array_equal(lib["ptr"], ptr)
    info = lib["info"]
    assert info["nnz_s"] == 2 * (int(cp[-1]) - n) + n
    assert info["flops"] == float(metrics.flops(cp))
    bi, _, _ = blocking.nonempty_blocks(n, cp, ri, ptr)
    assert info["nonempty_blocks"] == len(bi)
