"""The solve as a torch.autograd.Function (paper_2512_04389_amd.solve):
values and right-hand-side gradients against the oracle's adjoint, central
finite differences through the GPU path, torch's gradcheck, and a refactor
between forward and backward."""
import numpy as np
import pytest

import synth
from gpu_common import announce
from oracle import adjoint, ordering

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _convdiff(k, seed):
    n, rp, ci, v = synth.convection_diffusion_3d(k)
    rng = np.random.default_rng(seed)
    return n, rp, ci, v * (1.0 + 0.05 * rng.uniform(-1, 1, v.shape))


def _close(got, ref, rtol=1e-9):
    scale = float(np.max(np.abs(ref)))
    return np.all(np.abs(got - ref) <= rtol * (np.abs(ref) + 1e-8 * scale))


def test_adjoint_matches_oracle_convdiff16():
    import paper_2512_04389_amd as slu
    k = 16
    n, rp, ci, v = _convdiff(k, seed=11)
    announce("adjoint convdiff-16, 16 right-hand sides")
    rng = np.random.default_rng(4)
    B = rng.uniform(-1, 1, (n, 16))
    W = rng.uniform(-1, 1, (n, 16))
    lu = slu.SparseLU(n, rp, ci, ordering="grid_nd", grid_dims=(k, k, k)).bind()
    vals = torch.from_numpy(v).cuda().requires_grad_(True)
    Bt = torch.from_numpy(B).cuda().requires_grad_(True)
    X = slu.solve(lu, vals, Bt)
    loss = (X * torch.from_numpy(W).cuda()).sum()
    loss.backward()
    Xr, Gr, gvr = adjoint.solve_gradients(n, rp, ci, v, ordering.nd_grid((k, k, k)), B, W)
    assert _close(X.detach().cpu().numpy(), Xr)
    assert _close(Bt.grad.cpu().numpy(), Gr)
    assert _close(vals.grad.cpu().numpy(), gvr)


def test_adjoint_finite_differences_convdiff16():
    import paper_2512_04389_amd as slu
    k = 16
    n, rp, ci, v = _convdiff(k, seed=12)
    announce("adjoint finite differences convdiff-16")
    rng = np.random.default_rng(6)
    b = torch.from_numpy(rng.uniform(-1, 1, n)).cuda()
    w = torch.from_numpy(rng.uniform(-1, 1, n)).cuda()
    lu = slu.SparseLU(n, rp, ci, ordering="grid_nd", grid_dims=(k, k, k)).bind()
    vals = torch.from_numpy(v).cuda().requires_grad_(True)
    bb = b.clone().requires_grad_(True)
    (slu.solve(lu, vals, bb) * w).sum().backward()
    gv = vals.grad.cpu().numpy()
    gb = bb.grad.cpu().numpy()

    def loss(vv, b0):
        with torch.no_grad():
            return float((slu.solve(lu, vv, b0) * w).sum())

    for q in rng.choice(len(v), 8, replace=False):
        h = 1e-6 * max(1.0, abs(v[q]))
        vp = torch.from_numpy(v).cuda()
        vm = vp.clone()
        vp[q] += h
        vm[q] -= h
        fd = (loss(vp, b) - loss(vm, b)) / (2 * h)
        assert abs(fd - gv[q]) <= 1e-5 * max(1.0, abs(fd)), (q, fd, gv[q])
    v0 = torch.from_numpy(v).cuda()
    for i in rng.choice(n, 4, replace=False):
        bp, bm = b.clone(), b.clone()
        bp[i] += 1e-6
        bm[i] -= 1e-6
        fd = (loss(v0, bp) - loss(v0, bm)) / 2e-6
        assert abs(fd - gb[i]) <= 1e-5 * max(1.0, abs(fd))


def test_gradcheck_small():
    import paper_2512_04389_amd as slu
    n, rp, ci, v = _convdiff(3, seed=13)
    lu = slu.SparseLU(n, rp, ci, ordering="grid_nd", grid_dims=(3, 3, 3)).bind()
    vals = torch.from_numpy(v).cuda().requires_grad_(True)
    b = torch.from_numpy(np.random.default_rng(1).uniform(-1, 1, n)).cuda().requires_grad_(True)
    assert torch.autograd.gradcheck(lambda vv, bb: slu.solve(lu, vv, bb), (vals, b), eps=1e-6, atol=1e-7,
                                    rtol=1e-5)


def test_refactor_between_forward_and_backward():
    # backward factors the forward's values again when the handle moved on
    import paper_2512_04389_amd as slu
    n, rp, ci, v = _convdiff(3, seed=14)
    lu = slu.SparseLU(n, rp, ci, ordering="grid_nd", grid_dims=(3, 3, 3)).bind()
    b = torch.ones(n, dtype=torch.float64, device="cuda")
    v1 = torch.from_numpy(v).cuda().requires_grad_(True)
    slu.solve(lu, v1, b).sum().backward()
    v2 = torch.from_numpy(v).cuda().requires_grad_(True)
    x = slu.solve(lu, v2, b)
    lu.factor(torch.from_numpy(v * 2.0).cuda())
    x.sum().backward()
    assert torch.equal(v1.grad, v2.grad)
