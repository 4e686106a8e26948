"""fp_closure_nn_noalloc (the learned closure for callers that cannot allocate) against
fp_closure_nn through the C ABI: same kernels, so the records and statuses must be equal
bit for bit; two calls in a row, the second on a smaller context, each for the checked
(with exact fallback) and the unchecked form; and the refusal above the array's size."""
import numpy as np
import pytest
import torch

from oracle import mlp_oracle as M
from oracle import oracle as O
from paper_2606_15622_amd import inputs as I

pytestmark = pytest.mark.gpu


def fp():
    from paper_2606_15622_amd import fpgpu
    fpgpu.load()
    return fpgpu


def params(seed):
    rng = np.random.default_rng(seed)
    d = {}
    for name, shp in M.SHAPES:
        if name.startswith("W"):
            d[name] = rng.standard_normal(shp) / np.sqrt(shp[1])
        elif name.startswith("b") or name.endswith("mean"):
            d[name] = rng.standard_normal(shp) * 0.05
        elif name == "x_std":
            d[name] = rng.uniform(0.3, 1.5, shp)
        else:
            d[name] = rng.uniform(0.01, 0.1, shp)
    return torch.from_numpy(M.pack(d).astype(np.float32)).cuda()


def moments(ncell, seed):
    rng = np.random.default_rng(seed)
    counts = rng.integers(0, 200, ncell)
    vx, vy, vz, off = I.mixture_cells(counts, seed=seed)
    return torch.from_numpy(O.moments(off, vx, vy, vz)).cuda()


def run_pair(F, ncell, seed, pd):
    w = I.couette(ncell=ncell, eps_hat=0.01)
    ctx = F.Context(w, 1)
    net = F.Network(ctx, 0)
    net.load(pd)
    md = moments(ncell, seed)
    for tol in (0.05, float("inf")):
        r1 = torch.full((ncell, 16), 7.0, dtype=torch.float64, device="cuda")
        r2 = r1.clone()
        s1 = torch.zeros(ncell, dtype=torch.int32, device="cuda")
        s2 = torch.full_like(s1, -1)
        net.closure(md, r1, s1, tol, 0.05)
        net.closure_noalloc(md, r2, s2, tol, 0.05)
        torch.cuda.synchronize()
        assert torch.equal(s1, s2), (ncell, tol)
        assert torch.equal(r1, r2), (ncell, tol)
        st = s1.cpu().numpy()
        assert np.sum(st == F.CELL_EMPTY) > 0
        if tol == 0.05:
            assert np.sum(st == F.CELL_NN_FALLBACK) > 0
        else:
            assert np.sum(st == F.CELL_NN) > 0
    return ctx, net


def test_noalloc_equals_closure_nn_two_calls_smaller_second():
    F = fp()
    pd = params(1)
    run_pair(F, 20_011, 3, pd)
    run_pair(F, 1_237, 4, pd)


def test_noalloc_refuses_more_cells_than_its_array():
    F = fp()
    n = 262_144 + 1
    w = I.couette(ncell=n, eps_hat=0.01)
    ctx = F.Context(w, 1)
    net = F.Network(ctx, 0)
    net.load(params(2))
    md = torch.zeros((n, 32), dtype=torch.float64, device="cuda")
    rec = torch.zeros((n, 16), dtype=torch.float64, device="cuda")
    st = torch.zeros(n, dtype=torch.int32, device="cuda")
    with pytest.raises(RuntimeError, match="FP_NN_NOALLOC_CELLS"):
        net.closure_noalloc(md, rec, st, 0.05, 0.05)
