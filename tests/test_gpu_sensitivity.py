"""Coefficient-sensitivity probe on the GPU (fp_nn_sensitivity) against the FP64 oracle.

Both sides draw the same dropout masks (Philox, same counters), so the passes agree up to
the BF16 inference arithmetic; the oracle rounds weights, inputs and hidden activations
to bfloat16 where the GPU stores them in that format.  What remains is FP32 versus FP64
accumulation and the rare bfloat16 rounding flips it causes, each one ulp (2^-8
relative) of one activation; the standard deviation over the passes is of the size of
the outputs themselves (a fifth of the units dropped), so relative L2 2e-2 on the
sensitivity fields bounds those flips with margin, as for plain inference."""
import numpy as np
import pytest
import torch

from oracle import mlp_oracle as M
from paper_2606_15622_amd import inputs as I
from tests.test_gpu_nn import cells, dev, fp, random_params, rel_l2

pytestmark = pytest.mark.gpu


def run(F, ctx, net, mom, npass, p, seed):
    md = dev(mom, torch.float64)
    sens = torch.full((mom.shape[0], 2), -1.0, dtype=torch.float64, device="cuda")
    net.sensitivity(md, npass, p, seed, sens)
    torch.cuda.synchronize()
    return sens.cpu().numpy()


@pytest.mark.parametrize("nc,npass,p", [(1000 + 17, 12, 0.2), (64 * 3 + 5, 50, 0.2), (31, 5, 0.5)])
def test_sensitivity_matches_oracle(nc, npass, p):
    F = fp()
    mom = cells(nc, 11)
    mom[5] = 0
    mom[5, 0] = 1                      # one particle: no features, zeros
    w = I.couette(ncell=nc, eps_hat=0.01)
    ctx = F.Context(w, 1)
    net = F.Network(ctx, 0)
    pflat = M.pack(random_params(7)).astype(np.float32)
    net.load(dev(pflat, torch.float32))
    seed = (3 << 32) | 77
    g = run(F, ctx, net, mom, npass, p, seed)
    o = M.dropout_sensitivity(pflat.astype(np.float64), mom, 0.01, npass, p, seed)
    assert np.all(g[5] == 0.0)
    assert np.all(np.isfinite(g))
    valid = np.ones(nc, bool)
    valid[5] = False
    assert np.all(g[valid] > 0.0)
    for k in range(2):
        assert rel_l2(g[valid, k], o[valid, k]) < 2e-2, k


def test_sensitivity_degenerate_cases_are_exactly_zero():
    """No dropout, or a single pass: every pass equals the first, the deviations the GPU
    sums are exactly zero."""
    F = fp()
    nc = 300
    mom = cells(nc, 12)
    w = I.couette(ncell=nc, eps_hat=0.01)
    ctx = F.Context(w, 1)
    net = F.Network(ctx, 0)
    net.load(dev(M.pack(random_params(8)).astype(np.float32), torch.float32))
    assert np.all(run(F, ctx, net, mom, 20, 0.0, 5) == 0.0)
    assert np.all(run(F, ctx, net, mom, 1, 0.4, 5) == 0.0)
    with pytest.raises(RuntimeError):
        run(F, ctx, net, mom, 0, 0.2, 5)
    with pytest.raises(RuntimeError):
        run(F, ctx, net, mom, 4, 1.0, 5)


def test_sensitivity_at_the_cylinder_mesh_size_sampled():
    """1.2e5 cells (the 400 x 300 cylinder mesh), 50 passes at p = 0.2 as in the paper's
    probe: 400 sampled cells against the oracle evaluated for those cells alone."""
    F = fp()
    nc = 400 * 300
    rng = np.random.default_rng(13)
    mom = np.zeros((nc, 32))             # random central-moment records (valid features)
    mom[:, 0] = rng.uniform(20, 400, nc)
    mom[:, 1:4] = rng.standard_normal((nc, 3))
    mom[:, 4] = rng.uniform(0.5, 2.0, nc)
    mom[:, 5:32] = rng.standard_normal((nc, 27)) * 0.1
    for q in (5, 8, 10):
        mom[:, q] += mom[:, 4]
    for q in (21, 24, 26):
        mom[:, q] += 5 * mom[:, 4] ** 2
    w = I.couette(ncell=nc, eps_hat=0.01)
    ctx = F.Context(w, 1)
    net = F.Network(ctx, 0)
    pflat = M.pack(random_params(9)).astype(np.float32)
    net.load(dev(pflat, torch.float32))
    seed = (11 << 32) | 5
    g = run(F, ctx, net, mom, 50, 0.2, seed)
    pick = np.sort(np.random.default_rng(2).choice(nc, 400, replace=False))
    o = M.dropout_sensitivity(pflat.astype(np.float64), mom[pick], 0.01, 50, 0.2, seed, cells=pick)
    assert np.all(np.isfinite(g)) and np.all(g > 0)
    for k in range(2):
        assert rel_l2(g[pick, k], o[:, k]) < 2e-2, k
