"""Pins of the differentiable torch oracle (CPU, FP64)."""
import numpy as np
import pytest
import torch

from oracle import diff_oracle as D
from oracle import oracle as O
from paper_2606_15622_amd import inputs as I


def _setup(counts, seed, n_min=4):
    vx, vy, vz, off = I.mixture_cells(counts, seed=seed)
    w = I.couette(ncell=len(counts), eps_hat=0.01, n_min=n_min)
    v = np.stack([vx, vy, vz], 1)
    return w, v, off


def test_forward_matches_c_oracle():
    counts = [2, 3, 5, 40, 300, 1000]
    w, v, off = _setup(counts, 3)
    y = D.coefficients(torch.tensor(v), off, w).numpy()
    mom = O.moments(off, v[:, 0], v[:, 1], v[:, 2])
    rec, st = O.closure(w, mom)
    for c in range(len(counts)):
        if st[c] == O.OR_OK:
            sc = np.abs(rec[c, :9]).max()
            np.testing.assert_allclose(y[c], rec[c, :9], rtol=1e-9, atol=1e-11 * sc)
        else:
            assert np.all(y[c] == 0) and np.all(rec[c, :9] == 0)


def test_autograd_matches_central_differences():
    counts = [7, 25, 120]
    w, v, off = _setup(counts, 4)
    rng = np.random.default_rng(5)
    wts = rng.standard_normal((len(counts), 9))
    th = I.KB / I.MASS_AR * 273.0
    scale = np.array([1.0] * 6 + [np.sqrt(th)] * 3)  # balance Ct and Gamma magnitudes

    def L(vv):
        return (D.coefficients(vv, off, w) * torch.tensor(wts * scale)).sum()

    vt = torch.tensor(v, requires_grad=True)
    L(vt).backward()
    g = vt.grad.numpy()
    h = 1e-6 * np.sqrt(th)
    for p, a in [(0, 0), (3, 1), (10, 2), (40, 0), (100, 1), (151, 2)]:
        vp, vm = v.copy(), v.copy()
        vp[p, a] += h
        vm[p, a] -= h
        fd = (L(torch.tensor(vp)).item() - L(torch.tensor(vm)).item()) / (2 * h)
        assert g[p, a] == pytest.approx(fd, rel=1e-5, abs=1e-9 * np.abs(g).max()), (p, a)
