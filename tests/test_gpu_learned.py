"""What the trained surrogate gains over the method without a closure (Langevin drift).

A network is trained on the GPU by the library's MFMA kernels on Couette moment records
(Kn 0.1 and 0.5), then
  * on held-out Couette cells its normalised coefficients are compared with the exact
    ones; the Langevin drift corresponds to zero coefficients (relative error 1);
  * the Couette channel is run with the exact closure, the pure network (no fallback)
    and the Langevin drift.  The Langevin drift has Pr = 3/2 instead of 2/3 (the heat
    flux relaxes at 3/tau instead of 4/(3 tau)), so viscous heating raises the centre
    temperature about twice as much; the network must reproduce the cubic-FP rise.
"""
import numpy as np
import pytest
import torch

from paper_2606_15622_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def trained():
    from paper_2606_15622_amd import fpgpu as F
    from paper_2606_15622_amd import learned as L
    F.load()
    mom = L.couette_dataset(kns=(0.1, 0.5), n_transient=300, n_samples=1000, seed=11)
    feats, tg, sys = L.dataset(I.couette(), mom)
    sc = L.fit_scalers(feats, tg)
    p0 = L.init_params(sc, seed=0)
    params, hist = L.train(I.couette(), p0, feats, tg, epochs=40, lr=1e-3, batch=4096,
                           patience=8)
    return params, hist


def test_training_decreases_validation_loss(trained):
    params, hist = trained
    assert hist[-1] < 0.5 * hist[0]
    assert min(hist) < 0.7   # standardised MSE summed over 9 outputs; a constant gives 9


def test_heldout_coefficients_beat_the_langevin_drift(trained):
    from paper_2606_15622_amd import fpgpu as F
    from paper_2606_15622_amd import learned as L
    params, _ = trained
    mom = L.couette_dataset(kns=(0.3,), n_transient=300, n_samples=200, seed=99)
    n = mom.shape[0]
    wd = dict(I.couette(), nx=n, ny=1, lx=1e-5 * n)
    ctx = F.Context(wd, 1)
    net = F.Network(ctx, 0)
    net.load(params)
    rec_nn = torch.zeros((n, 16), dtype=torch.float64, device="cuda")
    rec_ex = torch.zeros_like(rec_nn)
    st = torch.zeros(n, dtype=torch.int32, device="cuda")
    net.closure(mom, rec_nn, st, 1e30, 0.0)
    assert bool((st == F.CELL_NN).all())
    ctx.closure_solve(mom, rec_ex, st)
    tn = torch.zeros((n, 16), dtype=torch.float32, device="cuda")
    te = torch.zeros_like(tn)
    ctx.nn_targets(rec_nn, n, tn)
    ctx.nn_targets(rec_ex, n, te)
    eh = I.couette()["eps_hat"]
    shift = torch.tensor([5 * eh, 0, 0, 5 * eh, 0, 5 * eh, 0, 0, 0], device="cuda")
    yn = (tn[:, :9] + shift).double().cpu().numpy()     # normalised coefficients
    ye = (te[:, :9] + shift).double().cpu().numpy()
    err_nn = np.linalg.norm(yn - ye) / np.linalg.norm(ye)
    assert err_nn < 0.5, err_nn   # Langevin (zero coefficients) has relative error 1


def _center_rise(params=None, langevin=False, seed=5, steps=2500, avg=2000):
    from paper_2606_15622_amd import learned as L
    w = I.couette(kn=0.1, ncell=100, ppc=100, precision="f64", seed=seed, n_skip=steps - avg)
    sim = L.LearnedSimulation(w, I.maxwellian_state(w), params=params, tol_abs=1e30, tol_rel=0.0,
                              langevin=langevin)
    sim.run(0, steps)
    f = L.fields(w, sim.samp)
    T = f["T"]
    return T[45:55].mean() - 0.5 * (T[:5].mean() + T[-5:].mean())


def test_network_reproduces_cubic_fp_viscous_heating(trained):
    params, _ = trained
    d_ex = _center_rise()
    d_nn = _center_rise(params=params)
    d_lan = _center_rise(langevin=True)
    print(f"centre temperature rise: exact {d_ex:.3f} K, network {d_nn:.3f} K, "
          f"Langevin {d_lan:.3f} K")
    # the closure matters here: without it the heat flux relaxes at 3/tau instead of
    # 4/(3 tau) and the channel heats more (measured 6.9 K vs 5.2 K); the run-to-run noise
    # of the rise over 2000 averaged steps is about 0.1 K
    assert d_lan > d_ex + 1.0
    assert abs(d_nn - d_ex) < 0.35 * abs(d_lan - d_ex), (d_ex, d_nn, d_lan)
