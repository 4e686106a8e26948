"""What the trained surrogate gains over the method without a closure (Langevin drift).

A network is trained on the GPU by the library's MFMA kernels on Couette moment records
(Kn 0.1 and 0.5), then
  * on held-out Couette cells its normalised coefficients are compared with the exact
    ones; the Langevin drift corresponds to zero coefficients (relative error 1);
  * homogeneous cells carrying shear stress and heat flux relax under the exact closure,
    the pure network (no check, no fallback) and the Langevin drift: the closure sets the
    heat-flux relaxation rate to 4/(3 tau) (Pr = 2/3) where the Langevin drift gives
    3/tau, and the network must reproduce the closure's rate.
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
    mom = L.couette_dataset(kns=(0.1, 0.5), n_transient=300, n_samples=3000, seed=11)
    feats, tg, sys = L.dataset(I.couette(), mom)
    sc = L.fit_scalers(feats, tg)
    p0 = L.init_params(sc, seed=0)
    params, hist = L.train(I.couette(), p0, feats, tg, epochs=50, lr=1e-3, batch=4096,
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


def _relaxation_rates(params=None, langevin=False, cells=4000, ppc=500, steps=12, seed=21):
    """Homogeneous relaxation (collision only, no flight) of a Grad-type state with shear
    stress and heat flux in every cell; returns the decay rates of P_xy and S_x in units
    of 1/tau (fitted on the cell-averaged moments)."""
    import math
    from paper_2606_15622_amd import fpgpu as F
    w = I.couette(kn=0.1, ncell=cells, ppc=ppc, precision="f64", seed=seed)
    T = w["T_init"]
    mu = w["mu_ref"] * (T / w["T_ref"]) ** w["omega"]
    tau = 2.0 * mu / (w["n_number"] * w["kB"] * T)
    w = dict(w, dt=tau / 20.0, n_min=(1 << 30) if langevin else w["n_min"])
    sim = F.Simulation(w, I.grad_state(w, ppc, 0.08, 0.08, seed=seed))
    net = None
    if params is not None:
        net = F.Network(sim.ctx, 0)
        net.load(params)
    pxy, sx, taus = [], [], []
    for s in range(steps + 1):
        sim.sort(mom=sim.mom)
        m = sim.mom
        th = m[:, 4]
        pxy.append(float((m[:, 6] / th).mean()))
        sx.append(float(((m[:, 11] + m[:, 14] + m[:, 16]) / th ** 1.5).mean()))
        if net is not None:
            net.closure(sim.mom, sim.rec, sim.status, math.inf, 0.0)
        else:
            sim.ctx.closure_solve(sim.mom, sim.rec, sim.status)
        taus.append(float(sim.rec[:, 9].mean()))
        sim.ctx.step(sim.a, sim.offsets, sim.mom, sim.rec, s, F.STEP_COLLIDE)
    t = np.arange(steps + 1) * w["dt"] / np.mean(taus)
    rs = -np.polyfit(t, np.log(np.array(pxy) / pxy[0]), 1)[0]
    rq = -np.polyfit(t, np.log(np.array(sx) / sx[0]), 1)[0]
    return rs, rq


def test_network_restores_the_prandtl_number_of_the_closure(trained):
    """The closure's job is transport: with it the heat flux relaxes at 4/(3 tau)
    (Pr = 2/3), without it (Langevin drift) at 3/tau; the stress relaxes at 2/tau in
    both.  The network, run without any check or fallback, must land near the closure's
    rate, far from the Langevin one."""
    params, _ = trained
    rs_ex, rq_ex = _relaxation_rates()
    rs_nn, rq_nn = _relaxation_rates(params=params)
    rs_lan, rq_lan = _relaxation_rates(langevin=True)
    print(f"stress rate: exact {rs_ex:.3f} network {rs_nn:.3f} Langevin {rs_lan:.3f}; "
          f"heat-flux rate: exact {rq_ex:.3f} network {rq_nn:.3f} Langevin {rq_lan:.3f}")
    assert rq_ex == pytest.approx(4.0 / 3.0, rel=0.1)
    assert rq_lan == pytest.approx(3.0, rel=0.1)
    assert rs_ex == pytest.approx(2.0, rel=0.1) and rs_lan == pytest.approx(2.0, rel=0.1)
    assert abs(rq_nn - rq_ex) < 0.25 * abs(rq_lan - rq_ex), (rq_ex, rq_nn, rq_lan)
    assert rs_nn == pytest.approx(rs_ex, rel=0.1)
