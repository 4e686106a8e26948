"""The LITE learned closure (the paper's speed mechanism: moments through third order only,
the high-order gather skipped, the network unchecked) and the temporal under-relaxation of
the network's coefficients, through the C ABI.

* A context with moment_order 3 gathers N, U, theta, P and T exactly as the full gather
  does (same operations, same order: bit for bit) and writes R, W, H as zero, in the
  first sort (fp_bin + fp_moments) and in the re-sort (fp_rebin with mom); against the
  oracle's moments of the oracle-sorted cells to 1e-10 of the natural scale.
* Such a context refuses the exact closure and the checked learned closure.
* relax blends the network's coefficients with the previous record's: checked bit for
  bit against C = relax C_net + (1 - relax) C_prev evaluated in FP64 on the host.
* The LITE loop runs: finite, every particle kept, every solved cell from the network.
"""
import math

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


def random_params(seed=0):
    rng = np.random.default_rng(seed)
    d = {}
    for name, shp in M.SHAPES:
        if name.startswith("W"):
            d[name] = rng.standard_normal(shp) / np.sqrt(shp[1])
        elif name.startswith("b"):
            d[name] = rng.standard_normal(shp) * 0.1
        elif name in ("x_mean", "y_mean"):
            d[name] = np.zeros(shp)
        elif name == "x_std":
            d[name] = np.full(shp, 2.0)
        else:
            d[name] = np.full(shp, 0.02)
    return torch.tensor(M.pack(d), dtype=torch.float32, device="cuda")


def moment_scale(o):
    th = np.maximum(o[:, 4], 1e-300)
    scale = np.ones(o.shape)
    scale[:, 1:4] = np.sqrt(th)[:, None] + np.abs(o[:, 1:4])
    scale[:, 4:11] = th[:, None]
    scale[:, 11:21] = th[:, None] ** 1.5
    return scale


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_low_order_records_equal_the_first_entries_of_the_full_ones(prec):
    F = fp()
    w = I.cavity(kn=1.0, ncell=30, ppc=80, precision=prec, seed=21)
    s = I.maxwellian_state(w)
    full = F.Simulation(w, s)
    low = F.Simulation(dict(w, moment_order=3), s)
    for rep in range(3):               # fp_bin + fp_moments, then fp_rebin with mom twice
        for sim in (full, low):
            sim.sort(mom=sim.mom, samp=sim.samp)
        torch.cuda.synchronize()
        mf, ml = full.mom.cpu().numpy(), low.mom.cpu().numpy()
        np.testing.assert_array_equal(ml[:, :21], mf[:, :21], err_msg=f"sort {rep}")
        assert np.all(ml[:, 21:] == 0.0)
        np.testing.assert_array_equal(low.samp.cpu().numpy(), full.samp.cpu().numpy())
        a = low.a.numpy()
        o = O.moments(low.offsets.cpu().numpy(), a["vx"], a["vy"], a["vz"])
        assert np.all(np.abs(ml[:, :21] - o[:, :21]) <= 1e-10 * moment_scale(o)[:, :21])
        # move the particles so that the next sort is a real re-sort (Langevin drift from
        # the full context's closure records; the same update on both)
        full.ctx.closure_solve(full.mom, full.rec, full.status)
        for sim in (full, low):
            sim.ctx.step(sim.a, sim.offsets, full.mom, full.rec, rep, F.STEP_COLLIDE | F.STEP_MOVE)


def test_low_order_context_refuses_the_exact_and_the_checked_closure():
    F = fp()
    w = dict(I.cavity(kn=1.0, ncell=10, ppc=50), moment_order=3)
    sim = F.Simulation(w, I.maxwellian_state(w))
    sim.sort(mom=sim.mom)
    with pytest.raises(RuntimeError):
        sim.ctx.closure_solve(sim.mom, sim.rec, sim.status)
    net = F.Network(sim.ctx, 0)
    net.load(random_params())
    with pytest.raises(RuntimeError):
        net.closure(sim.mom, sim.rec, sim.status, 0.05, 0.05)
    net.closure(sim.mom, sim.rec, sim.status, math.inf, 0.0)
    torch.cuda.synchronize()
    st = sim.status.cpu().numpy()
    assert np.all((st == F.CELL_NN) | (st == F.CELL_EMPTY) | (st == F.CELL_FEW))
    assert np.isfinite(sim.rec.cpu().numpy()).all()
    with pytest.raises(RuntimeError):
        F.Context(dict(w, moment_order=4), 1)


def test_relax_blends_network_coefficients_with_the_previous_ones():
    F = fp()
    rng = np.random.default_rng(22)
    counts = rng.integers(10, 300, 200)
    counts[[3, 50]] = [0, 1]                          # empty cells: no coefficients
    vx, vy, vz, off = I.mixture_cells(counts, seed=22)
    mom = torch.from_numpy(O.moments(off, vx, vy, vz)).cuda()
    n = mom.shape[0]
    w = I.couette(ncell=n)
    ctx = F.Context(w, 1)
    net = F.Network(ctx, 0)
    net.load(random_params(3))
    rec0 = torch.zeros((n, F.REC_STRIDE), dtype=torch.float64, device="cuda")
    st = torch.zeros(n, dtype=torch.int32, device="cuda")
    ctx.closure_solve(mom, rec0, st)
    rec0[7, 14] = float(F.CELL_EMPTY)                 # a previous record without coefficients
    ra, rb = rec0.clone(), rec0.clone()
    net.closure(mom, ra, st, math.inf, 0.0, 1.0)
    net.closure(mom, rb, st, math.inf, 0.0, 0.2)
    torch.cuda.synchronize()
    a, b, p = ra.cpu().numpy(), rb.cpu().numpy(), rec0.cpu().numpy()
    s = st.cpu().numpy()
    blend = (s == F.CELL_NN) & np.isin(p[:, 14], [F.CELL_OK, F.CELL_NN, F.CELL_NN_FALLBACK])
    assert blend.sum() > 150 and not blend[7]
    expect = a.copy()
    expect[blend, :9] = 0.2 * a[blend, :9] + (1.0 - 0.2) * p[blend, :9]
    np.testing.assert_array_equal(b, expect)
    with pytest.raises(RuntimeError):
        net.closure(mom, rb, st, math.inf, 0.0, 0.0)


def test_lite_loop_runs_with_every_solved_cell_from_the_network():
    F = fp()
    from paper_2606_15622_amd import learned as L
    w = I.cavity(kn=1.0, ncell=20, ppc=60, precision="f32", seed=23)
    s = I.maxwellian_state(w)
    sim = L.LearnedSimulation(w, s, params=random_params(4), lite=True, relax=0.5)
    n0 = s["x"].shape[0]
    for k in range(12):
        sim.step(k, sample=k >= 6)
    torch.cuda.synchronize()
    st = sim.status.cpu().numpy()
    assert np.all((st == F.CELL_NN) | (st == F.CELL_FEW) | (st == F.CELL_EMPTY))
    assert (st == F.CELL_NN).sum() > 300
    a = sim.a.numpy()
    assert a["x"].shape[0] == n0 and int(sim.offsets[-1]) == n0
    assert all(np.isfinite(a[k]).all() for k in ("x", "y", "vx", "vy", "vz"))
    assert np.isfinite(sim.samp.cpu().numpy()).all()
