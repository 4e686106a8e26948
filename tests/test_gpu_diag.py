"""fp_diagnostics (averaged state, normalised stress and heat flux, covariance entropy
proxies) against the FP64 oracle oracle/diag_oracle.py, through the C ABI: sums of
mixture cells (with empty cells), the sums a cavity loop accumulates, and a small
cylinder domain (cut-cell densities).  Both sides are FP64 with different operation
orders (determinant, logarithms): 1e-9 of each quantity's scale; NaN where the oracle
has NaN."""
import numpy as np
import pytest
import torch

from oracle import diag_oracle as D
from oracle import oracle as O
from paper_2606_15622_amd import inputs as I

pytestmark = pytest.mark.gpu


def fp():
    from paper_2606_15622_amd import fpgpu
    fpgpu.load()
    return fpgpu


def run(F, ctx, samp, dens, mkB, ref):
    n = samp.shape[0]
    diag = torch.full((n, F.DIAG_STRIDE), -7.0, dtype=torch.float64, device="cuda")
    ctx.diagnostics(torch.from_numpy(np.ascontiguousarray(samp)).cuda(), *ref, diag)
    torch.cuda.synchronize()
    g = diag.cpu().numpy()
    o = D.diagnostics(samp, dens, mkB, *ref)
    assert np.array_equal(np.isnan(g), np.isnan(o))
    ok = ~np.isnan(o)
    scale = np.maximum(np.abs(o), 1.0)
    scale[:, 1] = np.maximum(np.abs(o[:, 1]), 1e-300)
    scale[:, 2:5] = np.maximum(np.abs(o[:, 2:5]), 1.0) + np.sqrt(np.nan_to_num(o[:, 5:6]))
    assert np.all(np.abs(g - o)[ok] <= 1e-9 * scale[ok])
    return g, o


def test_mixture_cells_and_empty_ones():
    F = fp()
    rng = np.random.default_rng(31)
    counts = rng.integers(4, 400, 300)
    counts[[0, 17, 200]] = 0
    counts[[5, 6]] = [1, 2]                            # singular covariance: D_G undefined
    vx, vy, vz, off = I.mixture_cells(counts, seed=31)
    vx = vx + 120.0                                    # a drift: U enters every conversion
    samp = O.sample(off, vx, vy, vz)
    samp = O.sample(off, vx, vy, vz, samp)
    w = I.couette(ncell=len(counts))
    ctx = F.Context(w, 1)
    g, o = run(F, ctx, samp, np.full(len(counts), w["fnum_over_vol"]), I.MASS_AR / I.KB,
               (300.0 * I.KB / I.MASS_AR, 1e22, 0.01))
    assert np.isnan(g[17, 2:20]).all() and (g[:, 20:] == 0).all()
    assert np.isnan(g[[5, 6], 17]).all() and np.isfinite(g[6, 5])
    assert np.nanmin(g[:, 17]) >= -1e-12


def test_cavity_loop_sums():
    F = fp()
    w = I.cavity(kn=1.0, ncell=24, ppc=80, precision="f32", seed=32)
    sim = F.Simulation(w, I.maxwellian_state(w))
    sim.run(0, 30, n_skip=10)
    torch.cuda.synchronize()
    samp = sim.samp.cpu().numpy()
    th = 273.0 * I.KB / I.MASS_AR
    run(F, sim.ctx, samp, np.full(samp.shape[0], w["fnum_over_vol"]), I.MASS_AR / I.KB,
        (th, w["n_number"], 0.0))


def test_cylinder_cut_cell_densities():
    F = fp()
    w = I.cylinder(cell=2e-2, nx=40, ny=30, fnum=2.5e14, precision="f64", seed=33)
    sim = F.OpenSimulation(w, I.freestream_state(w))
    sim.run(0, 12, n_skip=4)
    torch.cuda.synchronize()
    samp = sim.samp.cpu().numpy()
    vol = O.cell_volumes(w)
    full = w["dx"] * w["dy"] * w["depth"]
    dens = w["fnum"] / np.where(vol > 0, vol, full)
    th_inf = I.KB / I.MASS_AR * w["T_inf"]
    g, o = run(F, sim.ctx, samp, dens, I.MASS_AR / I.KB, (th_inf, w["n_inf"], 0.0))
    free = np.isfinite(o[:, 16]) & (np.abs(o[:, 2] - w["u_inf"][0]) < 0.05 * w["u_inf"][0])
    assert free.sum() > 100


def test_high_order_fields_match_oracle():
    """fp_sample_high over two steps' moment records (mixture cells, some empty) and
    fp_high_order against the oracle: the same products, sums and quotients in the same
    order, so the same bits; NaN where the oracle has NaN."""
    F = fp()
    rng = np.random.default_rng(5)
    ncell = 1000 + 37
    w = I.couette(ncell=ncell, eps_hat=0.01)
    ctx = F.Context(w, 1)
    hs = torch.zeros((ncell, 16), dtype=torch.float64, device="cuda")
    ho = None
    for step in range(2):
        counts = rng.integers(0, 60, ncell)
        counts[::17] = 0
        vx, vy, vz, off = I.mixture_cells(counts, seed=20 + step)
        mom = O.moments(off, vx, vy, vz)
        ctx.sample_high(torch.from_numpy(mom).cuda(), hs)
        ho = D.sample_high(mom, ho)
    out = torch.full((ncell, 8), -7.0, dtype=torch.float64, device="cuda")
    ctx.high_order(hs, out)
    torch.cuda.synchronize()
    g = hs.cpu().numpy()
    np.testing.assert_array_equal(g[:, :10], ho[:, :10])
    assert np.all(g[:, 10:] == 0)
    go, oo = out.cpu().numpy(), D.high_order(ho)
    assert np.array_equal(np.isnan(go), np.isnan(oo)) and np.isnan(oo).any()
    np.testing.assert_array_equal(np.nan_to_num(go), np.nan_to_num(oo))
