"""Pins of the oracle's open cylinder domain (configuration 5 geometry) (CPU)."""
import math

import numpy as np
import pytest
from scipy import special, stats

from oracle import oracle as O
from paper_2606_15622_amd import inputs as I


def small(**kw):
    # 80 x 60 cells of 10 mm: the same box and cylinder, coarse
    return I.cylinder(cell=1e-2, nx=80, ny=60, fnum=2.5e14, precision="f64", **kw)


def test_cut_cell_volumes_sum_and_symmetry():
    w = I.cylinder(precision="f64")
    vol = O.cell_volumes(w).reshape(w["ny"], w["nx"])
    R = w["circle"][2]
    full = w["dx"] * w["dy"]
    assert vol.sum() == pytest.approx(w["lx"] * w["ly"] - math.pi * R * R, rel=1e-12)
    assert vol.max() == pytest.approx(full, rel=1e-15) and vol.min() == 0.0
    # the circle is centred on a grid node (x0 = -0.3 = -150 dx): 4-fold symmetry
    ix0, iy0 = 150, 150
    q1 = vol[iy0:iy0 + 60, ix0:ix0 + 60]
    q2 = vol[iy0 - 60:iy0, ix0:ix0 + 60][::-1, :]
    q3 = vol[iy0:iy0 + 60, ix0 - 60:ix0][:, ::-1]
    np.testing.assert_allclose(q1, q2, rtol=0, atol=1e-13 * full)
    np.testing.assert_allclose(q1, q3, rtol=0, atol=1e-13 * full)
    np.testing.assert_allclose(q1, q1.T, rtol=0, atol=1e-13 * full)
    n_inactive = int((vol == 0).sum())
    assert 0 < n_inactive < math.pi * (R / w["dx"]) ** 2


def test_cut_cell_volume_against_fine_midpoint_rule():
    w = I.cylinder(precision="f64")
    vol = O.cell_volumes(w).reshape(w["ny"], w["nx"])
    R = w["circle"][2]
    rng = np.random.default_rng(0)
    cut = np.argwhere((vol > 0) & (vol < w["dx"] * w["dy"]))
    for ky, kx in cut[rng.choice(len(cut), 5, replace=False)]:
        m = 2000
        xs = w["x0"] + (kx + (np.arange(m) + 0.5) / m) * w["dx"]
        ys = w["y0"] + (ky + (np.arange(m) + 0.5) / m) * w["dy"]
        X, Y = np.meshgrid(xs, ys)
        outside = (X * X + Y * Y > R * R).mean() * w["dx"] * w["dy"]
        assert vol[ky, kx] == pytest.approx(outside, abs=2e-3 * w["dx"] * w["dy"])


def test_circle_reemission_distribution_ks():
    w = small()
    n = 20000
    R = w["circle"][2]
    # particles just outside the front stagnation point moving into the body
    x = np.full(n, -R - 1e-9)
    y = np.zeros(n)
    vx = np.full(n, 3000.0)
    vy = np.zeros(n)
    vz = np.zeros(n)
    pid = np.arange(n, dtype=np.uint32)
    x1, y1, ux, uy, uz, key = O.move(w, x, y, vx, vy, vz, pid, step=3)
    RT = I.KB / I.MASS_AR * w["T_body"]
    # normal at the hit point is -x: re-emitted speed along -x is Rayleigh
    assert np.all(ux < 0)
    assert stats.kstest(-ux, lambda v: 1 - np.exp(-v * v / (2 * RT))).pvalue > 1e-3
    assert stats.kstest(uy / math.sqrt(RT), "norm").pvalue > 1e-3
    assert stats.kstest(uz / math.sqrt(RT), "norm").pvalue > 1e-3
    assert np.all(x1 * x1 + y1 * y1 >= R * R * (1 - 1e-12))


def test_exit_deletes_and_keys_mark_it():
    w = small()
    nc = w["nx"] * w["ny"]
    x = np.array([0.499, -0.299, 0.0])
    y = np.array([0.0, 0.0, 0.299])
    vx = np.array([1e4, -1e4, 0.0])
    vy = np.array([0.0, 0.0, 1e4])
    x1, y1, ux, uy, uz, key = O.move(w, x, y, vx, vy, np.zeros(3), np.arange(3, dtype=np.uint32), 0)
    assert list(key) == [nc, nc, nc]
    perm, off = O.bin_particles(nc, key)
    assert off[-1] == 0


def _one_sided_flux(n, u_n, RT):
    """Particles per unit area and time crossing a plane from a drifting Maxwellian."""
    c = math.sqrt(2 * RT)
    s = u_n / c
    return n * (c / (2 * math.sqrt(math.pi)) * math.exp(-s * s) + u_n / 2 * (1 + special.erf(s)))


def test_injection_matches_equilibrium_influx():
    w = small(mach=3.0)
    RT = I.KB / I.MASS_AR * w["T_inf"]
    u = w["u_inf"][0]
    depth = w["depth"]
    # influx per step: left face (u_n = u), top and bottom (u_n = 0), right face (u_n = -u)
    per_step = (_one_sided_flux(w["n_inf"], u, RT) * w["ly"] + 2 * _one_sided_flux(w["n_inf"], 0.0, RT)
                * w["lx"] + _one_sided_flux(w["n_inf"], -u, RT) * w["ly"]) * depth * w["dt"] / w["fnum"]
    pn = 0
    total = 0
    steps = 200
    for s in range(steps):
        a, pn = O.inject(w, s, pn)
        total += a["x"].shape[0]
        assert np.all((a["x"] >= w["x0"]) & (a["x"] <= w["x0"] + w["lx"]))
    expected = per_step * steps
    assert total == pytest.approx(expected, rel=4 * math.sqrt(expected) / expected + 1e-3)


def test_empty_domain_keeps_the_free_stream():
    """No body (radius 0): inflow and outflow balance, the gas stays uniform."""
    w = small(mach=3.0, radius=0.0)
    s = I.freestream_state(w, seed=3)
    s["key"] = O.keys(w, s["x"], s["y"])
    n0 = s["x"].shape[0]
    out, pn, mom, rec, st, samp = O.run_open(w, s, n0, 0, 30, capacity=3 * n0, n_skip=10)
    n1 = out["x"].shape[0]
    assert abs(n1 - n0) < 5 * math.sqrt(n0)
    N = samp[:, 0] / 20
    assert abs(N.mean() - n0 / (w["nx"] * w["ny"])) < 0.02 * N.mean()
    U = samp[:, 1].sum() / samp[:, 0].sum()
    assert U == pytest.approx(w["u_inf"][0], rel=5e-3)
    np.testing.assert_array_equal(np.sort(out["pid"])[:0], [])
    assert len(np.unique(out["pid"])) == n1
