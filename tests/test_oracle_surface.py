"""Pins of the cylinder's wall-exchange sums and surface coefficients (oracle flight with
diffuse re-emission): a gas at rest around the body against the kinetic-theory fluxes
onto a diffuse wall, and a cold hypersonic beam against the free-molecular (Newtonian
plus diffuse re-emission) closed forms of C_p, C_f and C_h."""
import math

import numpy as np
import pytest

from oracle import diag_oracle as D
from oracle import oracle as O
from paper_2606_15622_amd import inputs as I


def body_world(T_gas, T_wall, U=0.0, dt=1e-6):
    w = I.cylinder(cell=1e-2, nx=60, ny=60, fnum=1.0, precision="f64", T_body=T_wall,
                   T_inf=T_gas, mach=1.0, dt=dt)
    w.update(x0=-0.3, y0=-0.3, lx=0.6, ly=0.6, u_inf=(U, 0.0, 0.0))
    return w


def annulus(rng, n, R, width):
    r = np.sqrt(rng.uniform(R * R, (R + width) ** 2, n))
    a = rng.uniform(-np.pi, np.pi, n)
    return r * np.cos(a), r * np.sin(a)


@pytest.mark.parametrize("ratio", [1.0, 2.0])
def test_gas_at_rest_fluxes(ratio):
    """Maxwellian gas at rest, density n and temperature T, around a diffuse wall at T_w:
    particle flux n sqrt(RT / 2 pi); pressure n k (T + sqrt(T T_w)) / 2; energy flux into
    the wall m n sqrt(RT / 2 pi) 2 R (T - T_w); no shear."""
    Tw = 300.0
    T = ratio * Tw
    w = body_world(T, Tw)
    R, Rg = w["circle"][2], I.KB / w["mass"]
    rng = np.random.default_rng(7)
    n_p, width = 2_000_000, 3e-3
    x, y = annulus(rng, n_p, R, width)
    s = math.sqrt(Rg * T)
    v = rng.standard_normal((3, n_p)) * s
    n = n_p / (math.pi * ((R + width) ** 2 - R * R) * w["depth"])
    wall = np.zeros((12, 4))
    O.move(w, x, y, v[0], v[1], v[2], np.arange(n_p, dtype=np.uint32), 0, wall=wall)
    A = 2 * math.pi * R * w["depth"]
    gam = n * math.sqrt(Rg * T / (2 * math.pi))
    hits = wall[:, 0].sum() / (A * w["dt"])
    p = w["mass"] * wall[:, 1].sum() / (A * w["dt"])
    tau = w["mass"] * wall[:, 2].sum() / (A * w["dt"])
    q = w["mass"] * wall[:, 3].sum() / (A * w["dt"])
    assert hits == pytest.approx(gam, rel=0.02)
    assert p == pytest.approx(n * I.KB * (T + math.sqrt(T * Tw)) / 2, rel=0.02)
    assert abs(tau) < 0.02 * p
    q_in = w["mass"] * gam * 2 * Rg * T
    assert q == pytest.approx(w["mass"] * gam * 2 * Rg * (T - Tw), abs=0.02 * q_in)


def test_cold_beam_newtonian_closed_forms():
    """Free-molecular cold beam along +x at U onto the diffuse cylinder: on the front half,
    with cos a = -cos(theta), C_p = 2 cos^2 a + 2 cos a sqrt(pi R T_w / 2) / U,
    C_f = 2 cos a sin a, C_h = cos a (1 - 4 R T_w / U^2); nothing on the rear half."""
    U, Tw, dt = 2624.0, 500.0, 1e-6
    w = body_world(1e-3, Tw, U=U, dt=dt)
    R, Rg = w["circle"][2], I.KB / w["mass"]
    rng = np.random.default_rng(8)
    n_p = 1_500_000
    # uniform upstream of the body, within reach of one step
    x0, x1 = -R - 1.5 * U * dt, 0.0
    x = rng.uniform(x0, x1, 6 * n_p)
    y = rng.uniform(-R, R, 6 * n_p)
    keep = x * x + y * y > R * R      # about a quarter of the rectangle is gas
    x, y = x[keep][:n_p], y[keep][:n_p]
    assert x.shape[0] == n_p
    gas_area = (x1 - x0) * 2 * R - math.pi * R * R / 2
    n = n_p / (gas_area * w["depth"])
    w["n_inf"] = n
    v = np.zeros((3, n_p))
    v[0] = U
    nb = 18
    wall = np.zeros((nb, 4))
    O.move(w, x, y, v[0], v[1], v[2], np.arange(n_p, dtype=np.uint32), 0, wall=wall)
    c = D.surface_coefficients(wall, dt, w)
    for b in range(nb):
        t = np.linspace(b * np.pi / nb, (b + 1) * np.pi / nb, 201)
        ca = np.clip(-np.cos(t), 0.0, None)
        sa = np.sin(t)
        cp = np.mean(2 * ca ** 2 + 2 * ca * math.sqrt(math.pi * Rg * Tw / 2) / U)
        cf = np.mean(2 * ca * sa)
        ch = np.mean(ca * (1 - 4 * Rg * Tw / U ** 2))
        if b < nb // 2:
            assert wall[b, 0] == 0 and c[b, 1] == pytest.approx(0.0, abs=1e-6)   # -p_inf term
            continue
        assert c[b, 0] == pytest.approx((b + 0.5) * 10.0)
        assert c[b, 1] == pytest.approx(cp, rel=0.03, abs=0.01), b
        assert c[b, 2] == pytest.approx(cf, rel=0.05, abs=0.01), b
        assert c[b, 3] == pytest.approx(ch, rel=0.03, abs=0.01), b
