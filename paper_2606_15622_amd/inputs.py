"""Seeded synthetic workloads and particle generators.

This module is shared by the GPU path and the oracle as their common INPUT source.  It
holds none of the method's arithmetic (no moments, closure, update, flight or binning):
only the workload definitions (geometry, gas constants, time step, particle weight) and
seeded numpy generators of particle states.

Gas and regime follow the paper's test cases: argon (m = 66.3e-27 kg, mu_ref =
2.117e-5 Pa s; Sec. "Case Study 1: 1D Couette Flow"), diffuse isothermal walls at 273 K,
a Couette channel of 1 mm and a 1 mm lid-driven cavity (Sec. "Case Study 2").  The
supplementary table with the paper's full setup is not available, so the density is set
from the nominal Knudsen number through the VHS mean free path
    lambda = 2 (7 - 2w)(5 - 2w) / 15 * mu / (rho sqrt(2 pi R T))   (Bird 1994),
the cell size is 10 um and the time step is half a cell crossing at sqrt(2 R T).
"""
import math

import numpy as np

KB = 1.380649e-23
MASS_AR = 66.3e-27
MU_REF = 2.117e-5
T_REF = 273.0
OMEGA = 0.81


def _vhs_density(kn, length, T=T_REF, omega=OMEGA):
    """Number density giving mean free path kn * length (VHS, Bird 1994)."""
    R = KB / MASS_AR
    mu = MU_REF * (T / T_REF) ** omega
    lam = kn * length
    rho = 2.0 * (7.0 - 2.0 * omega) * (5.0 - 2.0 * omega) / 15.0 * mu / (
        lam * math.sqrt(2.0 * math.pi * R * T))
    return rho / MASS_AR


def _base(**kw):
    R = KB / MASS_AR
    w = dict(kB=KB, mass=MASS_AR, mu_ref=MU_REF, T_ref=T_REF, omega=OMEGA,
             eps_hat=0.01, n_min=5, max_bounces=8, pivot_tol=1e-12, conserve="exact",
             seed=1, x0=0.0, y0=0.0, T_init=273.0)
    w.update(kw)
    w["R"] = R
    return w


def couette(kn=0.1, ncell=100, ppc=100, length=1e-3, u_ratio=0.3, precision="f64",
            n_steps=1000, seed=1, **kw):
    """Planar Couette flow: walls at x = 0 and x = L moving along y at -U and +U with
    U / sqrt(2 R T) = u_ratio, both diffuse at 273 K; 1-D in space, 3-D in velocity."""
    R = KB / MASS_AR
    T = 273.0
    dx = length / ncell
    n = _vhs_density(kn, length)
    uw = u_ratio * math.sqrt(2.0 * R * T)
    w = _base(name=f"couette1d_kn{kn}", geometry="couette1d", precision=precision,
              nx=ncell, ny=1, lx=length, ly=1.0, dx=dx, dy=1.0,
              dt=0.5 * dx / math.sqrt(2.0 * R * T), kn=kn, ppc=ppc, n_number=n,
              fnum_over_vol=n / ppc, T_wall=[T, T, T, T],
              u_wall=[[0.0, -uw, 0.0], [0.0, uw, 0.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]],
              n_steps=n_steps, n_skip=n_steps // 2, seed=seed)
    w.update(kw)
    return w


def cavity(kn=1.0, ncell=100, ppc=100, cell=1e-5, lid=50.0, precision="f32", n_steps=5000,
           n_skip=3000, seed=1, kn_length=None, **kw):
    """Square lid-driven cavity of ncell x ncell cells of size ``cell``; the lid at y = L
    moves along +x at ``lid`` m/s; all walls diffuse at 273 K.  The density is the one
    of nominal Kn on the 1 mm cavity unless ``kn_length`` says otherwise."""
    R = KB / MASS_AR
    T = 273.0
    length = cell * ncell
    n = _vhs_density(kn, kn_length if kn_length is not None else 1e-3)
    w = _base(name=f"cavity2d_{ncell}x{ncell}_ppc{ppc}_kn{kn}", geometry="cavity2d",
              precision=precision, nx=ncell, ny=ncell, lx=length, ly=length, dx=cell, dy=cell,
              dt=0.5 * cell / math.sqrt(2.0 * R * T), kn=kn, ppc=ppc, n_number=n,
              fnum_over_vol=n / ppc, T_wall=[T, T, T, T],
              u_wall=[[0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [lid, 0.0, 0.0]],
              n_steps=n_steps, n_skip=n_skip, seed=seed)
    w.update(kw)
    return w


def cylinder(cell=2e-3, nx=400, ny=300, radius=0.1, mach=10.0, T_inf=200.0, n_inf=1e20,
             T_body=500.0, fnum=2.5e12, dt=5e-7, precision="f32", n_steps=10000, n_skip=5000,
             seed=1, **kw):
    """Hypersonic flow of argon past a circular cylinder (Sec. "hypersonic cylinder"):
    Mach 10 at 200 K, n = 1e20 m^-3, diffuse isothermal wall at 500 K, radius 0.1 m at
    the origin in the box [-0.3, 0.5] x [-0.3, 0.3] m (400 x 300 cells of 2 mm), open
    boundaries with free-stream inflow, 1 m depth.  fnum real molecules per particle
    gives about 160 particles per free-stream cell."""
    R = KB / MASS_AR
    a_inf = math.sqrt(5.0 / 3.0 * R * T_inf)
    u = mach * a_inf
    w = _base(name=f"cylinder2d_{nx}x{ny}_M{mach}", geometry="cylinder2d", precision=precision,
              nx=nx, ny=ny, x0=-0.3, y0=-0.3, lx=nx * cell, ly=ny * cell, dx=cell, dy=cell,
              dt=dt, circle=(0.0, 0.0, radius), T_body=T_body, n_inf=n_inf, u_inf=(u, 0.0, 0.0),
              T_inf=T_inf, fnum=fnum, depth=1.0, fnum_over_vol=fnum / (cell * cell),
              T_wall=[T_inf] * 4, u_wall=[[0.0] * 3] * 4, T_init=T_inf, n_steps=n_steps,
              n_skip=n_skip, seed=seed, ppc=n_inf * cell * cell / fnum)
    w.update(kw)
    return w


def freestream_state(w, seed=None):
    """Uniform free stream in the gas part of the cylinder domain: the expected number
    n_inf (box area - pi R^2) depth / fnum of particles, uniform positions (those falling
    inside the circle are redrawn), Maxwellian(u_inf, T_inf) velocities."""
    seed = int(w["seed"] if seed is None else seed)
    rng = np.random.default_rng(seed)
    cx, cy, rad = w["circle"]
    area = w["lx"] * w["ly"] - math.pi * rad * rad
    n = int(round(w["n_inf"] * area * w["depth"] / w["fnum"]))
    x = np.empty(n)
    y = np.empty(n)
    filled = 0
    while filled < n:
        m = n - filled
        xs = w["x0"] + rng.random(m) * w["lx"]
        ys = w["y0"] + rng.random(m) * w["ly"]
        ok = (xs - cx) ** 2 + (ys - cy) ** 2 > rad * rad
        k = int(ok.sum())
        x[filled:filled + k] = xs[ok]
        y[filled:filled + k] = ys[ok]
        filled += k
    s = math.sqrt(KB / MASS_AR * w["T_inf"])
    v = rng.standard_normal((3, n)) * s + np.asarray(w["u_inf"])[:, None]
    return dict(x=_round(w, x), y=_round(w, y), vx=_round(w, v[0]), vy=_round(w, v[1]),
                vz=_round(w, v[2]), pid=np.arange(n, dtype=np.uint32))


def ncells(w):
    return int(w["nx"]) * int(w["ny"])


# ---------------------------------------------------------------------------------------
def _round(w, a):
    return a.astype(np.float32).astype(np.float64) if w["precision"] == "f32" else a


def maxwellian_state(w, ppc=None, seed=None, T=None, drift=(0.0, 0.0, 0.0)):
    """ppc particles in every cell, positions uniform inside the cell, velocities
    Maxwellian at temperature T about ``drift``.  The particles are generated cell by
    cell, so the arrays come out grouped by cell.  Values are rounded to the storage
    precision.  Returns dict(x, y, vx, vy, vz, pid)."""
    ppc = int(w["ppc"] if ppc is None else ppc)
    seed = int(w["seed"] if seed is None else seed)
    T = float(w["T_init"] if T is None else T)
    rng = np.random.default_rng(seed)
    nx, ny = int(w["nx"]), int(w["ny"])
    nc = nx * ny
    n = nc * ppc
    cell = np.repeat(np.arange(nc, dtype=np.int64), ppc)
    kx = cell % nx
    ky = cell // nx
    x = w["x0"] + (kx + rng.random(n)) * w["dx"]
    if w["geometry"] == "couette1d":
        y = np.zeros(n)
    else:
        y = w["y0"] + (ky + rng.random(n)) * w["dy"]
    s = math.sqrt(KB / MASS_AR * T)
    v = rng.standard_normal((3, n)) * s
    out = dict(x=_round(w, x), y=_round(w, y), vx=_round(w, v[0] + drift[0]),
               vy=_round(w, v[1] + drift[1]), vz=_round(w, v[2] + drift[2]),
               pid=np.arange(n, dtype=np.uint32))
    return out


def grad_state(w, ppc, shear, heat, seed=0):
    """ppc particles in every cell of w, velocities from the Maxwellian at T_init weighted
    by 1 + shear c_x c_y / theta + heat (c_x / sqrt(theta)) (|c|^2 / (5 theta) - 1)
    (a Grad-type perturbation carrying shear stress P_xy and heat flux along x), drawn
    by rejection from the Maxwellian; positions at the cell centres.  The same state in
    every cell, independent draws."""
    rng = np.random.default_rng(seed)
    nx, ny = int(w["nx"]), int(w["ny"])
    nc = nx * ny
    n = nc * ppc
    th = KB / MASS_AR * float(w["T_init"])
    s = math.sqrt(th)
    kmax = 6.0
    bound = 1.0 + abs(shear) * kmax * kmax + abs(heat) * kmax * (kmax * kmax / 5.0 + 1.0)
    out = np.empty((0, 3))
    while out.shape[0] < n:
        m = 2 * (n - out.shape[0]) + 1000
        z = rng.standard_normal((m, 3))
        z = z[(np.abs(z) < kmax).all(axis=1)]
        phi = shear * z[:, 0] * z[:, 1] + heat * z[:, 0] * ((z * z).sum(1) / 5.0 - 1.0)
        keep = rng.random(z.shape[0]) * bound < np.maximum(1.0 + phi, 0.0)
        out = np.concatenate([out, z[keep]])
    v = out[:n] * s
    cell = np.repeat(np.arange(nc, dtype=np.int64), ppc)
    x = w["x0"] + (cell % nx + 0.5) * w["dx"]
    y = np.zeros(n) if w["geometry"] == "couette1d" else w["y0"] + (cell // nx + 0.5) * w["dy"]
    return dict(x=_round(w, x), y=_round(w, y), vx=_round(w, v[:, 0]), vy=_round(w, v[:, 1]),
                vz=_round(w, v[:, 2]), pid=np.arange(n, dtype=np.uint32),
                key=cell.astype(np.int32))


def scattered_state(w, n, seed=0, face_hits=0.05):
    """n particles at uniformly random positions over the domain (not grouped), a
    fraction of them placed exactly on cell faces or domain walls."""
    rng = np.random.default_rng(seed)
    x = w["x0"] + rng.random(n) * w["lx"]
    y = w["y0"] + rng.random(n) * w["ly"] if w["geometry"] != "couette1d" else np.zeros(n)
    m = rng.random(n) < face_hits
    x[m] = w["x0"] + rng.integers(0, int(w["nx"]) + 1, m.sum()) * w["dx"]
    if w["geometry"] != "couette1d":
        m2 = rng.random(n) < face_hits
        y[m2] = w["y0"] + rng.integers(0, int(w["ny"]) + 1, m2.sum()) * w["dy"]
    s = math.sqrt(KB / MASS_AR * w["T_init"])
    v = rng.standard_normal((3, n)) * s
    return dict(x=_round(w, x), y=_round(w, y), vx=_round(w, v[0]), vy=_round(w, v[1]),
                vz=_round(w, v[2]), pid=rng.permutation(n).astype(np.uint32))


def mixture_cells(counts, seed=0, theta=None, precision="f64"):
    """Velocities of cells with the given particle counts, grouped by cell.  Each cell
    draws from a two-component anisotropic Gaussian mixture (random mean offset up to
    0.5 sqrt(theta), axis temperatures 0.5..1.5 theta, weight 0.1..0.5) so that stress,
    heat flux and the higher moments are all non-zero.  Returns (vx, vy, vz, offsets)."""
    rng = np.random.default_rng(seed)
    theta = KB / MASS_AR * 273.0 if theta is None else theta
    counts = np.asarray(counts, dtype=np.int64)
    off = np.zeros(counts.shape[0] + 1, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    v = np.empty((3, int(off[-1])))
    st = math.sqrt(theta)
    for c, nc in enumerate(counts):
        if nc == 0:
            continue
        wgt = rng.uniform(0.1, 0.5)
        comp = rng.random(nc) < wgt
        for k, mask in enumerate((~comp, comp)):
            m = int(mask.sum())
            if m == 0:
                continue
            mean = rng.uniform(-0.5, 0.5, 3) * st
            temps = rng.uniform(0.5, 1.5, 3) * theta
            v[:, off[c]:off[c + 1]][:, mask] = (mean[:, None] + rng.standard_normal((3, m))
                                                * np.sqrt(temps)[:, None])
        v[:, off[c]:off[c + 1]] += rng.uniform(-300, 300, 3)[:, None]
    if precision == "f32":
        v = v.astype(np.float32).astype(np.float64)
    return v[0], v[1], v[2], off.astype(np.int32)


def gauss_hermite3_cell(theta, drift=(0.0, 0.0, 0.0)):
    """216 equal-weight particles on the tensor grid of the 3-point Gauss-Hermite rule
    (nodes -sqrt(3 theta), 0, +sqrt(3 theta) with multiplicities 1, 4, 1 per axis).
    The rule integrates polynomials up to degree 5 exactly against the Maxwellian."""
    a = math.sqrt(3.0 * theta)
    nodes = [-a] + [0.0] * 4 + [a]
    g = np.array([(p, q, r) for p in nodes for q in nodes for r in nodes], dtype=np.float64)
    g += np.asarray(drift)[None, :]
    return g[:, 0].copy(), g[:, 1].copy(), g[:, 2].copy()
