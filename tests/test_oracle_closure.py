"""Pins of the oracle's 9x9 closure (CPU)."""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import oracle as O
from paper_2606_15622_amd import inputs as I
from tests.closure_exact import exact_system, solve_exact

S2 = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]


def _mom_of(v):
    v = np.asarray(v, dtype=np.float64)
    return O.moments(np.array([0, v.shape[0]], dtype=np.int32), v[:, 0], v[:, 1], v[:, 2])[0]


def test_table1_V_and_W_blocks_literal():
    """V and W of Table matrix_system, with the V entries read as second-order moments
    P_ij and the W entries as <c_i |c|^2>, appear verbatim in the stress rows."""
    vx, vy, vz, off = I.mixture_cells([300], seed=8)
    m = O.moments(off, vx, vy, vz)[0]
    A, b = O.closure_system(m, 0.0)
    th = m[4]
    P = lambda i, j: m[5 + S2.index((min(i, j), max(i, j)))] / th
    T = lambda q: m[11 + q] / th**1.5
    S = [T(0) + T(3) + T(5), T(1) + T(6) + T(8), T(2) + T(7) + T(9)]
    u = lambda i, j: P(i - 1, j - 1)
    u1 = lambda i: S[i - 1]
    V = np.array([
        [2 * u(1, 1), 2 * u(1, 2), 2 * u(1, 3), 0, 0, 0],
        [u(1, 2), u(2, 2) + u(1, 1), u(2, 3), u(1, 2), u(1, 3), 0],
        [u(1, 3), u(2, 3), u(3, 3) + u(1, 1), 0, u(1, 2), u(1, 3)],
        [0, 2 * u(1, 2), 0, 2 * u(2, 2), 2 * u(2, 3), 0],
        [0, u(1, 3), u(1, 2), u(2, 3), u(3, 3) + u(2, 2), u(2, 3)],
        [0, 0, 2 * u(1, 3), 0, 2 * u(2, 3), 2 * u(3, 3)]])
    W = np.array([
        [2 * u1(1), 0, 0], [u1(2), u1(1), 0], [u1(3), 0, u1(1)],
        [0, 2 * u1(2), 0], [0, u1(3), u1(2)], [0, 0, 2 * u1(3)]])
    np.testing.assert_allclose(A[:6, :6], V, rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(A[:6, 6:], W, rtol=1e-14, atol=1e-14)
    # with eps = 0 the stress right-hand side vanishes and the heat-flux one does not
    assert np.all(b[:6] == 0.0) and np.any(b[6:] != 0.0)


@pytest.mark.parametrize("seed,n", [(1, 5), (2, 6), (3, 9), (4, 12)])
def test_assembly_and_solution_match_exact_rational_construction(seed, n):
    rng = np.random.default_rng(seed)
    v = rng.integers(-3, 4, (n, 3)).tolist()
    tau = Fr(3, 7)
    eps_hat = Fr(1, 50)
    U = [Fr(sum(r[i] for r in v), n) for i in range(3)]
    theta = sum(sum((Fr(r[i]) - U[i]) ** 2 for i in range(3)) for r in v) / (3 * n)
    eps2 = eps_hat / (theta * tau)
    A, b, th2, _ = exact_system(v, tau, eps2)
    assert th2 == theta
    y = solve_exact(A, b)
    # oracle normalised system -> physical units
    m = _mom_of(v)
    An, bn = O.closure_system(m, float(eps_hat))
    t, th = float(tau), float(theta)
    rs = np.array([t / th] * 6 + [t / th**1.5] * 3)          # row scaling
    cs = np.array([t] * 6 + [t * math.sqrt(th)] * 3)          # column scaling
    Aex = np.array([[float(x) for x in row] for row in A])
    bex = np.array([float(x) for x in b])
    np.testing.assert_allclose(An, rs[:, None] * Aex / cs[None, :], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(bn, rs * bex, rtol=1e-12, atol=1e-12)
    yn = np.linalg.solve(An, bn)
    yex = np.array([float(q) for q in y])
    cond = np.linalg.cond(An)
    np.testing.assert_allclose(yn / cs, yex, rtol=cond * 1e-14, atol=cond * 1e-14 * np.abs(yex).max())


def _cfg_for_tau(m, tau_target):
    """Couette workload whose gas law gives tau_target for the cell record m."""
    w = I.couette(ncell=1, precision="f64")
    tau0, _ = O.cell_params(w, m)
    w["fnum_over_vol"] *= tau0 / tau_target      # tau is inversely proportional to density
    return w


def test_tau_at_the_reference_state():
    # argon at 273 K and n = 1.2954e22 m^-3 (Kn 0.1 on 1 mm): tau = 2 mu / (n k T) ~ 8.67e-7 s
    w = I.couette(kn=0.1, ncell=1, ppc=100)
    th = I.KB / I.MASS_AR * 273.0
    m = np.zeros(32); m[0] = 100; m[4] = th
    tau, eps2 = O.cell_params(w, m)
    assert w["n_number"] == pytest.approx(1.2954e22, rel=2e-4)
    assert tau == pytest.approx(8.67e-7, rel=2e-3)
    assert eps2 == pytest.approx(w["eps_hat"] / (th * tau), rel=1e-15)


def test_closure_matches_its_system_and_particle_space_identities():
    """The solved coefficients make the drift satisfy the moment conditions directly on
    the particles: sum_p (c N^T + N c^T) = 0 and <N_i |c|^2 + 2 c_i c.N> = 5 S_i/(3 tau)."""
    counts = [40, 200, 1000]
    vx, vy, vz, off = I.mixture_cells(counts, seed=21)
    mom = O.moments(off, vx, vy, vz)
    w = I.couette(ncell=3, precision="f64")
    rec, st = O.closure(w, mom)
    assert np.all(st == O.OR_OK)
    for c in range(3):
        m, r = mom[c], rec[c]
        v = np.stack([vx, vy, vz], 1)[off[c]:off[c + 1]]
        cc = v - m[1:4]
        c2 = (cc**2).sum(1)
        Ct = np.zeros((3, 3))
        for q, (i, j) in enumerate(S2):
            Ct[i, j] = Ct[j, i] = r[q]
        G = r[6:9]
        tau, th, eps2 = r[9], r[10], r[12]
        S = (cc * c2[:, None]).mean(0)
        N = cc @ Ct.T + G[None, :] * (c2 - 3 * th)[:, None] - eps2 * (cc * c2[:, None] - S)
        stress = (cc[:, :, None] * N[:, None, :] + N[:, :, None] * cc[:, None, :]).mean(0)
        scale_s = np.abs(cc @ Ct.T * cc).mean() + 1e-300
        np.testing.assert_allclose(stress, 0.0, atol=1e-11 * scale_s)
        heat = (N * c2[:, None]).mean(0) + 2 * (cc * (cc * N).sum(1)[:, None]).mean(0)
        np.testing.assert_allclose(heat, 5.0 / (3.0 * tau) * S, rtol=1e-9,
                                   atol=1e-11 * np.abs(N * c2[:, None]).mean())
        # energy: <c . N> = 0 for the exact closure
        assert abs((cc * N).sum(1).mean()) < 1e-11 * np.abs(cc * N).sum(1).mean()
        # the record agrees with the normalised system solved by a library routine
        An, bn = O.closure_system(m, w["eps_hat"])
        yn = np.linalg.solve(An, bn)
        np.testing.assert_allclose(r[:6] * tau, yn[:6], rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(r[6:9] * tau * math.sqrt(th), yn[6:], rtol=1e-10, atol=1e-12)
        assert r[11] == pytest.approx(math.exp(-w["dt"] / tau), rel=1e-15)
        assert r[13] == pytest.approx(math.sqrt(th * (1 - math.exp(-2 * w["dt"] / tau))), rel=1e-14)


@pytest.mark.parametrize("eps_hat", [0.0, 0.01, 0.2])
def test_maxwellian_gives_isotropic_coefficients(eps_hat):
    th = I.KB / I.MASS_AR * 273.0
    vx, vy, vz = I.gauss_hermite3_cell(th, drift=(10.0, 0.0, -4.0))
    m = O.moments(np.array([0, 216], dtype=np.int32), vx, vy, vz)
    w = I.couette(ncell=1, precision="f64", eps_hat=eps_hat)
    rec, st = O.closure(w, m)
    r = rec[0]
    tau = r[9]
    Ch = r[:6] * tau
    np.testing.assert_allclose(Ch, [5 * eps_hat, 0, 0, 5 * eps_hat, 0, 5 * eps_hat], atol=1e-12)
    np.testing.assert_allclose(r[6:9] * tau * math.sqrt(th), 0.0, atol=1e-12)


def test_axis_reflection_symmetric_cell():
    rng = np.random.default_rng(5)
    base = rng.standard_normal((40, 3)) * np.array([1.0, 1.6, 0.7]) * 300
    signs = np.array([[a, b, c] for a in (1, -1) for b in (1, -1) for c in (1, -1)])
    v = (base[None, :, :] * signs[:, None, :]).reshape(-1, 3)
    m = _mom_of(v)
    eh = 0.05
    A, b = O.closure_system(m, eh)
    y = np.linalg.solve(A, b)
    th = m[4]
    Ph = np.array([m[5], m[8], m[10]]) / th
    Rh = np.array([m[21], m[24], m[26]]) / th**2
    np.testing.assert_allclose(y[[0, 3, 5]], eh * Rh / Ph, rtol=1e-12)
    np.testing.assert_allclose(y[[1, 2, 4, 6, 7, 8]], 0.0, atol=1e-12)


def test_four_particle_cells_are_singular():
    """Four centred velocities span three directions: the 9x9 system has no unique
    solution, which is why cells need at least five particles (default n_min)."""
    import scipy.linalg as sl
    vx, vy, vz, off = I.mixture_cells([4] * 50 + [5] * 50, seed=4)
    mom = O.moments(off, vx, vy, vz)
    piv4 = [np.abs(np.diag(sl.lu_factor(O.closure_system(m, 0.01)[0])[0])).min() for m in mom[:50]]
    cond5 = [np.linalg.cond(O.closure_system(m, 0.01)[0]) for m in mom[50:]]
    assert np.median(piv4) < 1e-12
    assert max(cond5) < 1e9
    assert I.couette()["n_min"] == 5


def test_status_codes():
    w = I.couette(ncell=1, precision="f64", n_min=4)
    th = 1e4
    cells = [
        np.zeros((0, 3)),                                   # empty
        np.array([[1.0, 2.0, 3.0]]),                        # one particle
        np.array([[1.0, 2.0, 3.0]] * 5),                    # zero temperature
        np.array([[1.0, 0, 0], [-1.0, 0, 0], [0, 2.0, 0]]), # fewer than n_min
        np.array([[1.0, 0, 0], [-1.0, 0, 0], [2.0, 0, 0], [-2.0, 0, 0], [0.5, 0, 0]]),  # 1-D: singular
        np.array([[1.0, 0, 0], [np.nan, 0, 0], [2.0, 1, 0], [-2.0, 0, 1], [0.5, 0, 0]]),  # NaN
    ]
    counts = [c.shape[0] for c in cells]
    off = np.zeros(len(cells) + 1, dtype=np.int32)
    off[1:] = np.cumsum(counts)
    v = np.concatenate(cells, 0)
    mom = O.moments(off, v[:, 0] * th, v[:, 1] * th, v[:, 2] * th)
    rec, st = O.closure(w, mom)
    assert list(st) == [O.OR_EMPTY, O.OR_EMPTY, O.OR_EMPTY, O.OR_FEW, O.OR_SINGULAR, O.OR_NONFINITE]
    assert np.all(rec[:, 14] == st)
    # Langevin fallback rows carry no drift coefficients and no cubic term
    assert np.all(rec[3:5, :9] == 0.0) and np.all(rec[3:5, 12] == 0.0)
    assert rec[3, 11] < 1.0 and rec[3, 13] > 0.0
