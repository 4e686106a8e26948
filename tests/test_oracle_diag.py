"""Pins of the diagnostics oracle (oracle/diag_oracle.py), independent of its code:
  * a cell whose sums come from particles: U, Theta and <c_i |c|^2> against direct
    averages of the particles' peculiar velocities (brute force, no raw-sum algebra);
  * isotropic covariance: D_G = 0; diagonal covariance diag(a, b, c): D_G = -1/2 sum of
    log(a_i / theta) (closed form); D_G >= 0 for random positive-definite covariances
    (the Gaussian relative entropy is non-negative);
  * ds_eq = 0 at the reference state and 3/2 log 2 at twice its temperature;
  * empty cells: NaN state, zero particles per sample."""
import numpy as np

from oracle import diag_oracle as D


def sums_of(v, nsamp=1):
    """Cumulative sums of one cell, repeated nsamp times, from particle velocities v."""
    s = np.zeros(16)
    s[0] = len(v) * nsamp
    s[1:4] = v.sum(0) * nsamp
    for q, (i, j) in enumerate(D.S2):
        s[4 + q] = (v[:, i] * v[:, j]).sum() * nsamp
    s[10:13] = (v * (v * v).sum(1)[:, None]).sum(0) * nsamp
    s[13] = nsamp
    return s


def test_state_and_heat_flux_against_direct_particle_averages():
    rng = np.random.default_rng(1)
    v = rng.standard_normal((4000, 3)) * [300.0, 200.0, 250.0] + [50.0, -20.0, 5.0]
    v[:, 0] += 0.002 * v[:, 1] ** 2          # skewed: non-zero heat flux
    out = D.diagnostics(sums_of(v, 3)[None], np.array([2.0]), 4.8e-3, 1.0, 1.0, 0.0)[0]
    c = v - v.mean(0)
    Th = c.T @ c / len(c)
    theta = np.trace(Th) / 3
    qh = (c * (c * c).sum(1)[:, None]).mean(0) / (2 * theta ** 1.5)
    np.testing.assert_allclose(out[2:5], v.mean(0), rtol=1e-12)
    np.testing.assert_allclose(out[5], theta, rtol=1e-10)
    assert out[0] == 4000 and out[1] == 8000
    for q, (i, j) in enumerate(D.S2):
        np.testing.assert_allclose(out[7 + q], Th[i, j] / theta - (i == j), atol=1e-9)
    np.testing.assert_allclose(out[13:16], qh, rtol=1e-7, atol=1e-9)
    np.testing.assert_allclose(out[19], qh @ qh / 5, rtol=1e-7)


def cell_with_covariance(Th, U=(0.0, 0.0, 0.0), n=1.0):
    """Sums of a cell with exactly the given mean and covariance (no third moment)."""
    U = np.asarray(U, dtype=float)
    s = np.zeros(16)
    s[0], s[13] = n, 1.0
    s[1:4] = n * U
    for q, (i, j) in enumerate(D.S2):
        s[4 + q] = n * (Th[i, j] + U[i] * U[j])
    theta = np.trace(Th) / 3
    s[10:13] = n * (U * (U @ U) + 3 * theta * U + 2 * Th @ U)
    return s


def test_gaussian_entropy_deficit_closed_forms():
    iso = cell_with_covariance(np.eye(3) * 7.0, U=(3.0, -1.0, 2.0))
    out = D.diagnostics(iso[None], np.array([1.0]), 1.0, 7.0, 1.0, 0.0)[0]
    assert abs(out[17]) < 1e-14 and abs(out[16]) < 1e-14 and abs(out[19]) < 1e-20
    a = np.array([2.0, 5.0, 11.0])
    out = D.diagnostics(cell_with_covariance(np.diag(a))[None], np.array([1.0]), 1.0, 1.0, 1.0,
                        0.25)[0]
    theta = a.mean()
    np.testing.assert_allclose(out[17], -0.5 * np.log(a / theta).sum(), rtol=1e-13)
    np.testing.assert_allclose(out[18], out[16] - (out[17] - 0.25), rtol=1e-13)
    rng = np.random.default_rng(2)
    for _ in range(50):
        A = rng.standard_normal((3, 3))
        out = D.diagnostics(cell_with_covariance(A @ A.T + 0.1 * np.eye(3))[None],
                            np.array([1.0]), 1.0, 1.0, 1.0, 0.0)[0]
        assert out[17] >= -1e-12


def test_equilibrium_entropy_reference_and_empty_cells():
    s = np.stack([cell_with_covariance(np.eye(3) * 4.0, n=10.0),
                  cell_with_covariance(np.eye(3) * 8.0, n=10.0), np.zeros(16)])
    s[2, 13] = 1.0
    out = D.diagnostics(s, np.array([0.5, 0.5, 0.5]), 1.0, 4.0, 5.0, 0.0)
    assert abs(out[0, 16]) < 1e-14
    np.testing.assert_allclose(out[1, 16], 1.5 * np.log(2.0), rtol=1e-14)
    assert out[2, 0] == 0.0 and np.isnan(out[2, 2:20]).all() and (out[2, 20:] == 0).all()


def test_singular_covariance_has_no_entropy_deficit():
    """Two particles span one direction: det(Theta/theta) = 0 exactly, D_G undefined."""
    v = np.array([[300.0, 100.0, -50.0], [-100.0, 20.0, 70.0]])
    out = D.diagnostics(sums_of(v)[None], np.array([1.0]), 1.0, 1.0, 1.0, 0.0)[0]
    assert np.isfinite(out[5]) and out[5] > 0
    assert np.isnan(out[17]) and np.isnan(out[18]) and np.isfinite(out[16])


def test_high_order_fields_maxwellian_and_brute_force():
    """Normalised high-order fields: a Maxwellian cell gives R_ij,norm = 5 delta_ij,
    Delta_4,norm = 0, DM6_norm = 105 (Gaussian moments <|c|^4> = 15 theta^2,
    <|c|^6> = 105 theta^3) within sampling error; and the sums over steps equal brute-force
    particle averages written out directly."""
    from oracle import oracle as O
    rng = np.random.default_rng(3)
    n, steps = 400_000, 3
    h = None
    for s in range(steps):
        v = rng.standard_normal((n, 3)) * 2.0 + np.array([1.0, -2.0, 0.5])
        mom = O.moments(np.array([0, n], dtype=np.int32), v[:, 0], v[:, 1], v[:, 2])
        h = D.sample_high(mom, h)
    f = D.high_order(h)[0]
    np.testing.assert_allclose(f[0:6], [5, 0, 0, 5, 0, 5], atol=0.05)
    assert abs(f[6]) < 0.1 and abs(f[7] - 105) < 2.0
    # brute force: two cells over two steps, central moments about each step's cell mean
    hs = np.zeros((2, D.HSAMP))
    acc = np.zeros((2, 5))
    for s in range(2):
        counts = [7, 13]
        v = rng.standard_normal((20, 3)) * np.array([1.0, 2.0, 0.5]) + rng.standard_normal(3)
        off = np.array([0, 7, 20], dtype=np.int32)
        hs = D.sample_high(O.moments(off, v[:, 0], v[:, 1], v[:, 2]), hs)
        for cidx in range(2):
            c = v[off[cidx]:off[cidx + 1]]
            c = c - c.mean(0)
            c2 = (c * c).sum(1)
            k = counts[cidx]
            acc[cidx] += [k, k * c2.mean() / 3, k * (c[:, 0] * c[:, 1] * c2).mean(),
                          k * (c2 * c2).mean(), k * (c2 ** 3).mean()]
    np.testing.assert_allclose(hs[:, 0], acc[:, 0], rtol=0)
    np.testing.assert_allclose(hs[:, 1], acc[:, 1], rtol=1e-13)
    np.testing.assert_allclose(hs[:, 3], acc[:, 2], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(hs[:, 8], acc[:, 3], rtol=1e-12)
    np.testing.assert_allclose(hs[:, 9], acc[:, 4], rtol=1e-12)
    f2 = D.high_order(hs)
    th = acc[:, 1] / acc[:, 0]
    np.testing.assert_allclose(f2[:, 7], acc[:, 4] / acc[:, 0] / th ** 3, rtol=1e-12)
    assert np.all(np.isnan(D.high_order(np.zeros((1, D.HSAMP)))))
