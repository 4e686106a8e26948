"""Plain FP64 NumPy oracle of the post-processing diagnostics of the sampled fields.

TEST INFRASTRUCTURE ONLY.  From the cumulative time-average sums of a cell (sample
layout: sum N, sum v_i, sum v_i v_j (11 12 13 22 23 33), sum v_i |v|^2, number of samples)
it forms the averaged state and the covariance-based entropy proxies of Sec. "Covariance-
based entropy-proxy audit on the stagnation line and cylinder surface":
  Theta_ij = <c_i c_j>, theta = tr(Theta) / 3                         (eq. cyl_theta_def)
  ds_eq    = 3/2 log(theta / theta_inf) - log(n / n_inf)              (eq. cyl_entropy_eq)
  D_G      = -1/2 log det(Theta / theta)                              (eq. cyl_DG)
  ds_kinG  = ds_eq - (D_G - D_G,inf)                                  (eq. cyl_entropy_kinG)
  D_q      = |q^|^2 / 5,  q^_i = <c_i |c|^2> / (2 theta^(3/2))
and the normalised stress Theta_ij / theta - delta_ij.  The averages are ratios of the
cumulative sums (the state of the time-averaged particle ensemble); with v = U + c,
<c_i |c|^2> = <v_i |v|^2> - U_i |U|^2 - 3 theta U_i - 2 Theta_ik U_k.

Output per cell, 24 entries: 0 particles per sample, 1 number density, 2-4 U, 5 theta,
6 T, 7-12 normalised stress, 13-15 q^, 16 ds_eq, 17 D_G, 18 ds_kinG, 19 D_q, 20-23 zero.
Cells without particles, or with theta <= 0, get NaN in 2-19; a covariance that is not
positive definite (det(Theta/theta) <= DET_MIN = 1e-12, as for fewer than four particles,
where rounding decides the sign of a zero determinant) gets NaN in D_G and ds_kinG.
"""
import numpy as np

S2 = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
DET_MIN = 1e-12


def diagnostics(samp, dens_factor, mass_over_kB, theta_inf, n_inf, dg_inf):
    """samp [ncell][16] cumulative sums; dens_factor [ncell] (real molecules per particle
    / gas volume of the cell); returns [ncell][24]."""
    samp = np.asarray(samp, dtype=np.float64)
    ncell = samp.shape[0]
    out = np.full((ncell, 24), np.nan)
    out[:, 20:] = 0.0
    for k in range(ncell):
        sN, nsamp = samp[k, 0], samp[k, 13]
        out[k, 0] = sN / nsamp if nsamp > 0 else 0.0
        out[k, 1] = out[k, 0] * dens_factor[k]
        if not (sN > 0):
            continue
        U = samp[k, 1:4] / sN
        Th = np.zeros((3, 3))
        for q, (i, j) in enumerate(S2):
            Th[i, j] = Th[j, i] = samp[k, 4 + q] / sN - U[i] * U[j]
        theta = np.trace(Th) / 3.0
        if not (theta > 0):
            continue
        vv = samp[k, 10:13] / sN
        ccc = vv - U * (U @ U) - 3.0 * theta * U - 2.0 * (Th @ U)
        qh = ccc / (2.0 * theta ** 1.5)
        out[k, 2:5] = U
        out[k, 5] = theta
        out[k, 6] = theta * mass_over_kB
        for q, (i, j) in enumerate(S2):
            out[k, 7 + q] = Th[i, j] / theta - (1.0 if i == j else 0.0)
        out[k, 13:16] = qh
        ds_eq = 1.5 * np.log(theta / theta_inf) - np.log(out[k, 1] / n_inf)
        det = np.linalg.det(Th / theta)
        dg = -0.5 * np.log(det) if det > DET_MIN else np.nan   # positive-definite Theta only
        out[k, 16] = ds_eq
        out[k, 17] = dg
        out[k, 18] = ds_eq - (dg - dg_inf)
        out[k, 19] = (qh @ qh) / 5.0
    return out


def surface_coefficients(wall, t_total, w):
    """Surface coefficients of the cylinder (Sec. "Extension to External Aerodynamics":
    C_p, C_f, C_h along the surface angle theta, 180 degrees at the front stagnation
    point) from the exchange sums wall[nbins][4] of the flights (per unit molecular mass:
    hits, normal momentum, tangential momentum towards the rear, energy given to the
    wall) accumulated over a time t_total.  Standard definitions, each bin taking both
    halves of the circle (area 2 R (pi / nbins) depth):
      p = m fnum S_n / (A t),  tau = m fnum S_t / (A t),  q = m fnum S_e / (A t),
      C_p = (p - p_inf) / (rho_inf U^2 / 2),  C_f = tau / (rho_inf U^2 / 2),
      C_h = q / (rho_inf U^3 / 2),  rho_inf = n_inf m, p_inf = n_inf k_B T_inf.
    Returns [nbins][4]: bin-centre theta in degrees, C_p, C_f, C_h."""
    wall = np.asarray(wall, dtype=np.float64)
    nb = wall.shape[0]
    m, fnum = float(w["mass"]), float(w["fnum"])
    R, depth = float(w["circle"][2]), float(w["depth"])
    area = 2.0 * R * (np.pi / nb) * depth
    U = float(np.sqrt(np.sum(np.asarray(w["u_inf"], dtype=np.float64) ** 2)))
    rho = float(w["n_inf"]) * m
    p_inf = float(w["n_inf"]) * float(w["kB"]) * float(w["T_inf"])
    dyn = 0.5 * rho * U * U
    scale = m * fnum / (area * t_total)
    out = np.zeros((nb, 4))
    out[:, 0] = (np.arange(nb) + 0.5) * 180.0 / nb
    out[:, 1] = (scale * wall[:, 1] - p_inf) / dyn
    out[:, 2] = scale * wall[:, 2] / dyn
    out[:, 3] = scale * wall[:, 3] / (dyn * U)
    return out


# ---------------------------------------------------------------------------------------
# Normalised high-order fields (Sec. "Conservation, stability, entropy proxy, and noise
# sensitivity" and the high-order diagnostics of the cavity): from the peculiar velocity
# c = v - U of a cell, R_ij = <c_i c_j |c|^2>, Delta_4 = <|c|^4> - 15 theta^2 and
# DM6 = <|c|^6>, theta = <|c|^2> / 3, each divided by the local Maxwellian scale
# (theta^2, theta^2, theta^3).  Reading: the averaged fields are particle-weighted time
# averages of each sampled step's cell moments (about that step's cell mean):
#   hsamp = [sum N, sum N theta, sum N R_ij (6), sum N <|c|^4>, sum N <|c|^6>, 0...]
#   R_ij,norm = Rbar_ij / thetabar^2, Delta_4,norm = <|c|^4>bar / thetabar^2 - 15,
#   DM6_norm = <|c|^6>bar / thetabar^3   (Maxwellian: 5 delta_ij, 0, 105).
HSAMP = 16


def sample_high(mom, hsamp=None):
    """Adds the high-order sums of moment records mom[ncell][32] to hsamp[ncell][16]."""
    mom = np.asarray(mom, dtype=np.float64)
    if hsamp is None:
        hsamp = np.zeros((mom.shape[0], HSAMP))
    N = mom[:, 0]
    has = N > 0
    R = mom[:, 21:27]
    hsamp[has, 0] += N[has]
    hsamp[has, 1] += N[has] * mom[has, 4]
    hsamp[has, 2:8] += N[has, None] * R[has]
    hsamp[has, 8] += N[has] * (R[has, 0] + R[has, 3] + R[has, 5])
    hsamp[has, 9] += N[has] * mom[has, 30]
    return hsamp


def high_order(hsamp):
    """[ncell][8]: R_ij,norm (11 12 13 22 23 33), Delta_4,norm, DM6_norm; NaN where a
    cell has no particles or zero temperature."""
    h = np.asarray(hsamp, dtype=np.float64)
    out = np.full((h.shape[0], 8), np.nan)
    ok = (h[:, 0] > 0) & (h[:, 1] > 0)
    th = h[ok, 1] / h[ok, 0]
    out[ok, 0:6] = h[ok, 2:8] / h[ok, 0][:, None] / (th * th)[:, None]
    out[ok, 6] = h[ok, 8] / h[ok, 0] / (th * th) - 15.0
    out[ok, 7] = h[ok, 9] / h[ok, 0] / (th * th * th)
    return out
