"""Plain PyTorch (CPU, FP64) oracle of the differentiable exact closure.

TEST INFRASTRUCTURE ONLY.  An independent re-statement, in torch operations that autograd
can differentiate, of: segmented central moments (1/N averages), the theta-normalised
moment-matching system (written term by term from the moment conditions for c_i c_j and
c_i |c|^2 under the cubic drift, eq. cubic_drift, noise rate 2 theta / tau, stress
relaxing at 2/tau and heat flux at 4/(3 tau)), its solution (torch.linalg.solve) and the
de-normalisation Ct = Ch / tau, Gamma = Gh / (tau sqrt(theta)) with tau = 2 mu / p
(eq. tau) and mu = mu_ref (T / T_ref)^omega.
"""
import numpy as np
import torch

PAIRS = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]


def coefficients(v, offsets, w):
    """v: [n][3] float64 tensor (cells contiguous per offsets).  Returns [ncell][9]
    (Ct11 Ct12 Ct13 Ct22 Ct23 Ct33 G1 G2 G3); cells with fewer than n_min particles get
    zeros (they use the Langevin drift)."""
    off = np.asarray(offsets, dtype=np.int64)
    counts = torch.tensor(np.diff(off), dtype=torch.float64)
    ncell = counts.shape[0]
    cell = torch.tensor(np.repeat(np.arange(ncell), np.diff(off)), dtype=torch.int64)
    cnt = counts.clamp(min=1.0)

    def seg_mean(x):
        out = torch.zeros((ncell,) + x.shape[1:], dtype=x.dtype).index_add(0, cell, x)
        return out / cnt.reshape((ncell,) + (1,) * (x.dim() - 1))

    U = seg_mean(v)
    c = v - U[cell]
    c2 = (c * c).sum(1)
    P = seg_mean(c[:, :, None] * c[:, None, :])                      # [ncell][3][3]
    T = seg_mean(c[:, :, None, None] * c[:, None, :, None] * c[:, None, None, :])
    R = seg_mean(c[:, :, None] * c[:, None, :] * c2[:, None, None])
    W = seg_mean(c * (c2 * c2)[:, None])
    th = (P[:, 0, 0] + P[:, 1, 1] + P[:, 2, 2]) / 3.0
    Ph = P / th[:, None, None]
    Th = T / th[:, None, None, None] ** 1.5
    Rh = R / th[:, None, None] ** 2
    Wh = W / th[:, None] ** 2.5
    Sh = torch.einsum("nikk->ni", Th)
    Qh = torch.einsum("nkk->n", Rh)
    eh = float(w["eps_hat"])
    rows = []
    rhs = []
    eye = torch.eye(3, dtype=torch.float64)
    # stress rows: sum_k (Ch_ik P_kj + Ch_jk P_ki) + Gh_i S_j + Gh_j S_i = 2 eh R_ij
    for (i, j) in PAIRS:
        coef = [torch.zeros(ncell, dtype=torch.float64) for _ in range(9)]
        for k in range(3):
            coef[PAIRS.index(tuple(sorted((i, k))))] = coef[PAIRS.index(tuple(sorted((i, k))))] + Ph[:, k, j]
            coef[PAIRS.index(tuple(sorted((j, k))))] = coef[PAIRS.index(tuple(sorted((j, k))))] + Ph[:, k, i]
        coef[6 + i] = coef[6 + i] + Sh[:, j]
        coef[6 + j] = coef[6 + j] + Sh[:, i]
        rows.append(torch.stack(coef, 1))
        rhs.append(2.0 * eh * Rh[:, i, j])
    # heat-flux rows
    for i in range(3):
        coef = [torch.zeros(ncell, dtype=torch.float64) for _ in range(9)]
        for j in range(3):
            q = PAIRS.index(tuple(sorted((i, j))))
            coef[q] = coef[q] + Sh[:, j]
        for j in range(3):
            for k in range(3):
                q = PAIRS.index(tuple(sorted((j, k))))
                coef[q] = coef[q] + 2.0 * Th[:, i, j, k]
        coef[6 + i] = coef[6 + i] + (Qh - 9.0)
        for k in range(3):
            coef[6 + k] = coef[6 + k] + 2.0 * (Rh[:, i, k] - 3.0 * Ph[:, i, k])
        rows.append(torch.stack(coef, 1))
        PS = (Ph[:, i, :] * Sh).sum(1)
        rhs.append(5.0 / 3.0 * Sh[:, i] + eh * (3.0 * Wh[:, i] - 3.0 * Sh[:, i] - 2.0 * PS))
    A = torch.stack(rows, 1)
    b = torch.stack(rhs, 1)
    ok = counts >= max(int(w.get("n_min", 4)), 2)
    A = torch.where(ok[:, None, None], A, eye.new_zeros(9, 9) + torch.eye(9, dtype=torch.float64))
    b = torch.where(ok[:, None], b, torch.zeros_like(b))
    y = torch.linalg.solve(A, b)
    T_gas = th * float(w["mass"]) / float(w["kB"])
    p = counts * float(w["fnum_over_vol"]) * float(w["kB"]) * T_gas
    mu = float(w["mu_ref"]) * (T_gas / float(w["T_ref"])) ** float(w["omega"])
    tau = 2.0 * mu / p
    out = torch.cat([y[:, :6] / tau[:, None], y[:, 6:] / (tau * torch.sqrt(th))[:, None]], 1)
    return torch.where(ok[:, None], out, torch.zeros_like(out))
