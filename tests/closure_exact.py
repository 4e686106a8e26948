"""Exact-rational construction of the cubic-FP closure of a tiny cell (test helper).

Independent of the oracle's assembly: the conditions are generated from first
principles.  For the Ito process dM = A dt + sqrt(2 theta / tau) dW (eq. sde_vel) the
rate of a test-function average is <A . grad Psi> + (theta / tau) <lap Psi>.  The drift
is the cubic one (eq. cubic_drift) written as A = c1 c + Gamma (|c|^2 - 3 theta)
- eps^2 (c |c|^2 - S) with c1 = Ct - I / tau.  The conditions ask stress averages
<c_i c_j> to relax at 2/tau toward theta delta_ij and heat-flux averages <c_i |c|^2> at
4/(3 tau) (Prandtl number 2/3).  Each condition is affine in the nine unknowns
(Ct11 Ct12 Ct13 Ct22 Ct23 Ct33, G1 G2 G3); the matrix is read off column by column.
"""
from fractions import Fraction as Fr

PAIRS = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]


def _unit(u):
    Ct = [[Fr(0)] * 3 for _ in range(3)]
    G = [Fr(0)] * 3
    if u is not None:
        if u < 6:
            i, j = PAIRS[u]
            Ct[i][j] = Ct[j][i] = Fr(1)
        else:
            G[u - 6] = Fr(1)
    return Ct, G


def _residuals(cs, theta, tau, eps2, Ct, G):
    n = len(cs)
    S = [sum(c[i] * sum(x * x for x in c) for c in cs) / n for i in range(3)]
    P = [[sum(c[i] * c[j] for c in cs) / n for j in range(3)] for i in range(3)]
    rates_stress, rates_heat = [], []
    acc_s = {pq: Fr(0) for pq in PAIRS}
    acc_h = [Fr(0)] * 3
    for c in cs:
        c2 = sum(x * x for x in c)
        A = [sum((Ct[i][j] - (Fr(1) / tau if i == j else 0)) * c[j] for j in range(3))
             + G[i] * (c2 - 3 * theta) - eps2 * (c[i] * c2 - S[i]) for i in range(3)]
        for (i, j) in PAIRS:
            # grad(c_i c_j) = e_i c_j + e_j c_i
            acc_s[(i, j)] += A[i] * c[j] + A[j] * c[i]
        for i in range(3):
            # grad(c_i |c|^2) = e_i |c|^2 + 2 c_i c
            acc_h[i] += A[i] * c2 + 2 * c[i] * sum(A[k] * c[k] for k in range(3))
    for (i, j) in PAIRS:
        lap = 2 if i == j else 0                      # laplacian of c_i c_j
        rate = acc_s[(i, j)] / n + theta / tau * lap
        target = -Fr(2) / tau * (P[i][j] - (theta if i == j else 0))
        rates_stress.append(rate - target)
    for i in range(3):
        # laplacian of c_i |c|^2 is 10 c_i, whose average is zero
        rate = acc_h[i] / n
        target = -Fr(4) / (3 * tau) * S[i]
        rates_heat.append(rate - target)
    return rates_stress + rates_heat


def exact_system(v_int, tau, eps2):
    """(A, b, theta, cs) exactly, for integer/rational velocities v_int (list of 3-lists)."""
    n = len(v_int)
    U = [sum(Fr(v[i]) for v in v_int) / n for i in range(3)]
    cs = [[Fr(v[i]) - U[i] for i in range(3)] for v in v_int]
    theta = sum(sum(x * x for x in c) for c in cs) / (3 * n)
    F0 = _residuals(cs, theta, tau, eps2, *_unit(None))
    cols = []
    for u in range(9):
        Fu = _residuals(cs, theta, tau, eps2, *_unit(u))
        cols.append([Fu[r] - F0[r] for r in range(9)])
    A = [[cols[u][r] for u in range(9)] for r in range(9)]
    b = [-F0[r] for r in range(9)]
    return A, b, theta, cs


def solve_exact(A, b):
    n = len(b)
    M = [row[:] + [b[r]] for r, row in enumerate(A)]
    for k in range(n):
        p = next(r for r in range(k, n) if M[r][k] != 0)
        M[k], M[p] = M[p], M[k]
        for r in range(n):
            if r != k and M[r][k] != 0:
                f = M[r][k] / M[k][k]
                M[r] = [M[r][c] - f * M[k][c] for c in range(n + 1)]
    return [M[k][n] / M[k][k] for k in range(n)]
