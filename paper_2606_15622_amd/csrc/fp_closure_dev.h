// fp_closure_dev.h -- device functions of the 9x9 closure shared by the exact and the
// learned closure kernels: the theta-normalised system of one cell and its LU solve.
//
// The system (eq. system9x9) in theta-normalised form, unknowns Ch = tau Ct and
// Gh = tau sqrt(theta) Gamma.  Its blocks, written out entry by entry:
//   V (rows 11 12 13 22 23 33): Table matrix_system with u^(2)_ij = P_ij
//   W:                           Table matrix_system with u^(2)_i  = S_i = T_ikk
//   X^T(i,aa) = delta_ia S_a + 2 T_iaa,  X^T(i,ab) = delta_ia S_b + delta_ib S_a + 4 T_iab
//   Z(i,k)    = delta_ik (Q - 9) + 2 (R_ik - 3 P_ik),  Q = R_kk
//   rhs       = [2 eps_hat R_ij ; 5/3 S_i + eps_hat (3 W_i - 3 S_i - 2 P_ik S_k)]
// These follow from the moment conditions (eq. moment_match) for c_i c_j and c_i |c|^2
// under the cubic drift (eq. cubic_drift) with noise variance rate 2 theta / tau
// (eq. sde_vel), stress relaxing at 2/tau and heat flux at 4/(3 tau).
#pragma once
#include "fp_internal.h"

namespace fpg {

struct CellSystem {
    double a[9][10];  // augmented matrix [A | b]
};

__device__ __forceinline__ void build_system(const double* __restrict__ m, double eps_hat,
                                             CellSystem& s) {
    const double th = m[M_TH];
    const double i1 = 1.0 / th;
    const double i15 = i1 / sqrt(th);
    const double i2 = i1 * i1;
    const double i25 = i2 / sqrt(th);
    const double P11 = m[M_P + 0] * i1, P12 = m[M_P + 1] * i1, P13 = m[M_P + 2] * i1;
    const double P22 = m[M_P + 3] * i1, P23 = m[M_P + 4] * i1, P33 = m[M_P + 5] * i1;
    const double T111 = m[M_T + 0] * i15, T112 = m[M_T + 1] * i15, T113 = m[M_T + 2] * i15;
    const double T122 = m[M_T + 3] * i15, T123 = m[M_T + 4] * i15, T133 = m[M_T + 5] * i15;
    const double T222 = m[M_T + 6] * i15, T223 = m[M_T + 7] * i15, T233 = m[M_T + 8] * i15;
    const double T333 = m[M_T + 9] * i15;
    const double R11 = m[M_R + 0] * i2, R12 = m[M_R + 1] * i2, R13 = m[M_R + 2] * i2;
    const double R22 = m[M_R + 3] * i2, R23 = m[M_R + 4] * i2, R33 = m[M_R + 5] * i2;
    const double W1 = m[M_W + 0] * i25, W2 = m[M_W + 1] * i25, W3 = m[M_W + 2] * i25;
    const double S1 = T111 + T122 + T133, S2 = T112 + T222 + T233, S3 = T113 + T223 + T333;
    const double Q = R11 + R22 + R33;
    const double e = eps_hat;
    double(&a)[9][10] = s.a;
    // V | W | Q6
    a[0][0] = 2 * P11; a[0][1] = 2 * P12; a[0][2] = 2 * P13; a[0][3] = 0; a[0][4] = 0; a[0][5] = 0;
    a[0][6] = 2 * S1; a[0][7] = 0; a[0][8] = 0; a[0][9] = 2 * e * R11;
    a[1][0] = P12; a[1][1] = P22 + P11; a[1][2] = P23; a[1][3] = P12; a[1][4] = P13; a[1][5] = 0;
    a[1][6] = S2; a[1][7] = S1; a[1][8] = 0; a[1][9] = 2 * e * R12;
    a[2][0] = P13; a[2][1] = P23; a[2][2] = P33 + P11; a[2][3] = 0; a[2][4] = P12; a[2][5] = P13;
    a[2][6] = S3; a[2][7] = 0; a[2][8] = S1; a[2][9] = 2 * e * R13;
    a[3][0] = 0; a[3][1] = 2 * P12; a[3][2] = 0; a[3][3] = 2 * P22; a[3][4] = 2 * P23; a[3][5] = 0;
    a[3][6] = 0; a[3][7] = 2 * S2; a[3][8] = 0; a[3][9] = 2 * e * R22;
    a[4][0] = 0; a[4][1] = P13; a[4][2] = P12; a[4][3] = P23; a[4][4] = P33 + P22; a[4][5] = P23;
    a[4][6] = 0; a[4][7] = S3; a[4][8] = S2; a[4][9] = 2 * e * R23;
    a[5][0] = 0; a[5][1] = 0; a[5][2] = 2 * P13; a[5][3] = 0; a[5][4] = 2 * P23; a[5][5] = 2 * P33;
    a[5][6] = 0; a[5][7] = 0; a[5][8] = 2 * S3; a[5][9] = 2 * e * R33;
    // X^T | Z | R3
    a[6][0] = S1 + 2 * T111; a[6][1] = S2 + 4 * T112; a[6][2] = S3 + 4 * T113;
    a[6][3] = 2 * T122; a[6][4] = 4 * T123; a[6][5] = 2 * T133;
    a[7][0] = 2 * T112; a[7][1] = S1 + 4 * T122; a[7][2] = 4 * T123;
    a[7][3] = S2 + 2 * T222; a[7][4] = S3 + 4 * T223; a[7][5] = 2 * T233;
    a[8][0] = 2 * T113; a[8][1] = 4 * T123; a[8][2] = S1 + 4 * T133;
    a[8][3] = 2 * T223; a[8][4] = S2 + 4 * T233; a[8][5] = S3 + 2 * T333;
    a[6][6] = Q - 9 + 2 * (R11 - 3 * P11); a[6][7] = 2 * (R12 - 3 * P12); a[6][8] = 2 * (R13 - 3 * P13);
    a[7][6] = 2 * (R12 - 3 * P12); a[7][7] = Q - 9 + 2 * (R22 - 3 * P22); a[7][8] = 2 * (R23 - 3 * P23);
    a[8][6] = 2 * (R13 - 3 * P13); a[8][7] = 2 * (R23 - 3 * P23); a[8][8] = Q - 9 + 2 * (R33 - 3 * P33);
    const double PS1 = P11 * S1 + P12 * S2 + P13 * S3;
    const double PS2 = P12 * S1 + P22 * S2 + P23 * S3;
    const double PS3 = P13 * S1 + P23 * S2 + P33 * S3;
    a[6][9] = 5.0 / 3.0 * S1 + e * (3 * W1 - 3 * S1 - 2 * PS1);
    a[7][9] = 5.0 / 3.0 * S2 + e * (3 * W2 - 3 * S2 - 2 * PS2);
    a[8][9] = 5.0 / 3.0 * S3 + e * (3 * W3 - 3 * S3 - 2 * PS3);
}

// returns false if a pivot falls below tol (or is NaN)
__device__ __forceinline__ bool lu_solve(CellSystem& s, double tol, double y[9]) {
    double(&a)[9][10] = s.a;
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        double best = fabs(a[k][k]);
        int piv = k;
#pragma unroll
        for (int r = k + 1; r < 9; ++r) {
            const double v = fabs(a[r][k]);
            const bool gt = v > best;
            best = gt ? v : best;
            piv = gt ? r : piv;
        }
        ok = ok && (best >= tol);
        // the row swap is a predicated select on every candidate row; it is skipped when no
        // lane of the wave pivots off the diagonal (the common case near equilibrium)
        if (__any(piv != k)) {
#pragma unroll
            for (int r = k + 1; r < 9; ++r) {
                const bool sw = (piv == r);
#pragma unroll
                for (int cidx = k; cidx < 10; ++cidx) {
                    const double t = a[k][cidx];
                    a[k][cidx] = sw ? a[r][cidx] : t;
                    a[r][cidx] = sw ? t : a[r][cidx];
                }
            }
        }
        const double inv = 1.0 / a[k][k];
#pragma unroll
        for (int r = k + 1; r < 9; ++r) {
            const double f = a[r][k] * inv;
#pragma unroll
            for (int cidx = k + 1; cidx < 10; ++cidx) a[r][cidx] = fma(-f, a[k][cidx], a[r][cidx]);
        }
    }
#pragma unroll
    for (int k = 8; k >= 0; --k) {
        double t = a[k][9];
#pragma unroll
        for (int cidx = k + 1; cidx < 9; ++cidx) t = fma(-a[k][cidx], y[cidx], t);
        y[k] = t / a[k][k];
    }
    return ok;
}

// cell gas state: tau = 2 mu / p (eq. tau), VHS viscosity, eps^2 = eps_hat/(theta tau)
// ndens: real number density of the cell (particles times molecules per particle / volume)
__device__ __forceinline__ double cell_tau(const fp_config& g, double ndens, double theta) {
    const double T = theta * g.mass / g.kB;
    const double p = ndens * g.kB * T;
    const double mu = g.mu_ref * pow(T / g.T_ref, g.omega);
    return 2.0 * mu / p;
}

}  // namespace fpg
