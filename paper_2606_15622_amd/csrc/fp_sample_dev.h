// fp_sample_dev.h -- time-average sums of one cell from its moment record (device code
// shared by the sampling kernel and the re-sort that gathers the moments).
//
// Raw sums are rebuilt from the central moments of the cell, with v = U + c and <c> = 0:
//   sum v_i          = N U_i
//   sum v_i v_j      = N (P_ij + U_i U_j)
//   sum v_i |v|^2    = N (S_i + 2 P_ik U_k + 3 theta U_i + U_i |U|^2),  S_i = T_ikk
// o[0] N, o[1..3] momentum, o[4..9] second moments (xx xy xz yy yz zz), o[10..12] energy
// flux, o[13] the number of samples; o[14], o[15] are not touched.
#pragma once
#include "fp_internal.h"

namespace fpg {

__device__ __forceinline__ void sample_add(const double* m, double* o) {
    const double N = m[M_N];
    o[13] += 1.0;
    if (!(N > 0.0)) return;
    const double U[3] = {m[M_U], m[M_U + 1], m[M_U + 2]};
    const double P[3][3] = {{m[M_P + 0], m[M_P + 1], m[M_P + 2]},
                            {m[M_P + 1], m[M_P + 3], m[M_P + 4]},
                            {m[M_P + 2], m[M_P + 4], m[M_P + 5]}};
    const double S[3] = {m[M_T + 0] + m[M_T + 3] + m[M_T + 5],
                         m[M_T + 1] + m[M_T + 6] + m[M_T + 8],
                         m[M_T + 2] + m[M_T + 7] + m[M_T + 9]};
    const double th = m[M_TH];
    const double UU = U[0] * U[0] + U[1] * U[1] + U[2] * U[2];
    o[0] += N;
#pragma unroll
    for (int i = 0; i < 3; ++i) o[1 + i] += N * U[i];
    const int ii[6] = {0, 0, 0, 1, 1, 2}, jj[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int q = 0; q < 6; ++q) o[4 + q] += N * (P[ii[q]][jj[q]] + U[ii[q]] * U[jj[q]]);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double PU = P[i][0] * U[0] + P[i][1] * U[1] + P[i][2] * U[2];
        o[10 + i] += N * (S[i] + 2.0 * PU + 3.0 * th * U[i] + U[i] * UU);
    }
}

}  // namespace fpg
