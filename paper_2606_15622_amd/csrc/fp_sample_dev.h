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

// Increment of time-average sum e (0..13) by the moment record m: the conserved-variable
// sums N, N U_i, N <v_i v_j> (P + U U) and N <v_i |v|^2> / 2 written out (S + 2 P U +
// 3 theta U + U |U|^2), then the sample count; records without particles add only the
// count.  sample_add applies every entry, callers with one lane per entry call this.
__device__ __forceinline__ double sample_term(const double* m, int e) {
    if (e == 13) return 1.0;
    const double N = m[M_N];
    if (!(N > 0.0) || e > 13) return 0.0;
    if (e == 0) return N;
    const double U[3] = {m[M_U], m[M_U + 1], m[M_U + 2]};
    if (e < 4) return N * U[e - 1];
    const int ii[6] = {0, 0, 0, 1, 1, 2}, jj[6] = {0, 1, 2, 1, 2, 2};
    if (e < 10) {
        const int q = e - 4;
        return N * (m[M_P + q] + U[ii[q]] * U[jj[q]]);
    }
    const int i = e - 10;
    // P[i][j] of the symmetric stress from its six stored entries (11 12 13 22 23 33)
    const int pidx[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
    const int tidx[3][3] = {{0, 3, 5}, {1, 6, 8}, {2, 7, 9}};
    const double S = m[M_T + tidx[i][0]] + m[M_T + tidx[i][1]] + m[M_T + tidx[i][2]];
    const double th = m[M_TH];
    const double UU = U[0] * U[0] + U[1] * U[1] + U[2] * U[2];
    const double PU = m[M_P + pidx[i][0]] * U[0] + m[M_P + pidx[i][1]] * U[1] + m[M_P + pidx[i][2]] * U[2];
    return N * (S + 2.0 * PU + 3.0 * th * U[i] + U[i] * UU);
}

__device__ __forceinline__ void sample_add(const double* m, double* o) {
#pragma unroll
    for (int e = 0; e < 14; ++e) o[e] += sample_term(m, e);
}

}  // namespace fpg
