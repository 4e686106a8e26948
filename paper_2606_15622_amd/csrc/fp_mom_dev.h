// fp_mom_dev.h -- device pieces of the central-moment gather shared by fp_moments and the
// re-sort that also gathers moments: the 26 monomials of c = v - U entering the closure
// (P, T, R = c c |c|^2, W = c |c|^4, H = |c|^6; the moments u^(p) of eq. system9x9 and
// Table matrix_system), the cross-lane sums through LDS and the moment record.
#pragma once
#include "fp_internal.h"

namespace fpg {

constexpr int NV = 26;   // accumulated monomials: P (6), T (10), R (6), W (3), H
constexpr int NV_LOW = 16;   // through third order only: P and T
constexpr int MR = 13;   // values per LDS reduction round

// acc[0..5] P (11 12 13 22 23 33), acc[6..15] T (111 112 113 122 123 133 222 223 233 333),
// acc[16..21] R, acc[22..24] W, acc[25] H; FP64 products and sums.  With NVX = NV_LOW
// only P and T are accumulated (the same operations, in the same order).
template <int NVX = NV>
__device__ __forceinline__ void mom_accum(double a, double bb, double d, double (&acc)[NVX]) {
    const double aa = a * a, ab = a * bb, ad = a * d, b2 = bb * bb, bd = bb * d, dd = d * d;
    acc[0] += aa; acc[1] += ab; acc[2] += ad; acc[3] += b2; acc[4] += bd; acc[5] += dd;
    acc[6] = fma(aa, a, acc[6]);
    acc[7] = fma(aa, bb, acc[7]);
    acc[8] = fma(aa, d, acc[8]);
    acc[9] = fma(b2, a, acc[9]);
    acc[10] = fma(ab, d, acc[10]);
    acc[11] = fma(dd, a, acc[11]);
    acc[12] = fma(b2, bb, acc[12]);
    acc[13] = fma(b2, d, acc[13]);
    acc[14] = fma(dd, bb, acc[14]);
    acc[15] = fma(dd, d, acc[15]);
    if constexpr (NVX == NV) {
        const double c2 = aa + b2 + dd;
        acc[16] = fma(aa, c2, acc[16]); acc[17] = fma(ab, c2, acc[17]); acc[18] = fma(ad, c2, acc[18]);
        acc[19] = fma(b2, c2, acc[19]); acc[20] = fma(bd, c2, acc[20]); acc[21] = fma(dd, c2, acc[21]);
        const double c4 = c2 * c2;
        acc[22] = fma(c4, a, acc[22]); acc[23] = fma(c4, bb, acc[23]); acc[24] = fma(c4, d, acc[24]);
        acc[25] = fma(c4, c2, acc[25]);
    }
}

// LDS for the cross-lane sums of one workgroup of BLOCK threads in groups of G lanes
template <int BLOCK, int G>
struct MomShared {
    double red[MR][BLOCK + 1];   // +1: rows start on different banks
    double fin[BLOCK / G][NV];
};

// entry e of the moment record from the group's final sums in LDS
template <int BLOCK, int G, int NVX = NV>
__device__ __forceinline__ double mom_entry(const MomShared<BLOCK, G>& sm, int grp, int32_t n,
                                            double U0, double U1, double U2, int e) {
    const double inv_n = n > 0 ? 1.0 / (double)n : 0.0;
    if (e == M_N) return (double)n;
    if (e < M_TH) return e == M_U ? U0 : (e == M_U + 1 ? U1 : U2);
    if (e == M_TH)
        return (sm.fin[grp][0] * inv_n + sm.fin[grp][3] * inv_n + sm.fin[grp][5] * inv_n) / 3.0;
    if (e < M_P + NVX) return sm.fin[grp][e - M_P] * inv_n;
    return 0.0;
}

// Cross-lane sums of acc over the group (lane v adds the partials of value v in lane
// order, MR values per round), then the record of the cell, one entry per lane:
// N, U, theta, P, T, R, W, H (moments / N; R, W, H zero when only NV_LOW values were
// accumulated), pad.  Every thread of the block must call.
template <int BLOCK, int G, int NVX = NV>
__device__ __forceinline__ void mom_finish(MomShared<BLOCK, G>& sm, const double (&acc)[NVX], int grp,
                                           int lg, bool in, int32_t n, double U0, double U1,
                                           double U2, double* __restrict__ rec) {
#pragma unroll
    for (int r0 = 0; r0 < NVX; r0 += MR) {
#pragma unroll
        for (int v = 0; v < MR; ++v)
            if (r0 + v < NVX) sm.red[v][threadIdx.x] = acc[r0 + v];
        __syncthreads();
        for (int v = lg; v < MR && r0 + v < NVX; v += G) {
            double t = 0.0;
            for (int i = 0; i < G; ++i) t += sm.red[v][grp * G + i];
            sm.fin[grp][r0 + v] = t;
        }
        __syncthreads();
    }
    if (in)
        for (int e = lg; e < MOM; e += G) rec[e] = mom_entry<BLOCK, G, NVX>(sm, grp, n, U0, U1, U2, e);
}

}  // namespace fpg
