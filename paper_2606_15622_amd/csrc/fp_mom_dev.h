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
// The values acc[LO .. LO + N) of the above into o[0 .. N): the same operations in the same
// order as for the whole set (a subset of the monomials gives the same sums bit for bit).
template <int LO, int N>
__device__ __forceinline__ void mom_accum_range(double a, double bb, double d, double (&o)[N]) {
    const double aa = a * a, ab = a * bb, ad = a * d, b2 = bb * bb, bd = bb * d, dd = d * d;
#define FP_MA_ADD(i, x) \
    if constexpr ((i) >= LO && (i) < LO + N) o[(i) - LO] += (x)
#define FP_MA_FMA(i, x, y) \
    if constexpr ((i) >= LO && (i) < LO + N) o[(i) - LO] = fma((x), (y), o[(i) - LO])
    FP_MA_ADD(0, aa); FP_MA_ADD(1, ab); FP_MA_ADD(2, ad);
    FP_MA_ADD(3, b2); FP_MA_ADD(4, bd); FP_MA_ADD(5, dd);
    FP_MA_FMA(6, aa, a);
    FP_MA_FMA(7, aa, bb);
    FP_MA_FMA(8, aa, d);
    FP_MA_FMA(9, b2, a);
    FP_MA_FMA(10, ab, d);
    FP_MA_FMA(11, dd, a);
    FP_MA_FMA(12, b2, bb);
    FP_MA_FMA(13, b2, d);
    FP_MA_FMA(14, dd, bb);
    FP_MA_FMA(15, dd, d);
    if constexpr (LO + N > 16) {
        const double c2 = aa + b2 + dd;
        FP_MA_FMA(16, aa, c2); FP_MA_FMA(17, ab, c2); FP_MA_FMA(18, ad, c2);
        FP_MA_FMA(19, b2, c2); FP_MA_FMA(20, bd, c2); FP_MA_FMA(21, dd, c2);
        const double c4 = c2 * c2;
        FP_MA_FMA(22, c4, a); FP_MA_FMA(23, c4, bb); FP_MA_FMA(24, c4, d);
        FP_MA_FMA(25, c4, c2);
    }
#undef FP_MA_ADD
#undef FP_MA_FMA
}

template <int NVX = NV>
__device__ __forceinline__ void mom_accum(double a, double bb, double d, double (&acc)[NVX]) {
    mom_accum_range<0, NVX>(a, bb, d, acc);
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
// order, MR values per round; with 32 or more lanes per group two stripes of G/2 lanes each
// add half of the partials and one lane exchange joins the halves: chains of G/2 instead
// of G dependent adds), then the record of the cell, one entry per lane:
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
        if constexpr (G >= 32) {
            constexpr int H = G / 2;   // stripe width, at least MR
            const int v = lg % H, h = lg / H;
            double t = 0.0;
            if (v < MR && r0 + v < NVX)
                for (int i = 0; i < H; ++i) t += sm.red[v][grp * G + h * H + i];
            t += __shfl_xor(t, H, 64);
            if (h == 0 && v < MR && r0 + v < NVX) sm.fin[grp][r0 + v] = t;
        } else {
            for (int v = lg; v < MR && r0 + v < NVX; v += G) {
                double t = 0.0;
                for (int i = 0; i < G; ++i) t += sm.red[v][grp * G + i];
                sm.fin[grp][r0 + v] = t;
            }
        }
        __syncthreads();
    }
    if (in)
        for (int e = lg; e < MOM; e += G) rec[e] = mom_entry<BLOCK, G, NVX>(sm, grp, n, U0, U1, U2, e);
}

}  // namespace fpg
