// fp_moments.hip -- segmented central velocity moments of particles sorted by cell.
//
// G lanes per cell.  Pass 1 sums velocities (mean U), pass 2 sums the 26 monomials of
// c = v - U that enter the closure: P (6), T (10), R = P |c|^2 (6), W = c |c|^4 (3),
// H = |c|^6.  Up to K velocities per lane stay in registers between the passes; larger
// cells re-read the rest (L2-resident).  All products and sums are FP64: on CDNA4 a
// double FMA issues at the same rate as a single-precision one (no packed FP32 here),
// so FP64 accumulation costs nothing over FP32 and needs no compensation.  Cross-lane
// sums: the mean by DPP inside the group, the 26 monomial sums through LDS (lane v adds
// the partials of value v in lane order); fixed orders, so results are deterministic.
#include "fp_internal.h"

namespace fpg {

constexpr int MOM_BLOCK = 256;
constexpr int NV = 26;   // accumulated monomials: P (6), T (10), R (6), W (3), H
constexpr int MR = 13;   // values per LDS reduction round
constexpr int MOM_K = 8;

template <typename T, int G, int K>
__global__ __launch_bounds__(MOM_BLOCK) void moments_kernel(
    int32_t ncell, const int32_t* __restrict__ offsets, const T* __restrict__ vx,
    const T* __restrict__ vy, const T* __restrict__ vz, double* __restrict__ mom) {
    const int64_t gt = (int64_t)blockIdx.x * MOM_BLOCK + threadIdx.x;
    const int32_t cell = (int32_t)(gt / G);
    const int lg = (int)(gt % G);
    const bool in = cell < ncell;
    int32_t b = 0, n = 0;
    if (in) {
        b = offsets[cell];
        n = offsets[cell + 1] - b;
    }
    T cx[K], cy[K], cz[K];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int32_t j = lg + k * G;
        if (j < n) {
            cx[k] = vx[b + j];
            cy[k] = vy[b + j];
            cz[k] = vz[b + j];
            s0 += (double)cx[k];
            s1 += (double)cy[k];
            s2 += (double)cz[k];
        }
    }
    for (int32_t j = lg + K * G; j < n; j += G) {
        s0 += (double)vx[b + j];
        s1 += (double)vy[b + j];
        s2 += (double)vz[b + j];
    }
    s0 = group_sum<G>(s0);
    s1 = group_sum<G>(s1);
    s2 = group_sum<G>(s2);
    const double inv_n = n > 0 ? 1.0 / (double)n : 0.0;
    const double U0 = s0 * inv_n, U1 = s1 * inv_n, U2 = s2 * inv_n;

    double P[6] = {0, 0, 0, 0, 0, 0};
    double Tm[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    double R[6] = {0, 0, 0, 0, 0, 0};
    double W[3] = {0, 0, 0};
    double H = 0.0;
    auto accum = [&](double a, double bb, double d) {
        const double aa = a * a, ab = a * bb, ad = a * d, b2 = bb * bb, bd = bb * d, dd = d * d;
        const double c2 = aa + b2 + dd;
        P[0] += aa; P[1] += ab; P[2] += ad; P[3] += b2; P[4] += bd; P[5] += dd;
        Tm[0] = fma(aa, a, Tm[0]);   // 111
        Tm[1] = fma(aa, bb, Tm[1]);  // 112
        Tm[2] = fma(aa, d, Tm[2]);   // 113
        Tm[3] = fma(b2, a, Tm[3]);   // 122
        Tm[4] = fma(ab, d, Tm[4]);   // 123
        Tm[5] = fma(dd, a, Tm[5]);   // 133
        Tm[6] = fma(b2, bb, Tm[6]);  // 222
        Tm[7] = fma(b2, d, Tm[7]);   // 223
        Tm[8] = fma(dd, bb, Tm[8]);  // 233
        Tm[9] = fma(dd, d, Tm[9]);   // 333
        R[0] = fma(aa, c2, R[0]); R[1] = fma(ab, c2, R[1]); R[2] = fma(ad, c2, R[2]);
        R[3] = fma(b2, c2, R[3]); R[4] = fma(bd, c2, R[4]); R[5] = fma(dd, c2, R[5]);
        const double c4 = c2 * c2;
        W[0] = fma(c4, a, W[0]); W[1] = fma(c4, bb, W[1]); W[2] = fma(c4, d, W[2]);
        H = fma(c4, c2, H);
    };
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int32_t j = lg + k * G;
        if (j < n) accum((double)cx[k] - U0, (double)cy[k] - U1, (double)cz[k] - U2);
    }
    for (int32_t j = lg + K * G; j < n; j += G)
        accum((double)vx[b + j] - U0, (double)vy[b + j] - U1, (double)vz[b + j] - U2);

    // cross-lane sums through LDS, MR values per round: every lane stores its partial sums
    // (value-major, so consecutive lanes hit consecutive banks), then lane v of the group
    // adds the G partials of value v in lane order.  Far fewer instructions than a DPP
    // tree per value, and the finished values end up spread over the lanes.
    double acc[NV];
#pragma unroll
    for (int i = 0; i < 6; ++i) acc[i] = P[i];
#pragma unroll
    for (int i = 0; i < 10; ++i) acc[6 + i] = Tm[i];
#pragma unroll
    for (int i = 0; i < 6; ++i) acc[16 + i] = R[i];
#pragma unroll
    for (int i = 0; i < 3; ++i) acc[22 + i] = W[i];
    acc[25] = H;
    constexpr int GROUPS = MOM_BLOCK / G;
    __shared__ double red[MR][MOM_BLOCK + 1];   // +1: rows start on different banks
    __shared__ double fin[GROUPS][NV];
    const int grp = threadIdx.x / G;
#pragma unroll
    for (int r0 = 0; r0 < NV; r0 += MR) {
#pragma unroll
        for (int v = 0; v < MR; ++v)
            if (r0 + v < NV) red[v][threadIdx.x] = acc[r0 + v];
        __syncthreads();
        for (int v = lg; v < MR && r0 + v < NV; v += G) {
            double t = 0.0;
            for (int i = 0; i < G; ++i) t += red[v][grp * G + i];
            fin[grp][r0 + v] = t;
        }
        __syncthreads();
    }
    if (in) {
        // the record, one entry per lane: N, U, theta, P, T, R, W, H (moments / N), pad
        double* o = mom + (int64_t)cell * MOM;
        for (int e = lg; e < MOM; e += G) {
            double val;
            if (e == M_N) val = (double)n;
            else if (e < M_TH) val = e == M_U ? U0 : (e == M_U + 1 ? U1 : U2);
            else if (e == M_TH)
                val = (fin[grp][0] * inv_n + fin[grp][3] * inv_n + fin[grp][5] * inv_n) / 3.0;
            else if (e < 31) val = fin[grp][e - M_P] * inv_n;
            else val = 0.0;
            o[e] = val;
        }
    }
}

template <typename T, int G>
static void mom_launch(fp_ctx* c, const fp_particles* p, const int32_t* off, double* mom,
                       hipStream_t s) {
    const int64_t threads = (int64_t)c->ncell * G;
    const unsigned grid = (unsigned)((threads + MOM_BLOCK - 1) / MOM_BLOCK);
    hipLaunchKernelGGL((moments_kernel<T, G, MOM_K>), dim3(grid), dim3(MOM_BLOCK), 0, s,
                       c->ncell, off, (const T*)p->vx, (const T*)p->vy, (const T*)p->vz, mom);
}

template <typename T>
static void mom_dispatch(fp_ctx* c, const fp_particles* p, const int32_t* off, double* mom,
                         hipStream_t s) {
    switch (lanes_per_cell(c, p->n)) {
        case 4: mom_launch<T, 4>(c, p, off, mom, s); break;
        case 8: mom_launch<T, 8>(c, p, off, mom, s); break;
        case 16: mom_launch<T, 16>(c, p, off, mom, s); break;
        case 32: mom_launch<T, 32>(c, p, off, mom, s); break;
        default: mom_launch<T, 64>(c, p, off, mom, s); break;
    }
}

int launch_moments(fp_ctx* c, const fp_particles* p, const int32_t* offsets, double* mom,
                   hipStream_t s) {
    if (c->cfg.precision == FP_F32)
        mom_dispatch<float>(c, p, offsets, mom, s);
    else
        mom_dispatch<double>(c, p, offsets, mom, s);
    return check_launch(c, "fp_moments");
}

}  // namespace fpg
