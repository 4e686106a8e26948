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
#include "fp_mom_dev.h"
#include "fp_sample_dev.h"

namespace fpg {

// one-wave workgroups: the moment reduction's LDS (MomShared) then takes 7 KB per wave
// instead of 33 KB per four, and no longer caps the resident waves
constexpr int MOM_BLOCK = 64;
constexpr int MOM_K = 8;

// samp0, samp1 (optional): time-average sums that also receive the cell's record, added
// exactly as fp_sample adds them (lanes 0..13 of the group, one sum each, rebuilt from the
// final sums in LDS instead of the stored record)
template <typename T, int G, int K, int NVX>
__global__ __launch_bounds__(MOM_BLOCK) void moments_kernel(
    int32_t ncell, const int32_t* __restrict__ offsets, const T* __restrict__ vx,
    const T* __restrict__ vy, const T* __restrict__ vz, double* __restrict__ mom,
    double* __restrict__ samp0, double* __restrict__ samp1) {
    const int64_t gt = (int64_t)blockIdx.x * MOM_BLOCK + threadIdx.x;
    const int32_t cell = (int32_t)(gt / G);
    const int lg = (int)(gt % G);
    const bool in = cell < ncell;
    int32_t b = 0, n = 0;
    if (in) {
        b = offsets[cell];
        n = offsets[cell + 1] - b;
    }
    // the sums to update, loaded now (their latency hides behind the velocities')
    constexpr int SQ = (14 + G - 1) / G;
    double sv0[SQ], sv1[SQ];
#pragma unroll
    for (int u = 0; u < SQ; ++u) {
        const int e = lg + u * G;
        const int64_t at = (int64_t)cell * SAMP + e;
        sv0[u] = in && samp0 && e < 14 ? samp0[at] : 0.0;
        sv1[u] = in && samp1 && e < 14 ? samp1[at] : 0.0;
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

    double acc[NVX];
#pragma unroll
    for (int i = 0; i < NVX; ++i) acc[i] = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int32_t j = lg + k * G;
        if (j < n) mom_accum<NVX>((double)cx[k] - U0, (double)cy[k] - U1, (double)cz[k] - U2, acc);
    }
    for (int32_t j = lg + K * G; j < n; j += G)
        mom_accum<NVX>((double)vx[b + j] - U0, (double)vy[b + j] - U1, (double)vz[b + j] - U2, acc);
    __shared__ MomShared<MOM_BLOCK, G> sm;
    const int grp = (int)(threadIdx.x / G);
    mom_finish<MOM_BLOCK, G, NVX>(sm, acc, grp, lg, in, n, U0, U1, U2, mom + (int64_t)(in ? cell : 0) * MOM);
    if (in && (samp0 || samp1)) {
        // every term with a compile-time entry index (no indexed access to m), the lane's
        // own ones kept
        double m[M_T + 10];
#pragma unroll
        for (int e = 0; e < M_T + 10; ++e) m[e] = mom_entry<MOM_BLOCK, G, NVX>(sm, grp, n, U0, U1, U2, e);
        double t[SQ];
#pragma unroll
        for (int u = 0; u < SQ; ++u) t[u] = 0.0;
#pragma unroll
        for (int e = 0; e < 14; ++e) {
            const double v = sample_term(m, e);
#pragma unroll
            for (int u = 0; u < SQ; ++u) t[u] = lg + u * G == e ? v : t[u];
        }
#pragma unroll
        for (int u = 0; u < SQ; ++u) {
            const int e = lg + u * G;
            if (e >= 14) continue;
            const int64_t at = (int64_t)cell * SAMP + e;
            if (samp0) samp0[at] = sv0[u] + t[u];
            if (samp1) samp1[at] = sv1[u] + t[u];
        }
    }
}

template <typename T, int G>
static void mom_launch(fp_ctx* c, const fp_particles* p, const int32_t* off, double* mom,
                       double* samp0, double* samp1, hipStream_t s) {
    const int64_t threads = (int64_t)c->ncell * G;
    const unsigned grid = (unsigned)((threads + MOM_BLOCK - 1) / MOM_BLOCK);
    if (c->cfg.moment_order == 3)
        hipLaunchKernelGGL((moments_kernel<T, G, MOM_K, NV_LOW>), dim3(grid), dim3(MOM_BLOCK), 0, s,
                           c->ncell, off, (const T*)p->vx, (const T*)p->vy, (const T*)p->vz, mom, samp0,
                           samp1);
    else
        hipLaunchKernelGGL((moments_kernel<T, G, MOM_K, NV>), dim3(grid), dim3(MOM_BLOCK), 0, s,
                           c->ncell, off, (const T*)p->vx, (const T*)p->vy, (const T*)p->vz, mom, samp0,
                           samp1);
}

template <typename T>
static void mom_dispatch(fp_ctx* c, const fp_particles* p, const int32_t* off, double* mom,
                         double* samp0, double* samp1, hipStream_t s) {
    // about five particles per lane (the smallest width with 4.8 G >= mean count): on
    // cells of 24, 52 and 150 particles 8, 16 and 32 lanes beat their neighbours
    switch (lanes_per_cell(c, p->n, 0, 6)) {
        case 4: mom_launch<T, 4>(c, p, off, mom, samp0, samp1, s); break;
        case 8: mom_launch<T, 8>(c, p, off, mom, samp0, samp1, s); break;
        case 16: mom_launch<T, 16>(c, p, off, mom, samp0, samp1, s); break;
        case 32: mom_launch<T, 32>(c, p, off, mom, samp0, samp1, s); break;
        default: mom_launch<T, 64>(c, p, off, mom, samp0, samp1, s); break;
    }
}

int launch_moments(fp_ctx* c, const fp_particles* p, const int32_t* offsets, double* mom,
                   double* samp0, double* samp1, hipStream_t s) {
    if (c->cfg.precision == FP_F32)
        mom_dispatch<float>(c, p, offsets, mom, samp0, samp1, s);
    else
        mom_dispatch<double>(c, p, offsets, mom, samp0, samp1, s);
    return check_launch(c, samp0 || samp1 ? "fp_moments_sample" : "fp_moments");
}

}  // namespace fpg
