// fp_sample.hip -- time averaging of cell sums (the "average_results" step).
//
// Raw sums are rebuilt from the central moments of the cell, with v = U + c and <c> = 0:
//   sum v_i          = N U_i
//   sum v_i v_j      = N (P_ij + U_i U_j)
//   sum v_i |v|^2    = N (S_i + 2 P_ik U_k + 3 theta U_i + U_i |U|^2),  S_i = T_ikk
#include "fp_internal.h"

namespace fpg {

// 64 cells per workgroup: their moment records and sums are staged through LDS with
// coalesced loads and stores (one lane per cell would touch a new cache line per lane)
constexpr int SA_CELLS = 64, SA_BLOCK = 256, SA_MPAD = 33, SA_SPAD = 17;

__global__ __launch_bounds__(SA_BLOCK) void sample_kernel(int32_t ncell, const double* __restrict__ mom,
                                                          double* __restrict__ samp) {
    __shared__ double sm[SA_CELLS * SA_MPAD];
    __shared__ double ss[SA_CELLS * SA_SPAD];
    const int32_t c0 = blockIdx.x * SA_CELLS;
    const int32_t nc = min(SA_CELLS, ncell - c0);
    const double* mb = mom + (int64_t)c0 * MOM;
    double* sb = samp + (int64_t)c0 * SAMP;
    {
        // all loads in flight before their LDS writes
        constexpr int LM = SA_CELLS * MOM / SA_BLOCK, LS = SA_CELLS * SAMP / SA_BLOCK;
        double vm[LM], vs[LS];
#pragma unroll
        for (int u = 0; u < LM; ++u) {
            const int t = u * SA_BLOCK + threadIdx.x;
            vm[u] = t < nc * MOM ? mb[t] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < LS; ++u) {
            const int t = u * SA_BLOCK + threadIdx.x;
            vs[u] = t < nc * SAMP ? sb[t] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < LM; ++u) {
            const int t = u * SA_BLOCK + threadIdx.x;
            if (t < nc * MOM) sm[(t / MOM) * SA_MPAD + t % MOM] = vm[u];
        }
#pragma unroll
        for (int u = 0; u < LS; ++u) {
            const int t = u * SA_BLOCK + threadIdx.x;
            if (t < nc * SAMP) ss[(t / SAMP) * SA_SPAD + t % SAMP] = vs[u];
        }
    }
    __syncthreads();
    if (threadIdx.x < nc) {
        const double* m = sm + threadIdx.x * SA_MPAD;
        double* o = ss + threadIdx.x * SA_SPAD;
        const double N = m[M_N];
        o[13] += 1.0;
        if (N > 0.0) {
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
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < SA_CELLS * SAMP / SA_BLOCK; ++u) {
        const int t = u * SA_BLOCK + threadIdx.x;
        if (t < nc * SAMP) sb[t] = ss[(t / SAMP) * SA_SPAD + t % SAMP];
    }
}

int launch_sample(fp_ctx* c, const double* mom, double* samp, hipStream_t s) {
    hipLaunchKernelGGL(sample_kernel, dim3((c->ncell + SA_CELLS - 1) / SA_CELLS), dim3(SA_BLOCK), 0, s,
                       c->ncell, mom, samp);
    return check_launch(c, "fp_sample");
}

}  // namespace fpg
