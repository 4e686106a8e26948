// fp_sample.hip -- time averaging of cell sums (the "average_results" step): the raw
// velocity sums of every cell, rebuilt from its moment record (fp_sample_dev.h), are
// added to the running sums.
#include "fp_sample_dev.h"

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
    if (threadIdx.x < nc) sample_add(sm + threadIdx.x * SA_MPAD, ss + threadIdx.x * SA_SPAD);
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
