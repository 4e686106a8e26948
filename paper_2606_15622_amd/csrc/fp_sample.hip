// fp_sample.hip -- time averaging of cell sums (the "average_results" step): the raw
// velocity sums of every cell, rebuilt from its moment record (fp_sample_dev.h), are
// added to the running sums.
#include "fp_sample_dev.h"

#include <cmath>

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

// Diagnostics of the time-averaged fields, one lane per cell, FP64: the averaged state
// (ratios of the cumulative sums), normalised stress Theta_ij / theta - delta_ij, heat flux
// q^_i = <c_i |c|^2> / (2 theta^1.5) with <c_i |c|^2> = <v_i |v|^2> - U_i |U|^2
// - 3 theta U_i - 2 Theta_ik U_k, and the covariance entropy proxies of the cylinder audit
// (eqs. cyl_theta_def, cyl_entropy_eq, cyl_DG, cyl_entropy_kinG; D_q = |q^|^2 / 5).
// Layout of diag[ncell][24]: 0 particles per sample, 1 number density, 2-4 U, 5 theta,
// 6 T, 7-12 stress (11 12 13 22 23 33), 13-15 q^, 16 ds_eq, 17 D_G, 18 ds_kinG, 19 D_q,
// 20-23 zero; 2-19 NaN without particles or with theta <= 0, D_G and ds_kinG NaN unless
// det(Theta / theta) > 1e-12.
__global__ __launch_bounds__(256) void diag_kernel(int32_t ncell, const double* __restrict__ samp,
                                                   const double* __restrict__ nvol, double dens,
                                                   double m_over_kB, double theta_inf, double n_inf,
                                                   double dg_inf, double* __restrict__ diag) {
    const int32_t k = blockIdx.x * 256 + threadIdx.x;
    if (k >= ncell) return;
    const double* sm = samp + (int64_t)k * SAMP;
    double o[DIAG];
    const double qnan = __builtin_nan("");
#pragma unroll
    for (int i = 0; i < DIAG; ++i) o[i] = i < 20 ? qnan : 0.0;
    const double sN = sm[0], ns = sm[13];
    o[0] = ns > 0.0 ? sN / ns : 0.0;
    o[1] = o[0] * (nvol ? nvol[k] : dens);
    if (sN > 0.0) {
        const double U[3] = {sm[1] / sN, sm[2] / sN, sm[3] / sN};
        double Th[3][3];
        const int ii[6] = {0, 0, 0, 1, 1, 2}, jj[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
        for (int q = 0; q < 6; ++q) Th[ii[q]][jj[q]] = Th[jj[q]][ii[q]] = sm[4 + q] / sN - U[ii[q]] * U[jj[q]];
        const double theta = (Th[0][0] + Th[1][1] + Th[2][2]) / 3.0;
        if (theta > 0.0) {
            const double UU = U[0] * U[0] + U[1] * U[1] + U[2] * U[2];
            double qh[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const double TU = Th[i][0] * U[0] + Th[i][1] * U[1] + Th[i][2] * U[2];
                qh[i] = (sm[10 + i] / sN - U[i] * UU - 3.0 * theta * U[i] - 2.0 * TU) /
                        (2.0 * theta * sqrt(theta));
            }
            o[2] = U[0]; o[3] = U[1]; o[4] = U[2];
            o[5] = theta;
            o[6] = theta * m_over_kB;
#pragma unroll
            for (int q = 0; q < 6; ++q) o[7 + q] = Th[ii[q]][jj[q]] / theta - (ii[q] == jj[q] ? 1.0 : 0.0);
            o[13] = qh[0]; o[14] = qh[1]; o[15] = qh[2];
            const double a = Th[0][0] / theta, b = Th[0][1] / theta, cc = Th[0][2] / theta;
            const double d = Th[1][1] / theta, e = Th[1][2] / theta, f = Th[2][2] / theta;
            const double det = a * (d * f - e * e) - b * (b * f - e * cc) + cc * (b * e - d * cc);
            const double ds_eq = 1.5 * log(theta / theta_inf) - log(o[1] / n_inf);
            // positive-definite Theta only (a singular sample covariance, e.g. of fewer than
            // four particles, has a zero determinant whose sign rounding decides)
            const double dg = det > 1e-12 ? -0.5 * log(det) : qnan;
            o[16] = ds_eq;
            o[17] = dg;
            o[18] = ds_eq - (dg - dg_inf);
            o[19] = (qh[0] * qh[0] + qh[1] * qh[1] + qh[2] * qh[2]) / 5.0;
        }
    }
    double* dst = diag + (int64_t)k * DIAG;
#pragma unroll
    for (int i = 0; i < DIAG; ++i) dst[i] = o[i];
}

int launch_diagnostics(fp_ctx* c, const double* samp, double theta_inf, double n_inf,
                       double dg_inf, double* diag, hipStream_t s) {
    hipLaunchKernelGGL(diag_kernel, dim3((c->ncell + 255) / 256), dim3(256), 0, s, c->ncell, samp,
                       (const double*)c->nvol, c->cfg.fnum_over_vol, c->cfg.mass / c->cfg.kB,
                       theta_inf, n_inf, dg_inf, diag);
    return check_launch(c, "fp_diagnostics");
}

// high-order sums of every cell, one lane per cell: hsamp += [N, N theta, N R_ij (6),
// N <|c|^4> = N tr R, N <|c|^6>] of this step's moment record (cells with particles)
__global__ void sample_high_kernel(int32_t ncell, const double* __restrict__ mom,
                                   double* __restrict__ hsamp) {
    const int32_t cell = blockIdx.x * 256 + threadIdx.x;
    if (cell >= ncell) return;
    const double* m = mom + (int64_t)cell * MOM;
    const double N = m[M_N];
    if (!(N > 0.0)) return;
    double* h = hsamp + (int64_t)cell * SAMP;
    h[0] += N;
    h[1] += N * m[M_TH];
#pragma unroll
    for (int i = 0; i < 6; ++i) h[2 + i] += N * m[M_R + i];
    h[8] += N * ((m[M_R + 0] + m[M_R + 3]) + m[M_R + 5]);
    h[9] += N * m[M_H];
}

// normalised high-order fields of the averaged cells: out[cell][8] = R_ij / theta^2 (6),
// <|c|^4> / theta^2 - 15, <|c|^6> / theta^3 with the particle-weighted averages of hsamp
__global__ void high_order_kernel(int32_t ncell, const double* __restrict__ hsamp,
                                  double* __restrict__ out) {
    const int32_t cell = blockIdx.x * 256 + threadIdx.x;
    if (cell >= ncell) return;
    const double* h = hsamp + (int64_t)cell * SAMP;
    double* o = out + (int64_t)cell * 8;
    if (!(h[0] > 0.0 && h[1] > 0.0)) {
#pragma unroll
        for (int i = 0; i < 8; ++i) o[i] = __longlong_as_double(0x7ff8000000000000LL);
        return;
    }
    const double th = h[1] / h[0];
    const double th2 = th * th;
#pragma unroll
    for (int i = 0; i < 6; ++i) o[i] = h[2 + i] / h[0] / th2;
    o[6] = h[8] / h[0] / th2 - 15.0;
    o[7] = h[9] / h[0] / (th2 * th);
}

int launch_sample_high(fp_ctx* c, const double* mom, double* hsamp, hipStream_t s) {
    hipLaunchKernelGGL(sample_high_kernel, dim3((c->ncell + 255) / 256), dim3(256), 0, s, c->ncell, mom,
                       hsamp);
    return check_launch(c, "fp_sample_high");
}

int launch_high_order(fp_ctx* c, const double* hsamp, double* out, hipStream_t s) {
    hipLaunchKernelGGL(high_order_kernel, dim3((c->ncell + 255) / 256), dim3(256), 0, s, c->ncell, hsamp,
                       out);
    return check_launch(c, "fp_high_order");
}

// surface coefficients of the cylinder from the exchange sums of the re-emissions: one
// thread per bin; each bin holds both halves of the circle (area 2 R (pi / nbins) depth)
__global__ void surface_kernel(int32_t nbins, const double* __restrict__ sums, double scale,
                               double p_inf, double dyn, double U, double* __restrict__ out) {
    const int32_t b = blockIdx.x * 256 + threadIdx.x;
    if (b >= nbins) return;
    const double* w = sums + 4 * (int64_t)b;
    double* o = out + 4 * (int64_t)b;
    o[0] = ((double)b + 0.5) * 180.0 / (double)nbins;
    o[1] = (scale * w[1] - p_inf) / dyn;
    o[2] = scale * w[2] / dyn;
    o[3] = scale * w[3] / (dyn * U);
}

int launch_surface(fp_ctx* c, const double* sums, int32_t nbins, double t_total, double* out,
                   hipStream_t s) {
    const fp_config& g = c->cfg;
    const double area = 2.0 * g.circle[2] * (3.14159265358979323846 / (double)nbins) * g.depth;
    const double U = std::sqrt(g.u_inf[0] * g.u_inf[0] + g.u_inf[1] * g.u_inf[1] + g.u_inf[2] * g.u_inf[2]);
    const double rho = g.n_inf * g.mass;
    const double dyn = 0.5 * rho * U * U;
    const double scale = g.mass * g.fnum / (area * t_total);
    hipLaunchKernelGGL(surface_kernel, dim3((nbins + 255) / 256), dim3(256), 0, s, nbins, sums, scale,
                       g.n_inf * g.kB * g.T_inf, dyn, U, out);
    return check_launch(c, "fp_surface_coefficients");
}

int launch_sample(fp_ctx* c, const double* mom, double* samp, hipStream_t s) {
    hipLaunchKernelGGL(sample_kernel, dim3((c->ncell + SA_CELLS - 1) / SA_CELLS), dim3(SA_BLOCK), 0, s,
                       c->ncell, mom, samp);
    return check_launch(c, "fp_sample");
}

}  // namespace fpg
