// fp_closure.hip -- batched exact closure: one lane per cell, FP64 in registers.
//
// Builds the theta-normalised 9x9 system of every cell (fp_closure_dev.h) and solves it
// by LU with partial pivoting, fully unrolled: the pivot row swap is a predicated select
// on every candidate row, so the 90 doubles of the augmented matrix stay in VGPRs.
#include "fp_closure_dev.h"

namespace fpg {

constexpr int CL_BLOCK = 64;

// NN = false: exact solve.  NN = true: the network's standardised outputs ynn[cell][16]
// are de-standardised (ysec = y_mean[16], y_std[16]) into normalised coefficients and
// accepted if the residual of the normalised system satisfies
// |A y - b| <= tol_abs + tol_rel |b|; otherwise the cell is solved exactly.  With
// tol_abs = +inf every finite output is accepted; a non-finite one is solved exactly, or,
// when the records hold moments through third order only (low), takes the Langevin drift
// (status SINGULAR).  relax < 1 blends the accepted coefficients with the cell's previous
// ones: C = relax C_net + (1 - relax) C_prev (the same for Gamma), where the previous
// record carries coefficients.
template <bool NN>
__global__ __launch_bounds__(CL_BLOCK) void closure_kernel(fp_config g, int32_t ncell,
                                                            const double* __restrict__ mom,
                                                            double* __restrict__ rec,
                                                            int32_t* __restrict__ status,
                                                            const float* __restrict__ ynn,
                                                            const float* __restrict__ ysec,
                                                            double tol_abs, double tol_rel,
                                                            const double* __restrict__ nvol,
                                                            double relax) {
    const int32_t cell = blockIdx.x * CL_BLOCK + threadIdx.x;
    if (cell >= ncell) return;
    double m[31];
    const double* src = mom + (int64_t)cell * MOM;
#pragma unroll
    for (int i = 0; i < 31; ++i) m[i] = src[i];
    bool finite = true;
#pragma unroll
    for (int i = 0; i < 31; ++i) finite = finite && isfinite(m[i]);
    const double N = m[M_N], theta = m[M_TH];
    int st = FP_CELL_OK;
    if (N <= 1.0)
        st = FP_CELL_EMPTY;
    else if (!finite)
        st = FP_CELL_NONFINITE;
    else if (!(theta > 0.0))
        st = FP_CELL_EMPTY;
    double out[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) out[i] = 0.0;
    if (st != FP_CELL_OK) {
        out[R_E] = 1.0;
        out[R_TH] = finite ? theta : 0.0;
    } else {
        const double tau = cell_tau(g, N * (nvol ? nvol[cell] : g.fnum_over_vol), theta);
        const double eps2 = g.eps_hat / (theta * tau);
        double y[9];
        if (N < (double)g.n_min) {
            st = FP_CELL_FEW;
        } else {
            bool accepted = false;
            const bool unchecked = NN && tol_abs == INFINITY;   // accept any finite output
            if (NN) {
                const float* yo = ynn + (int64_t)cell * 16;
#pragma unroll
                for (int i = 0; i < 9; ++i) y[i] = (double)yo[i] * (double)ysec[16 + i] + (double)ysec[i];
                y[0] += 5.0 * g.eps_hat;
                y[3] += 5.0 * g.eps_hat;
                y[5] += 5.0 * g.eps_hat;
                if (unchecked) {
                    accepted = true;
#pragma unroll
                    for (int i = 0; i < 9; ++i) accepted = accepted && isfinite(y[i]);
                }
            }
            if (!accepted && NN && unchecked && g.moment_order == 3) {
                st = FP_CELL_SINGULAR;   // no system to fall back on: Langevin drift
            } else if (!accepted) {
                CellSystem s;
                build_system(m, g.eps_hat, s);
                if (NN && !unchecked) {
                    double rr = 0.0, bb = 0.0;
#pragma unroll
                    for (int i = 0; i < 9; ++i) {
                        double t = -s.a[i][9];
#pragma unroll
                        for (int k = 0; k < 9; ++k) t = fma(s.a[i][k], y[k], t);
                        rr = fma(t, t, rr);
                        bb = fma(s.a[i][9], s.a[i][9], bb);
                    }
                    accepted = sqrt(rr) <= tol_abs + tol_rel * sqrt(bb);
#pragma unroll
                    for (int i = 0; i < 9; ++i) accepted = accepted && isfinite(y[i]);
                }
                if (!accepted) {
                    const bool ok = lu_solve(s, g.pivot_tol, y);
                    bool fin = true;
#pragma unroll
                    for (int i = 0; i < 9; ++i) fin = fin && isfinite(y[i]);
                    if (!ok || !fin) st = FP_CELL_SINGULAR;
                    else if (NN) st = FP_CELL_NN_FALLBACK;
                }
            }
            if (accepted) st = FP_CELL_NN;
        }
        if (st == FP_CELL_OK || st == FP_CELL_NN || st == FP_CELL_NN_FALLBACK) {
            const double it = 1.0 / tau;
            const double ig = 1.0 / (tau * sqrt(theta));
#pragma unroll
            for (int i = 0; i < 6; ++i) out[R_C + i] = y[i] * it;
#pragma unroll
            for (int i = 0; i < 3; ++i) out[R_G + i] = y[6 + i] * ig;
            out[R_EPS2] = eps2;
            if (NN && st == FP_CELL_NN && relax < 1.0) {
                const double* prev = rec + (int64_t)cell * REC;
                const int pst = (int)prev[R_ST];
                if (pst == FP_CELL_OK || pst == FP_CELL_NN || pst == FP_CELL_NN_FALLBACK) {
#pragma unroll
                    for (int i = 0; i < 9; ++i)
                        out[R_C + i] = relax * out[R_C + i] + (1.0 - relax) * prev[R_C + i];
                }
            }
        }
        out[R_TAU] = tau;
        out[R_TH] = theta;
        out[R_E] = exp(-g.dt / tau);
        out[R_SIG] = sqrt(theta * (1.0 - exp(-2.0 * g.dt / tau)));
    }
    out[R_ST] = (double)st;
    double* dst = rec + (int64_t)cell * REC;
#pragma unroll
    for (int i = 0; i < 16; ++i) dst[i] = out[i];
    status[cell] = st;
}

int launch_closure(fp_ctx* c, const double* mom, double* rec, int32_t* status, hipStream_t s) {
    const int grid = (c->ncell + CL_BLOCK - 1) / CL_BLOCK;
    hipLaunchKernelGGL(closure_kernel<false>, dim3(grid), dim3(CL_BLOCK), 0, s, c->cfg, c->ncell,
                       mom, rec, status, (const float*)nullptr, (const float*)nullptr, 0.0, 0.0,
                       (const double*)c->nvol, 1.0);
    return check_launch(c, "fp_closure_solve");
}

int launch_closure_nn(fp_ctx* c, const float* ynn, const float* ysec, double tol_abs,
                      double tol_rel, double relax, const double* mom, double* rec, int32_t* status,
                      hipStream_t s) {
    const int grid = (c->ncell + CL_BLOCK - 1) / CL_BLOCK;
    hipLaunchKernelGGL(closure_kernel<true>, dim3(grid), dim3(CL_BLOCK), 0, s, c->cfg, c->ncell,
                       mom, rec, status, ynn, ysec, tol_abs, tol_rel, (const double*)c->nvol, relax);
    return check_launch(c, "fp_closure_nn (check)");
}

}  // namespace fpg
