// fp_backward.hip -- reverse mode through the exact closure and the segmented moments.
//
// Forward (per cell): moments m(v) -> normalised system A(m_hat) y_hat = b(m_hat) ->
// coefficients Ct = y_hat_C / tau, Gamma = y_hat_G / (tau sqrt(theta)), with
// tau = 2 mu(T) / p (eq. tau) depending on theta through mu ~ T^omega and p ~ T.
// Reverse:
//   y_hat_bar from the coefficient gradients (and tau_bar, theta_bar of the scaling);
//   b_bar = A^-T y_hat_bar, A_bar = -b_bar y_hat^T        (adjoint of the linear solve)
//   m_hat_bar by transposing the entry-by-entry assembly of A and b (fp_closure_dev.h),
//   raw moments and theta by the theta scaling, theta = tr(P) / 3 folded into P_bar;
//   v_bar_p = (1/N) (G(c_p) - <G>), G(c) = sum_k m_bar_k grad f_k(c), recomputed from
//   the particle velocities (no per-particle moments are stored).
#include "fp_closure_dev.h"

namespace fpg {

constexpr int BW_BLOCK = 64;

// solve A^T x = r with partial pivoting (A is overwritten); false if a pivot < tol
__device__ __forceinline__ bool lu_solve_transposed(CellSystem& s, const double r[9], double tol,
                                                    double x[9]) {
    CellSystem t;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
#pragma unroll
        for (int k = 0; k < 9; ++k) t.a[i][k] = s.a[k][i];
        t.a[i][9] = r[i];
    }
    return lu_solve(t, tol, x);
}

__global__ __launch_bounds__(BW_BLOCK) void closure_backward_kernel(
    fp_config g, int32_t ncell, const double* __restrict__ mom, const double* __restrict__ rec,
    const double* __restrict__ ybar, double* __restrict__ mbar) {
    const int32_t cell = blockIdx.x * BW_BLOCK + threadIdx.x;
    if (cell >= ncell) return;
    const double* m = mom + (int64_t)cell * MOM;
    const double* r = rec + (int64_t)cell * REC;
    double* out = mbar + (int64_t)cell * MOM;
    double o[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) o[i] = 0.0;
    const int st = (int)r[R_ST];
    if (st == FP_CELL_OK) {
        double mm[31];
#pragma unroll
        for (int i = 0; i < 31; ++i) mm[i] = m[i];
        const double th = mm[M_TH], tau = r[R_TAU], sth = sqrt(th);
        const double e = g.eps_hat;
        double yh[9], yhb[9];
#pragma unroll
        for (int i = 0; i < 6; ++i) yh[i] = r[R_C + i] * tau;
#pragma unroll
        for (int i = 0; i < 3; ++i) yh[6 + i] = r[R_G + i] * tau * sth;
        const double* yb = ybar + (int64_t)cell * 16;
        double sC = 0.0, sG = 0.0;
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            yhb[i] = yb[i] / tau;
            sC = fma(yb[i], yh[i], sC);
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            yhb[6 + i] = yb[6 + i] / (tau * sth);
            sG = fma(yb[6 + i], yh[6 + i], sG);
        }
        const double taub = -sC / (tau * tau) - sG / (tau * tau * sth);
        double thb = -0.5 * sG / (tau * th * sth);
        thb += taub * tau * (g.omega - 1.0) / th;   // tau ~ T^(omega - 1) at fixed N

        CellSystem s;
        build_system(mm, e, s);
        double bb[9];
        lu_solve_transposed(s, yhb, 0.0, bb);
        // A_bar = -b_bar y_hat^T, b_bar = bb
        auto Ab = [&](int i, int k) { return -bb[i] * yh[k]; };
        // normalised-moment adjoints
        double P11 = 0, P12 = 0, P13 = 0, P22 = 0, P23 = 0, P33 = 0;
        double S1 = 0, S2 = 0, S3 = 0, Q = 0;
        double T111 = 0, T112 = 0, T113 = 0, T122 = 0, T123 = 0, T133 = 0, T222 = 0, T223 = 0,
               T233 = 0, T333 = 0;
        double R11 = 0, R12 = 0, R13 = 0, R22 = 0, R23 = 0, R33 = 0, W1 = 0, W2 = 0, W3 = 0;
        // V | W | Q6 rows
        P11 += 2 * Ab(0, 0); P12 += 2 * Ab(0, 1); P13 += 2 * Ab(0, 2); S1 += 2 * Ab(0, 6);
        R11 += 2 * e * bb[0];
        P12 += Ab(1, 0); P22 += Ab(1, 1); P11 += Ab(1, 1); P23 += Ab(1, 2); P12 += Ab(1, 3);
        P13 += Ab(1, 4); S2 += Ab(1, 6); S1 += Ab(1, 7); R12 += 2 * e * bb[1];
        P13 += Ab(2, 0); P23 += Ab(2, 1); P33 += Ab(2, 2); P11 += Ab(2, 2); P12 += Ab(2, 4);
        P13 += Ab(2, 5); S3 += Ab(2, 6); S1 += Ab(2, 8); R13 += 2 * e * bb[2];
        P12 += 2 * Ab(3, 1); P22 += 2 * Ab(3, 3); P23 += 2 * Ab(3, 4); S2 += 2 * Ab(3, 7);
        R22 += 2 * e * bb[3];
        P13 += Ab(4, 1); P12 += Ab(4, 2); P23 += Ab(4, 3); P33 += Ab(4, 4); P22 += Ab(4, 4);
        P23 += Ab(4, 5); S3 += Ab(4, 7); S2 += Ab(4, 8); R23 += 2 * e * bb[4];
        P13 += 2 * Ab(5, 2); P23 += 2 * Ab(5, 4); P33 += 2 * Ab(5, 5); S3 += 2 * Ab(5, 8);
        R33 += 2 * e * bb[5];
        // X^T rows
        S1 += Ab(6, 0); T111 += 2 * Ab(6, 0); S2 += Ab(6, 1); T112 += 4 * Ab(6, 1);
        S3 += Ab(6, 2); T113 += 4 * Ab(6, 2); T122 += 2 * Ab(6, 3); T123 += 4 * Ab(6, 4);
        T133 += 2 * Ab(6, 5);
        T112 += 2 * Ab(7, 0); S1 += Ab(7, 1); T122 += 4 * Ab(7, 1); T123 += 4 * Ab(7, 2);
        S2 += Ab(7, 3); T222 += 2 * Ab(7, 3); S3 += Ab(7, 4); T223 += 4 * Ab(7, 4);
        T233 += 2 * Ab(7, 5);
        T113 += 2 * Ab(8, 0); T123 += 4 * Ab(8, 1); S1 += Ab(8, 2); T133 += 4 * Ab(8, 2);
        T223 += 2 * Ab(8, 3); S2 += Ab(8, 4); T233 += 4 * Ab(8, 4); S3 += Ab(8, 5);
        T333 += 2 * Ab(8, 5);
        // Z block
        Q += Ab(6, 6) + Ab(7, 7) + Ab(8, 8);
        R11 += 2 * Ab(6, 6); P11 -= 6 * Ab(6, 6);
        R22 += 2 * Ab(7, 7); P22 -= 6 * Ab(7, 7);
        R33 += 2 * Ab(8, 8); P33 -= 6 * Ab(8, 8);
        R12 += 2 * (Ab(6, 7) + Ab(7, 6)); P12 -= 6 * (Ab(6, 7) + Ab(7, 6));
        R13 += 2 * (Ab(6, 8) + Ab(8, 6)); P13 -= 6 * (Ab(6, 8) + Ab(8, 6));
        R23 += 2 * (Ab(7, 8) + Ab(8, 7)); P23 -= 6 * (Ab(7, 8) + Ab(8, 7));
        // heat-flux right-hand side: 5/3 S_i + e (3 W_i - 3 S_i - 2 (P S)_i)
        {
            const double i1 = 1.0 / th, i15 = i1 / sth;
            const double pP11 = mm[M_P + 0] * i1, pP12 = mm[M_P + 1] * i1, pP13 = mm[M_P + 2] * i1;
            const double pP22 = mm[M_P + 3] * i1, pP23 = mm[M_P + 4] * i1, pP33 = mm[M_P + 5] * i1;
            const double sS1 = (mm[M_T + 0] + mm[M_T + 3] + mm[M_T + 5]) * i15;
            const double sS2 = (mm[M_T + 1] + mm[M_T + 6] + mm[M_T + 8]) * i15;
            const double sS3 = (mm[M_T + 2] + mm[M_T + 7] + mm[M_T + 9]) * i15;
            const double b6 = bb[6], b7 = bb[7], b8 = bb[8];
            const double k = 5.0 / 3.0 - 3.0 * e;
            S1 += k * b6; S2 += k * b7; S3 += k * b8;
            W1 += 3 * e * b6; W2 += 3 * e * b7; W3 += 3 * e * b8;
            // -2 e (P S)_i
            P11 -= 2 * e * b6 * sS1; P12 -= 2 * e * (b6 * sS2 + b7 * sS1); P13 -= 2 * e * (b6 * sS3 + b8 * sS1);
            P22 -= 2 * e * b7 * sS2; P23 -= 2 * e * (b7 * sS3 + b8 * sS2); P33 -= 2 * e * b8 * sS3;
            S1 -= 2 * e * (pP11 * b6 + pP12 * b7 + pP13 * b8);
            S2 -= 2 * e * (pP12 * b6 + pP22 * b7 + pP23 * b8);
            S3 -= 2 * e * (pP13 * b6 + pP23 * b7 + pP33 * b8);
        }
        // S_i = T_ikk, Q = R_kk
        T111 += S1; T122 += S1; T133 += S1;
        T112 += S2; T222 += S2; T233 += S2;
        T113 += S3; T223 += S3; T333 += S3;
        R11 += Q; R22 += Q; R33 += Q;
        // normalised -> raw moments, collecting theta
        const double i1 = 1.0 / th, i15 = i1 / sth, i2 = i1 * i1, i25 = i2 / sth;
        const double Pb[6] = {P11, P12, P13, P22, P23, P33};
        const double Tb[10] = {T111, T112, T113, T122, T123, T133, T222, T223, T233, T333};
        const double Rb[6] = {R11, R12, R13, R22, R23, R33};
        const double Wb[3] = {W1, W2, W3};
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            o[M_P + q] = Pb[q] * i1;
            thb -= Pb[q] * mm[M_P + q] * i1 * i1;
            o[M_R + q] = Rb[q] * i2;
            thb -= 2.0 * Rb[q] * mm[M_R + q] * i2 * i1;
        }
#pragma unroll
        for (int q = 0; q < 10; ++q) {
            o[M_T + q] = Tb[q] * i15;
            thb -= 1.5 * Tb[q] * mm[M_T + q] * i15 * i1;
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            o[M_W + q] = Wb[q] * i25;
            thb -= 2.5 * Wb[q] * mm[M_W + q] * i25 * i1;
        }
        // theta = (P11 + P22 + P33) / 3
        o[M_P + 0] += thb / 3.0;
        o[M_P + 3] += thb / 3.0;
        o[M_P + 5] += thb / 3.0;
    }
#pragma unroll
    for (int i = 0; i < 32; ++i) out[i] = o[i];
}

// G(c) = sum_k mbar_k grad f_k(c) for the monomials of the moment record
struct MomAdj {
    double Ps[3][3];     // symmetric: sum_ij Ps_ij c_i c_j reproduces sum_stored P_bar_ij c_i c_j
    double Ts[10];       // stored T_bar divided by the multiplicity of the index triple
    double Rs[3][3];
    double W[3];
    double H;
};

__device__ __forceinline__ void grad_G(const MomAdj& a, double c0, double c1, double c2, double G[3]) {
    const double c[3] = {c0, c1, c2};
    const double cc = c0 * c0 + c1 * c1 + c2 * c2;
    // P: 2 Ps c
    double Pc[3], Rc[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        Pc[i] = a.Ps[i][0] * c0 + a.Ps[i][1] * c1 + a.Ps[i][2] * c2;
        Rc[i] = a.Rs[i][0] * c0 + a.Rs[i][1] * c1 + a.Rs[i][2] * c2;
    }
    const double cRc = c0 * Rc[0] + c1 * Rc[1] + c2 * Rc[2];
    const double Wc = a.W[0] * c0 + a.W[1] * c1 + a.W[2] * c2;
    const double c4 = cc * cc;
    // T: 3 sum_jk Ts_ajk c_j c_k (fully symmetric tensor from the 10 stored entries)
    const double t111 = a.Ts[0], t112 = a.Ts[1], t113 = a.Ts[2], t122 = a.Ts[3], t123 = a.Ts[4],
                 t133 = a.Ts[5], t222 = a.Ts[6], t223 = a.Ts[7], t233 = a.Ts[8], t333 = a.Ts[9];
    const double q00 = c0 * c0, q01 = c0 * c1, q02 = c0 * c2, q11 = c1 * c1, q12 = c1 * c2, q22 = c2 * c2;
    const double TG0 = t111 * q00 + t122 * q11 + t133 * q22 + 2 * (t112 * q01 + t113 * q02 + t123 * q12);
    const double TG1 = t112 * q00 + t222 * q11 + t233 * q22 + 2 * (t122 * q01 + t123 * q02 + t223 * q12);
    const double TG2 = t113 * q00 + t223 * q11 + t333 * q22 + 2 * (t123 * q01 + t133 * q02 + t233 * q12);
    const double TG[3] = {TG0, TG1, TG2};
#pragma unroll
    for (int i = 0; i < 3; ++i)
        G[i] = 2.0 * Pc[i] + 3.0 * TG[i] + 2.0 * Rc[i] * cc + 2.0 * cRc * c[i] + a.W[i] * c4 +
               4.0 * Wc * cc * c[i] + 6.0 * a.H * c4 * c[i];
}

__device__ __forceinline__ void load_adj(const double* mb, MomAdj& a, double Ub[3]) {
    const double thb = mb[M_TH] / 3.0;
    const double P[6] = {mb[M_P + 0] + thb, mb[M_P + 1], mb[M_P + 2], mb[M_P + 3] + thb, mb[M_P + 4],
                         mb[M_P + 5] + thb};
    a.Ps[0][0] = P[0]; a.Ps[1][1] = P[3]; a.Ps[2][2] = P[5];
    a.Ps[0][1] = a.Ps[1][0] = 0.5 * P[1];
    a.Ps[0][2] = a.Ps[2][0] = 0.5 * P[2];
    a.Ps[1][2] = a.Ps[2][1] = 0.5 * P[4];
    const double R[6] = {mb[M_R + 0], mb[M_R + 1], mb[M_R + 2], mb[M_R + 3], mb[M_R + 4], mb[M_R + 5]};
    a.Rs[0][0] = R[0]; a.Rs[1][1] = R[3]; a.Rs[2][2] = R[5];
    a.Rs[0][1] = a.Rs[1][0] = 0.5 * R[1];
    a.Rs[0][2] = a.Rs[2][0] = 0.5 * R[2];
    a.Rs[1][2] = a.Rs[2][1] = 0.5 * R[4];
    // multiplicities of 111 112 113 122 123 133 222 223 233 333
    const double mult[10] = {1, 3, 3, 3, 6, 3, 1, 3, 3, 1};
#pragma unroll
    for (int q = 0; q < 10; ++q) a.Ts[q] = mb[M_T + q] / mult[q];
#pragma unroll
    for (int i = 0; i < 3; ++i) a.W[i] = mb[M_W + i];
    a.H = mb[M_H];
    Ub[0] = mb[M_U]; Ub[1] = mb[M_U + 1]; Ub[2] = mb[M_U + 2];
}

constexpr int MB_BLOCK = 256;

template <typename T, int G>
__global__ __launch_bounds__(MB_BLOCK) void moments_backward_kernel(
    int32_t ncell, const int32_t* __restrict__ offsets, const T* __restrict__ vx,
    const T* __restrict__ vy, const T* __restrict__ vz, const double* __restrict__ mom,
    const double* __restrict__ mbar, double* __restrict__ gx, double* __restrict__ gy,
    double* __restrict__ gz) {
    const int64_t gt = (int64_t)blockIdx.x * MB_BLOCK + threadIdx.x;
    const int32_t cell = (int32_t)(gt / G);
    const int lg = (int)(gt % G);
    const bool in = cell < ncell;
    int32_t b = 0, n = 0;
    MomAdj a{};
    double Ub[3] = {0, 0, 0}, U[3] = {0, 0, 0};
    if (in) {
        b = offsets[cell];
        n = offsets[cell + 1] - b;
        load_adj(mbar + (int64_t)cell * MOM, a, Ub);
        const double* m = mom + (int64_t)cell * MOM;
        U[0] = m[M_U]; U[1] = m[M_U + 1]; U[2] = m[M_U + 2];
    }
    double s0 = 0, s1 = 0, s2 = 0;
    for (int32_t j = lg; j < n; j += G) {
        double Gv[3];
        grad_G(a, (double)vx[b + j] - U[0], (double)vy[b + j] - U[1], (double)vz[b + j] - U[2], Gv);
        s0 += Gv[0]; s1 += Gv[1]; s2 += Gv[2];
    }
    s0 = group_sum<G>(s0);
    s1 = group_sum<G>(s1);
    s2 = group_sum<G>(s2);
    if (n == 0) return;
    const double inv = 1.0 / (double)n;
    const double m0 = s0 * inv, m1 = s1 * inv, m2 = s2 * inv;
    for (int32_t j = lg; j < n; j += G) {
        double Gv[3];
        grad_G(a, (double)vx[b + j] - U[0], (double)vy[b + j] - U[1], (double)vz[b + j] - U[2], Gv);
        gx[b + j] = (Gv[0] - m0 + Ub[0]) * inv;
        gy[b + j] = (Gv[1] - m1 + Ub[1]) * inv;
        gz[b + j] = (Gv[2] - m2 + Ub[2]) * inv;
    }
}

template <typename T, int G>
static void mb_launch(fp_ctx* c, const fp_particles* p, const int32_t* off, const double* mom,
                      const double* mbar, double* gx, double* gy, double* gz, hipStream_t s) {
    const int64_t threads = (int64_t)c->ncell * G;
    const unsigned grid = (unsigned)((threads + MB_BLOCK - 1) / MB_BLOCK);
    hipLaunchKernelGGL((moments_backward_kernel<T, G>), dim3(grid), dim3(MB_BLOCK), 0, s, c->ncell, off,
                       (const T*)p->vx, (const T*)p->vy, (const T*)p->vz, mom, mbar, gx, gy, gz);
}

template <typename T>
static void mb_dispatch(fp_ctx* c, const fp_particles* p, const int32_t* off, const double* mom,
                        const double* mbar, double* gx, double* gy, double* gz, hipStream_t s) {
    switch (lanes_per_cell(c, p->n)) {
        case 4: mb_launch<T, 4>(c, p, off, mom, mbar, gx, gy, gz, s); break;
        case 8: mb_launch<T, 8>(c, p, off, mom, mbar, gx, gy, gz, s); break;
        case 16: mb_launch<T, 16>(c, p, off, mom, mbar, gx, gy, gz, s); break;
        case 32: mb_launch<T, 32>(c, p, off, mom, mbar, gx, gy, gz, s); break;
        default: mb_launch<T, 64>(c, p, off, mom, mbar, gx, gy, gz, s); break;
    }
}

}  // namespace fpg

using namespace fpg;

extern "C" int fp_closure_solve_backward(fp_ctx* c, const double* mom, const double* rec,
                                         const double* ybar, double* mombar, hipStream_t s) {
    if (!c || !mom || !rec || !ybar || !mombar)
        return set_err(c, FP_EINVAL, "fp_closure_solve_backward: bad argument");
    hipLaunchKernelGGL(closure_backward_kernel, dim3((c->ncell + BW_BLOCK - 1) / BW_BLOCK),
                       dim3(BW_BLOCK), 0, s, c->cfg, c->ncell, mom, rec, ybar, mombar);
    return check_launch(c, "fp_closure_solve_backward");
}

extern "C" int fp_moments_backward(fp_ctx* c, const fp_particles* p, const int32_t* offsets,
                                   const double* mom, const double* mombar, double* vbar_x,
                                   double* vbar_y, double* vbar_z, hipStream_t s) {
    if (!c || !p || !offsets || !mom || !mombar || !vbar_x || !vbar_y || !vbar_z || p->n < 0 ||
        p->n > c->cfg.capacity || (p->n > 0 && (!p->vx || !p->vy || !p->vz)))
        return set_err(c, FP_EINVAL, "fp_moments_backward: bad argument");
    if (c->cfg.precision == FP_F32)
        mb_dispatch<float>(c, p, offsets, mom, mombar, vbar_x, vbar_y, vbar_z, s);
    else
        mb_dispatch<double>(c, p, offsets, mom, mombar, vbar_x, vbar_y, vbar_z, s);
    return check_launch(c, "fp_moments_backward");
}
