// fp_lite.hip -- the paper's LITE surrogate on MFMA: 16 low-order inputs -> 256 -> 256 ->
// 256 -> 256 (ReLU) -> 9 (Secs. "Phase 1-2", "Neural Network Architecture", "Phase 3").
//
// Inference is one kernel: every wave keeps 32 cells (the MFMA columns) in registers
// through all five layers, and the workgroup stages one layer's BF16 weights at a time
// through LDS (the 408 KB of weights do not fit in LDS together; a 256 x 256 layer is
// 128 KB).  The activations never leave the registers: the columns of every next-layer
// weight matrix are permuted so that the rows a lane holds after one layer are exactly
// the k-slots it feeds into the next (the permutation of fp_nn.hip, over 16 k-steps).
// Training runs layer by layer over batches in HBM (MFMA forward, backward and split-K
// weight gradients, fixed-order reductions: bitwise reproducible) with Adam on FP32
// master weights.
//
// Inputs (solver units, then standardised): rho, T, U (3), Pi (11 12 13 22 23 33), q (3),
// DM2 = <|c|^2>, nu = 1/tau; targets Ct (6) and Gamma (3) of the update record, in solver
// units, standardised.
#include "fp_closure_dev.h"

#include <cmath>
#include <new>
#include <string>

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

namespace fpg {
namespace lite {

constexpr int NF = 16, NH = 256, NO = 16;
constexpr int NT = NH / 32;   // 32-row output tiles of a hidden layer
constexpr int KS = NH / 16;   // 16-row k-steps of a hidden layer's input
// flat FP32 parameters (include/fp.h)
constexpr int64_t OFF_W1 = 0, OFF_B1 = 4096, OFF_W2 = 4352, OFF_B2 = 69888, OFF_W3 = 70144,
                  OFF_B3 = 135680, OFF_W4 = 135936, OFF_B4 = 201472, OFF_W5 = 201728,
                  OFF_B5 = 205824, OFF_XM = 205840, OFF_XS = 205856, OFF_YM = 205872,
                  OFF_YS = 205888, N_PARAMS = 205904, N_TRAIN = 205840;
// BF16 fragment image: layer 1 NT tiles x 1 k-step, layers 2-4 NT x KS, layer 5 1 x KS
constexpr int IMG_L1 = 0, IMG_L2 = 4096, IMG_L3 = 69632, IMG_L4 = 135168, IMG_L5 = 200704,
              IMG_BF = 208896;
// FP32 section: biases, scalers, and an identity output scaler (16 zeros, 16 ones) for the
// check kernel, which receives normalised coefficients
constexpr int SEC_B1 = 0, SEC_B2 = 256, SEC_B3 = 512, SEC_B4 = 768, SEC_B5 = 1024, SEC_XM = 1040,
              SEC_XS = 1056, SEC_YM = 1072, SEC_YS = 1088, SEC_ID = 1104, SEC_N = 1136;
constexpr int TRAIN_CHUNK = 1024;
constexpr int INF_BLOCK = 512;                  // 8 waves, 256 cells per workgroup
constexpr int LDS_BF = NT * KS * 512;           // one hidden layer: 65536 BF16 (128 KB)

static_assert(IMG_L2 - IMG_L1 == NT * 512 && IMG_L3 - IMG_L2 == LDS_BF && IMG_L5 - IMG_L4 == LDS_BF &&
                  IMG_BF - IMG_L5 == KS * 512,
              "image layout");
static_assert(OFF_B5 + NO == N_TRAIN && OFF_YS + NO == N_PARAMS, "parameter layout");

__device__ __forceinline__ f32x16 mfma32(bf16x8 a, bf16x8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// k-slot K of a hidden layer's input holds activation row perm_k(K) of the previous layer
__device__ __forceinline__ int perm_k(int K) {
    const int s = K >> 4, h = (K >> 3) & 1, i = K & 7;
    return 16 * s + 8 * (i >> 2) + 4 * h + (i & 3);
}

// ---------------------------------------------------------------------------------------
// FP32 parameters -> permuted BF16 fragment image ([tile][k-step][lane][8]) + FP32 section
__global__ void lite_pack_kernel(const float* __restrict__ p, __bf16* __restrict__ img,
                                 float* __restrict__ sec) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < IMG_BF) {
        int base, ks_n, layer;
        if (t < IMG_L2) { layer = 1; base = IMG_L1; ks_n = 1; }
        else if (t < IMG_L3) { layer = 2; base = IMG_L2; ks_n = KS; }
        else if (t < IMG_L4) { layer = 3; base = IMG_L3; ks_n = KS; }
        else if (t < IMG_L5) { layer = 4; base = IMG_L4; ks_n = KS; }
        else { layer = 5; base = IMG_L5; ks_n = KS; }
        const int e = t - base;
        const int i = e & 7, lane = (e >> 3) & 63, frag = e >> 9;
        const int ks = frag % ks_n, mt = frag / ks_n;
        const int m = mt * 32 + (lane & 31), h = lane >> 5;
        const int K = ks * 16 + 8 * h + i;
        float v;
        if (layer == 1) v = p[OFF_W1 + m * NF + K];
        else if (layer == 2) v = p[OFF_W2 + m * NH + perm_k(K)];
        else if (layer == 3) v = p[OFF_W3 + m * NH + perm_k(K)];
        else if (layer == 4) v = p[OFF_W4 + m * NH + perm_k(K)];
        else v = m < NO ? p[OFF_W5 + m * NH + perm_k(K)] : 0.0f;
        img[t] = (__bf16)v;
    }
    if (t < SEC_N) {
        float v;
        if (t < SEC_B5) v = p[OFF_B1 + (t / NH) * (OFF_B2 - OFF_B1) + t % NH];
        else if (t < SEC_XM) v = p[OFF_B5 + t - SEC_B5];
        else if (t < SEC_XS) v = p[OFF_XM + t - SEC_XM];
        else if (t < SEC_YM) v = p[OFF_XS + t - SEC_XS];
        else if (t < SEC_YS) v = p[OFF_YM + t - SEC_YM];
        else if (t < SEC_ID) v = p[OFF_YS + t - SEC_YS];
        else v = t < SEC_ID + 16 ? 0.0f : 1.0f;
        sec[t] = v;
    }
}

// the 16 inputs of one cell (FP64 arithmetic, FP32 result) and its tau (eq. tau):
// rho, T, U, Pi_ij = rho (P_ij - theta delta_ij), q_i = rho S_i / 2, DM2 = 3 theta, nu = 1/tau
__device__ __forceinline__ void cell_inputs(const fp_config& g, const double* __restrict__ m, double nv,
                                            float f[NF], double& tau) {
    const double N = m[M_N], th = m[M_TH];
    const double ndens = N * nv;
    const double rho = ndens * g.mass;
    tau = cell_tau(g, ndens, th);
    f[0] = (float)rho;
    f[1] = (float)(th * g.mass / g.kB);
#pragma unroll
    for (int q = 0; q < 3; ++q) f[2 + q] = (float)m[M_U + q];
    const double d6[6] = {1, 0, 0, 1, 0, 1};
#pragma unroll
    for (int q = 0; q < 6; ++q) f[5 + q] = (float)(rho * (m[M_P + q] - th * d6[q]));
    // S_i = T_ikk: T111 T112 T113 T122 T123 T133 T222 T223 T233 T333
    const double S1 = m[M_T + 0] + m[M_T + 3] + m[M_T + 5];
    const double S2 = m[M_T + 1] + m[M_T + 6] + m[M_T + 8];
    const double S3 = m[M_T + 2] + m[M_T + 7] + m[M_T + 9];
    f[11] = (float)(0.5 * rho * S1);
    f[12] = (float)(0.5 * rho * S2);
    f[13] = (float)(0.5 * rho * S3);
    f[14] = (float)(3.0 * th);
    f[15] = (float)(1.0 / tau);
}

// ---------------------------------------------------------------------------------------
// fused inference.  mode 0: y[cell][16] = standardised network outputs (rows 9..15 zero);
// mode 1: y[cell][16] = normalised coefficients [tau Ct - 5 eps_hat I (6), tau sqrt(theta)
// Gamma (3), 0...] from the de-standardised outputs, for the check kernel with the
// identity scaler.  Cells without inputs (N <= 1 or theta <= 0) are evaluated on zero
// inputs in mode 0 and get zeros in mode 1.
template <int MT_GROUP>
__device__ __forceinline__ void hidden_layer(const __bf16* __restrict__ w, const float* __restrict__ bias,
                                             const bf16x8 (&bin)[KS], bf16x8 (&bout)[KS], int lane) {
    const int h = lane >> 5;
#pragma unroll
    for (int mp = 0; mp < NT; mp += MT_GROUP) {
        f32x16 acc[MT_GROUP];
#pragma unroll
        for (int t = 0; t < MT_GROUP; ++t)
#pragma unroll
            for (int jq = 0; jq < 4; ++jq) {
                const float4 bq = *(const float4*)(bias + (mp + t) * 32 + 8 * jq + 4 * h);
                acc[t][4 * jq + 0] = bq.x;
                acc[t][4 * jq + 1] = bq.y;
                acc[t][4 * jq + 2] = bq.z;
                acc[t][4 * jq + 3] = bq.w;
            }
#pragma unroll
        for (int s = 0; s < KS; ++s)
#pragma unroll
            for (int t = 0; t < MT_GROUP; ++t) {
                const bf16x8 a = *(const bf16x8*)(w + (((mp + t) * KS + s) * 64 + lane) * 8);
                acc[t] = mfma32(a, bin[s], acc[t]);
            }
#pragma unroll
        for (int t = 0; t < MT_GROUP; ++t)
#pragma unroll
            for (int j = 0; j < 16; ++j)
                bout[2 * (mp + t) + (j >> 3)][j & 7] = (__bf16)fmaxf(acc[t][j], 0.0f);
    }
}

// copy n16 16-byte chunks of the image into LDS (all threads of the workgroup)
__device__ __forceinline__ void stage(const __bf16* __restrict__ src, __bf16* __restrict__ dst, int n16) {
    __syncthreads();
    for (int t = threadIdx.x; t < n16; t += INF_BLOCK) ((bf16x8*)dst)[t] = ((const bf16x8*)src)[t];
    __syncthreads();
}

__global__ __launch_bounds__(INF_BLOCK) void lite_infer_kernel(fp_config g, int32_t ncell,
                                                               const double* __restrict__ mom,
                                                               const double* __restrict__ nvol,
                                                               const __bf16* __restrict__ gimg,
                                                               const float* __restrict__ gsec,
                                                               int mode, float* __restrict__ yout) {
    __shared__ __attribute__((aligned(16))) __bf16 wl[LDS_BF];
    __shared__ __attribute__((aligned(16))) float sec[SEC_N];
    for (int t = threadIdx.x; t < SEC_N; t += INF_BLOCK) sec[t] = gsec[t];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, h = lane >> 5, n = lane & 31;
    const int32_t cell = (blockIdx.x * (INF_BLOCK / 64) + wave) * 32 + n;
    const bool valid = cell < ncell;
    float f[NF];
#pragma unroll
    for (int q = 0; q < NF; ++q) f[q] = 0.0f;
    double tau = 1.0, th = 0.0;
    bool feat = false;
    if (valid) {
        const double* mr = mom + (int64_t)cell * MOM;
        th = mr[M_TH];
        feat = mr[M_N] > 1.0 && th > 0.0;
        if (feat) cell_inputs(g, mr, nvol ? nvol[cell] : g.fnum_over_vol, f, tau);
    }
    stage(gimg + IMG_L1, wl, (IMG_L2 - IMG_L1) / 8);   // also makes sec visible
    bf16x8 b0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int K = 8 * h + i;
        b0[i] = (__bf16)((f[K] - sec[SEC_XM + K]) / sec[SEC_XS + K]);
    }
    bf16x8 act0[KS], act1[KS];
    // layer 1: K = 16, one k-step per output tile
#pragma unroll
    for (int mt = 0; mt < NT; ++mt) {
        f32x16 acc;
#pragma unroll
        for (int jq = 0; jq < 4; ++jq) {
            const float4 bq = *(const float4*)(sec + SEC_B1 + mt * 32 + 8 * jq + 4 * h);
            acc[4 * jq + 0] = bq.x;
            acc[4 * jq + 1] = bq.y;
            acc[4 * jq + 2] = bq.z;
            acc[4 * jq + 3] = bq.w;
        }
        const bf16x8 a = *(const bf16x8*)(wl + (mt * 64 + lane) * 8);
        acc = mfma32(a, b0, acc);
#pragma unroll
        for (int j = 0; j < 16; ++j) act0[2 * mt + (j >> 3)][j & 7] = (__bf16)fmaxf(acc[j], 0.0f);
    }
    stage(gimg + IMG_L2, wl, LDS_BF / 8);
    hidden_layer<2>(wl, sec + SEC_B2, act0, act1, lane);
    stage(gimg + IMG_L3, wl, LDS_BF / 8);
    hidden_layer<2>(wl, sec + SEC_B3, act1, act0, lane);
    stage(gimg + IMG_L4, wl, LDS_BF / 8);
    hidden_layer<2>(wl, sec + SEC_B4, act0, act1, lane);
    stage(gimg + IMG_L5, wl, (IMG_BF - IMG_L5) / 8);
    f32x16 acc = f32x16{};
#pragma unroll
    for (int s = 0; s < KS; ++s) {
        const bf16x8 a = *(const bf16x8*)(wl + (s * 64 + lane) * 8);
        acc = mfma32(a, act1[s], acc);
    }
    // rows 0..3 and 8 live in half 0 (j = 0..3, 4), rows 4..7 in half 1 (j = 0..3)
    float o[9];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float mine = acc[j];
        o[j] = mine;
        o[4 + j] = __shfl_xor(mine, 32, 64);
    }
    o[8] = acc[4];
    if (valid && h == 0) {
        float* dst = yout + (int64_t)cell * NO;
        if (mode == 0) {
#pragma unroll
            for (int q = 0; q < 9; ++q) dst[q] = o[q] + sec[SEC_B5 + q];
        } else {
            const double d6[6] = {1, 0, 0, 1, 0, 1};
            const double sth = feat ? sqrt(th) : 0.0;
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                const double d = (double)(o[q] + sec[SEC_B5 + q]) * (double)sec[SEC_YS + q] +
                                 (double)sec[SEC_YM + q];
                double v = q < 6 ? tau * d - 5.0 * g.eps_hat * d6[q] : tau * sth * d;
                dst[q] = feat ? (float)v : 0.0f;
            }
        }
#pragma unroll
        for (int q = 9; q < NO; ++q) dst[q] = 0.0f;
    }
}

// ---------------------------------------------------------------------------------------
// training (batch along the MFMA columns, activations sample-major in HBM)

__global__ void lite_input_kernel(int64_t B, const float* __restrict__ feats, const float* __restrict__ p,
                                  __bf16* __restrict__ H0) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= B * NF) return;
    const int k = (int)(t % NF);
    H0[t] = (__bf16)((feats[t] - p[OFF_XM + k]) / p[OFF_XS + k]);
}

// Z[n][m] = sum_k W[m][k] H[n][k] + b[m]; H_out = bf16(relu(Z)) (hidden) or Y = Z (output)
template <int K, int M, bool ACT>
__global__ __launch_bounds__(64) void lite_fwd_kernel(int64_t B, const float* __restrict__ W,
                                                      const float* __restrict__ bias,
                                                      const __bf16* __restrict__ Hin,
                                                      float* __restrict__ Z, __bf16* __restrict__ Hout) {
    constexpr int MT = M >= 32 ? M / 32 : 1, KSN = K / 16;
    const int lane = threadIdx.x, h = lane >> 5, c = lane & 31;
    const int64_t n = (int64_t)blockIdx.x * 32 + c;
    const bool valid = n < B;
    bf16x8 bfr[KSN];
#pragma unroll
    for (int s = 0; s < KSN; ++s) {
        if (valid) bfr[s] = *(const bf16x8*)(Hin + n * K + 16 * s + 8 * h);
        else bfr[s] = bf16x8{};
    }
    for (int mt = 0; mt < MT; ++mt) {
        const int m = mt * 32 + c;
        f32x16 acc = f32x16{};
#pragma unroll
        for (int s = 0; s < KSN; ++s) {
            bf16x8 a;
#pragma unroll
            for (int i = 0; i < 8; ++i) a[i] = (__bf16)(m < M ? W[m * K + 16 * s + 8 * h + i] : 0.0f);
            acc = mfma32(a, bfr[s], acc);
        }
        if (valid) {
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int mm = mt * 32 + 8 * (j >> 2) + 4 * h + (j & 3);
                if (mm < M) {
                    const float z = acc[j] + bias[mm];
                    Z[n * M + mm] = z;
                    if (ACT) Hout[n * M + mm] = (__bf16)fmaxf(z, 0.0f);
                }
            }
        }
    }
}

// MSE of standardised targets: mean over samples of sum_o<9 (y_o - t_o)^2, dL/dY
constexpr int LOSS_BLOCK = 256;
__global__ __launch_bounds__(LOSS_BLOCK) void lite_loss_kernel(int64_t B, const float* __restrict__ p,
                                                                const float* __restrict__ Y,
                                                                const float* __restrict__ T,
                                                                float* __restrict__ dY,
                                                                double* __restrict__ lpart) {
    __shared__ double sh[LOSS_BLOCK];
    const int64_t n = (int64_t)blockIdx.x * LOSS_BLOCK + threadIdx.x;
    double l = 0.0;
    if (n < B) {
        const double invB = 1.0 / (double)B;
#pragma unroll
        for (int o = 0; o < NO; ++o) {
            float d = 0.0f;
            if (o < 9) {
                const double t = ((double)T[n * NO + o] - p[OFF_YM + o]) / p[OFF_YS + o];
                const double e = (double)Y[n * NO + o] - t;
                l += e * e;
                d = (float)(2.0 * e * invB);
            }
            dY[n * NO + o] = d;
        }
    }
    sh[threadIdx.x] = l;
    __syncthreads();
    for (int s = LOSS_BLOCK / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) lpart[blockIdx.x] = sh[0];
}

__global__ void lite_loss_final_kernel(int nb, int64_t B, const double* __restrict__ lpart,
                                       float* __restrict__ loss) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < nb; ++i) s += lpart[i];
        *loss = (float)(s / (double)B);
    }
}

// dH[n][k] = sum_m bf16(dZ[n][m]) bf16(W[m][k]);  dZprev[n][k] = dH * relu'(Zprev[n][k])
template <int M, int K>
__global__ __launch_bounds__(64) void lite_bwd_kernel(int64_t B, const float* __restrict__ W,
                                                      const float* __restrict__ dZ,
                                                      const float* __restrict__ Zprev,
                                                      float* __restrict__ dZprev) {
    constexpr int KT = K / 32, MS = M / 16;
    const int lane = threadIdx.x, h = lane >> 5, c = lane & 31;
    const int64_t n = (int64_t)blockIdx.x * 32 + c;
    const bool valid = n < B;
    bf16x8 bfr[MS];
#pragma unroll
    for (int s = 0; s < MS; ++s)
#pragma unroll
        for (int i = 0; i < 8; ++i) bfr[s][i] = (__bf16)(valid ? dZ[n * M + 16 * s + 8 * h + i] : 0.0f);
    for (int kt = 0; kt < KT; ++kt) {
        const int k = kt * 32 + c;
        f32x16 acc = f32x16{};
#pragma unroll
        for (int s = 0; s < MS; ++s) {
            bf16x8 a;
#pragma unroll
            for (int i = 0; i < 8; ++i) a[i] = (__bf16)W[(16 * s + 8 * h + i) * K + k];
            acc = mfma32(a, bfr[s], acc);
        }
        if (valid) {
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int kk = kt * 32 + 8 * (j >> 2) + 4 * h + (j & 3);
                dZprev[n * K + kk] = Zprev[n * K + kk] > 0.0f ? acc[j] : 0.0f;
            }
        }
    }
}

// partial weight gradient of one chunk: part[chunk][woff + m K + k] = sum_n bf16(dZ[n][m]) H[n][k]
template <int M, int K>
__global__ __launch_bounds__(64) void lite_wgrad_kernel(int64_t B, const float* __restrict__ dZ,
                                                        const __bf16* __restrict__ H,
                                                        float* __restrict__ part, int64_t pstride,
                                                        int64_t woff) {
    constexpr int KT = (K + 31) / 32;
    const int lane = threadIdx.x, h = lane >> 5, c = lane & 31;
    const int chunk = blockIdx.y;
    const int mt = blockIdx.x / KT, kt = blockIdx.x % KT;
    const int m = mt * 32 + c, k = kt * 32 + c;
    const int64_t n0 = (int64_t)chunk * TRAIN_CHUNK;
    f32x16 acc = f32x16{};
    for (int s = 0; s < TRAIN_CHUNK / 16; ++s) {
        bf16x8 a, b;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int64_t n = n0 + 16 * s + 8 * h + i;
            const bool v = n < B;
            a[i] = (__bf16)((v && m < M) ? dZ[n * M + m] : 0.0f);
            b[i] = (v && k < K) ? H[n * K + k] : (__bf16)0.0f;
        }
        acc = mfma32(a, b, acc);
    }
    if (k >= K) return;
    float* dst = part + (int64_t)chunk * pstride + woff;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int mm = mt * 32 + 8 * (j >> 2) + 4 * h + (j & 3);
        if (mm < M) dst[mm * K + k] = acc[j];
    }
}

// partial bias gradient of one chunk: sum_n dZ[n][m] (sequential, FP32)
__global__ void lite_bgrad_kernel(int64_t B, int M, const float* __restrict__ dZ,
                                  float* __restrict__ part, int64_t pstride, int64_t boff) {
    const int m = threadIdx.x;
    const int chunk = blockIdx.x;
    if (m >= M) return;
    const int64_t n0 = (int64_t)chunk * TRAIN_CHUNK;
    const int64_t n1 = n0 + TRAIN_CHUNK < B ? n0 + TRAIN_CHUNK : B;
    float s = 0.0f;
    for (int64_t n = n0; n < n1; ++n) s += dZ[n * M + m];
    part[(int64_t)chunk * pstride + boff + m] = s;
}

// grad[q] = sum over chunks in order of part[chunk][q]
__global__ void lite_reduce_kernel(int nchunk, const float* __restrict__ part, int64_t pstride,
                                   float* __restrict__ grad) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N_TRAIN) return;
    float s = 0.0f;
    for (int c = 0; c < nchunk; ++c) s += part[(int64_t)c * pstride + q];
    grad[q] = s;
}

__global__ void lite_adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                                 float* __restrict__ v, float lr, float b1, float b2, float eps, float c1,
                                 float c2) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N_TRAIN) return;
    const float gq = g[q];
    const float mq = b1 * m[q] + (1.0f - b1) * gq;
    const float vq = b2 * v[q] + (1.0f - b2) * gq * gq;
    m[q] = mq;
    v[q] = vq;
    p[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
}

// raw inputs of a batch of moment records (nvol per record, or the configuration's)
__global__ void lite_features_kernel(fp_config g, int64_t n, const double* __restrict__ mom,
                                     const double* __restrict__ nvol, float* __restrict__ feats) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    double m[M_R];
#pragma unroll
    for (int i = 0; i < M_R; ++i) m[i] = mom[c * MOM + i];
    float f[NF];
    double tau;
    cell_inputs(g, m, nvol ? nvol[c] : g.fnum_over_vol, f, tau);
#pragma unroll
    for (int q = 0; q < NF; ++q) feats[c * NF + q] = f[q];
}

// targets (Ct (6), Gamma (3), zeros) of a batch of update records
__global__ void lite_targets_kernel(int64_t n, const double* __restrict__ rec, float* __restrict__ tg) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
#pragma unroll
    for (int q = 0; q < NO; ++q) tg[c * NO + q] = q < 9 ? (float)rec[c * REC + q] : 0.0f;
}

}  // namespace lite

int launch_closure_nn(fp_ctx* c, const float* ynn, const float* ysec, double tol_abs, double tol_rel,
                      double relax, const double* mom, double* rec, int32_t* status, hipStream_t s);

}  // namespace fpg

// =========================================================================================
using namespace fpg;
using namespace fpg::lite;

struct fp_lite {
    fp_ctx* ctx = nullptr;
    int64_t max_batch = 0;
    __bf16* img = nullptr;
    float* sec = nullptr;
    float* ybuf = nullptr;   // [ncell][16] normalised coefficients of the last closure
    __bf16 *H0 = nullptr, *H[4] = {};
    float *Z[4] = {}, *Y = nullptr, *dY = nullptr, *dZa = nullptr, *dZb = nullptr;
    float *part = nullptr, *grad = nullptr;
    double* lpart = nullptr;
};

template <typename T>
static bool lalloc(T** p, size_t count) {
    return hipMalloc((void**)p, sizeof(T) * (count ? count : 1)) == hipSuccess;
}

extern "C" void fp_lite_destroy(fp_lite* n) {
    if (!n) return;
    (void)hipDeviceSynchronize();
    for (void* q : {(void*)n->img, (void*)n->sec, (void*)n->ybuf, (void*)n->H0, (void*)n->H[0], (void*)n->H[1],
                    (void*)n->H[2], (void*)n->H[3], (void*)n->Z[0], (void*)n->Z[1], (void*)n->Z[2],
                    (void*)n->Z[3], (void*)n->Y, (void*)n->dY, (void*)n->dZa, (void*)n->dZb, (void*)n->part,
                    (void*)n->grad, (void*)n->lpart})
        (void)hipFree(q);
    delete n;
}

extern "C" int fp_lite_create(fp_ctx* c, int64_t max_batch, fp_lite** out) {
    if (!c || !out || max_batch < 0 || max_batch > ((int64_t)1 << 24)) return FP_EINVAL;
    *out = nullptr;
    fp_lite* n = new (std::nothrow) fp_lite();
    if (!n) return FP_ENOMEM;
    n->ctx = c;
    n->max_batch = max_batch;
    const size_t B = (size_t)max_batch;
    const size_t nchunk = (B + TRAIN_CHUNK - 1) / TRAIN_CHUNK;
    bool ok = lalloc(&n->img, IMG_BF) && lalloc(&n->sec, SEC_N) && lalloc(&n->ybuf, (size_t)c->ncell * NO);
    if (ok && B > 0) {
        ok = lalloc(&n->H0, B * NF) && lalloc(&n->Y, B * NO) && lalloc(&n->dY, B * NO) &&
             lalloc(&n->dZa, B * NH) && lalloc(&n->dZb, B * NH) && lalloc(&n->part, nchunk * N_TRAIN) &&
             lalloc(&n->grad, N_PARAMS) && lalloc(&n->lpart, B / LOSS_BLOCK + 1);
        for (int l = 0; l < 4 && ok; ++l) ok = lalloc(&n->H[l], B * NH) && lalloc(&n->Z[l], B * NH);
    }
    if (!ok) {
        fp_lite_destroy(n);
        return FP_ENOMEM;
    }
    *out = n;
    return FP_OK;
}

extern "C" int fp_lite_load(fp_ctx* c, fp_lite* n, const float* params, hipStream_t s) {
    if (!c || !n || !params || n->ctx != c) return set_err(c, FP_EINVAL, "fp_lite_load: bad argument");
    hipLaunchKernelGGL(lite_pack_kernel, dim3((IMG_BF + 255) / 256), dim3(256), 0, s, params, n->img, n->sec);
    return check_launch(c, "fp_lite_load");
}

static void infer(fp_ctx* c, const fp_lite* n, const double* mom, int mode, float* y, hipStream_t s) {
    const int32_t cells_per_block = INF_BLOCK / 64 * 32;
    const int grid = (c->ncell + cells_per_block - 1) / cells_per_block;
    hipLaunchKernelGGL(lite_infer_kernel, dim3(grid), dim3(INF_BLOCK), 0, s, c->cfg, c->ncell, mom,
                       (const double*)c->nvol, (const __bf16*)n->img, (const float*)n->sec, mode, y);
}

extern "C" int fp_lite_infer(fp_ctx* c, const fp_lite* n, const double* mom, float* y, hipStream_t s) {
    if (!c || !n || !mom || !y || n->ctx != c) return set_err(c, FP_EINVAL, "fp_lite_infer: bad argument");
    if (c->ncell == 0) return FP_OK;
    infer(c, n, mom, 0, y, s);
    return check_launch(c, "fp_lite_infer");
}

extern "C" int fp_closure_lite(fp_ctx* c, const fp_lite* n, const double* mom, double* rec,
                               int32_t* status, double tol_abs, double tol_rel, double relax,
                               hipStream_t s) {
    if (!c || !n || !mom || !rec || !status || n->ctx != c || !(tol_abs >= 0) || !(tol_rel >= 0) ||
        !(relax > 0.0 && relax <= 1.0))
        return set_err(c, FP_EINVAL, "fp_closure_lite: bad argument");
    if (c->cfg.moment_order == 3 && tol_abs != INFINITY)
        return set_err(c, FP_EINVAL, "fp_closure_lite: the check needs moments through fifth order");
    if (c->ncell == 0) return FP_OK;
    infer(c, n, mom, 1, n->ybuf, s);
    const int rc = check_launch(c, "fp_closure_lite (network)");
    if (rc) return rc;
    return launch_closure_nn(c, n->ybuf, n->sec + SEC_ID, tol_abs, tol_rel, relax, mom, rec, status, s);
}

extern "C" int fp_lite_features(fp_ctx* c, const double* mom, const double* nvol, int64_t n, float* feats,
                                hipStream_t s) {
    if (!c || !mom || !feats || n < 0) return set_err(c, FP_EINVAL, "fp_lite_features: bad argument");
    if (n == 0) return FP_OK;
    hipLaunchKernelGGL(lite_features_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, c->cfg, n,
                       mom, nvol, feats);
    return check_launch(c, "fp_lite_features");
}

extern "C" int fp_lite_targets(fp_ctx* c, const double* rec, int64_t n, float* targets, hipStream_t s) {
    if (!c || !rec || !targets || n < 0) return set_err(c, FP_EINVAL, "fp_lite_targets: bad argument");
    if (n == 0) return FP_OK;
    hipLaunchKernelGGL(lite_targets_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, rec,
                       targets);
    return check_launch(c, "fp_lite_targets");
}

extern "C" int fp_lite_grad(fp_ctx* c, fp_lite* n, const float* params, const float* feats,
                            const float* targets, int64_t B, float* grad, float* loss, hipStream_t s) {
    if (!c || !n || !params || !feats || !targets || !grad || !loss || B <= 0 || B > n->max_batch ||
        n->ctx != c)
        return set_err(c, FP_EINVAL, "fp_lite_grad: bad argument");
    const unsigned g32 = (unsigned)((B + 31) / 32);
    const int nchunk = (int)((B + TRAIN_CHUNK - 1) / TRAIN_CHUNK);
    const int64_t ps = N_TRAIN;
    hipLaunchKernelGGL(lite_input_kernel, dim3((unsigned)((B * NF + 255) / 256)), dim3(256), 0, s, B, feats,
                       params, n->H0);
    hipLaunchKernelGGL((lite_fwd_kernel<NF, NH, true>), dim3(g32), dim3(64), 0, s, B, params + OFF_W1,
                       params + OFF_B1, n->H0, n->Z[0], n->H[0]);
    hipLaunchKernelGGL((lite_fwd_kernel<NH, NH, true>), dim3(g32), dim3(64), 0, s, B, params + OFF_W2,
                       params + OFF_B2, n->H[0], n->Z[1], n->H[1]);
    hipLaunchKernelGGL((lite_fwd_kernel<NH, NH, true>), dim3(g32), dim3(64), 0, s, B, params + OFF_W3,
                       params + OFF_B3, n->H[1], n->Z[2], n->H[2]);
    hipLaunchKernelGGL((lite_fwd_kernel<NH, NH, true>), dim3(g32), dim3(64), 0, s, B, params + OFF_W4,
                       params + OFF_B4, n->H[2], n->Z[3], n->H[3]);
    hipLaunchKernelGGL((lite_fwd_kernel<NH, NO, false>), dim3(g32), dim3(64), 0, s, B, params + OFF_W5,
                       params + OFF_B5, n->H[3], n->Y, (__bf16*)nullptr);
    const int nb = (int)((B + LOSS_BLOCK - 1) / LOSS_BLOCK);
    hipLaunchKernelGGL(lite_loss_kernel, dim3(nb), dim3(LOSS_BLOCK), 0, s, B, params, n->Y, targets, n->dY,
                       n->lpart);
    hipLaunchKernelGGL(lite_loss_final_kernel, dim3(1), dim3(64), 0, s, nb, B, n->lpart, loss);
    // output layer: dZ5 = dY
    hipLaunchKernelGGL((lite_wgrad_kernel<NO, NH>), dim3(NH / 32, nchunk), dim3(64), 0, s, B, n->dY, n->H[3],
                       n->part, ps, OFF_W5);
    hipLaunchKernelGGL(lite_bgrad_kernel, dim3(nchunk), dim3(256), 0, s, B, NO, n->dY, n->part, ps, OFF_B5);
    hipLaunchKernelGGL((lite_bwd_kernel<NO, NH>), dim3(g32), dim3(64), 0, s, B, params + OFF_W5, n->dY, n->Z[3],
                       n->dZa);
    // hidden layers 4, 3, 2 (weights W4, W3, W2; inputs H[2], H[1], H[0])
    const int64_t woff[3] = {OFF_W4, OFF_W3, OFF_W2}, boff[3] = {OFF_B4, OFF_B3, OFF_B2};
    float* dz[2] = {n->dZa, n->dZb};
    for (int q = 0; q < 3; ++q) {
        const int l = 3 - q;   // index of this layer's input activation H[l - 1] / Z[l - 1]
        hipLaunchKernelGGL((lite_wgrad_kernel<NH, NH>), dim3(NT * NT, nchunk), dim3(64), 0, s, B, dz[q & 1],
                           n->H[l - 1], n->part, ps, woff[q]);
        hipLaunchKernelGGL(lite_bgrad_kernel, dim3(nchunk), dim3(256), 0, s, B, NH, dz[q & 1], n->part, ps,
                           boff[q]);
        hipLaunchKernelGGL((lite_bwd_kernel<NH, NH>), dim3(g32), dim3(64), 0, s, B, params + woff[q], dz[q & 1],
                           n->Z[l - 1], dz[(q + 1) & 1]);
    }
    // layer 1 (input H0)
    hipLaunchKernelGGL((lite_wgrad_kernel<NH, NF>), dim3(NT, nchunk), dim3(64), 0, s, B, dz[1], n->H0, n->part,
                       ps, OFF_W1);
    hipLaunchKernelGGL(lite_bgrad_kernel, dim3(nchunk), dim3(256), 0, s, B, NH, dz[1], n->part, ps, OFF_B1);
    hipLaunchKernelGGL(lite_reduce_kernel, dim3((unsigned)((N_TRAIN + 255) / 256)), dim3(256), 0, s, nchunk,
                       n->part, ps, grad);
    return check_launch(c, "fp_lite_grad");
}

extern "C" int fp_lite_adam(fp_ctx* c, float* params, const float* grad, float* m, float* v, int64_t t,
                            float lr, hipStream_t s) {
    if (!c || !params || !grad || !m || !v || t < 1 || !(lr >= 0.0f))
        return set_err(c, FP_EINVAL, "fp_lite_adam: bad argument");
    const float c1 = (float)(1.0 - pow(0.9, (double)t)), c2 = (float)(1.0 - pow(0.999, (double)t));
    hipLaunchKernelGGL(lite_adam_kernel, dim3((unsigned)((N_TRAIN + 255) / 256)), dim3(256), 0, s, params, grad,
                       m, v, lr, 0.9f, 0.999f, 1e-8f, c1, c2);
    return check_launch(c, "fp_lite_adam");
}

extern "C" int fp_lite_train_step(fp_ctx* c, fp_lite* n, float* params, float* m, float* v, int64_t t,
                                  float lr, const float* feats, const float* targets, int64_t B, float* loss,
                                  hipStream_t s) {
    if (!n) return set_err(c, FP_EINVAL, "fp_lite_train_step: bad argument");
    const int rc = fp_lite_grad(c, n, params, feats, targets, B, n->grad, loss, s);
    if (rc) return rc;
    return fp_lite_adam(c, params, n->grad, m, v, t, lr, s);
}

// ---- column statistics of a training matrix (the standardising scaler of Sec. "Phase 3":
// per-column mean and population standard deviation) ------------------------------------
namespace fpg {
namespace lite {
constexpr int STAT_BLOCK = 256;
// one workgroup per column: FP64 sums in a fixed order (strided per thread, then a tree in
// LDS), two passes (mean, then squared deviations): bitwise reproducible
__global__ __launch_bounds__(STAT_BLOCK) void column_stats_kernel(const float* __restrict__ x, int64_t n,
                                                                 int32_t k, double* __restrict__ mean,
                                                                 double* __restrict__ stdev) {
    __shared__ double sh[STAT_BLOCK];
    const int col = blockIdx.x;
    double s = 0.0;
    for (int64_t r = threadIdx.x; r < n; r += STAT_BLOCK) s += (double)x[r * k + col];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = STAT_BLOCK / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    const double mu = sh[0] / (double)n;
    __syncthreads();
    double q = 0.0;
    for (int64_t r = threadIdx.x; r < n; r += STAT_BLOCK) {
        const double d = (double)x[r * k + col] - mu;
        q += d * d;
    }
    sh[threadIdx.x] = q;
    __syncthreads();
    for (int w = STAT_BLOCK / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        mean[col] = mu;
        stdev[col] = sqrt(sh[0] / (double)n);
    }
}
}  // namespace lite
}  // namespace fpg

extern "C" int fp_column_stats(fp_ctx* c, const float* x, int64_t n, int32_t k, double* mean, double* stdev,
                               hipStream_t s) {
    if (!c || !x || !mean || !stdev || n < 1 || k < 1 || k > 4096)
        return set_err(c, FP_EINVAL, "fp_column_stats: bad argument");
    hipLaunchKernelGGL(fpg::lite::column_stats_kernel, dim3(k), dim3(fpg::lite::STAT_BLOCK), 0, s, x, n, k,
                       mean, stdev);
    return check_launch(c, "fp_column_stats");
}
