// fp_nn.hip -- learned closure: BF16 MFMA inference and training of the surrogate MLP.
//
// Network (the surrogate of Sec. "Phase 1-2"/"Phase 3": standardised inputs and
// outputs, dense layers): 32 -> 128 -> 128 -> 128 -> 16 with SiLU; 27 features of the
// theta-normalised moments and 9 normalised coefficients, zero padded.  All products are
// v_mfma_f32_32x32x16_bf16 (BF16 operands, FP32 accumulation).
//
// Operand layouts of the 32x32x16 MFMA (wave64, lane l, half h = l / 32):
//   A (32 x 16):  lane holds A[l % 32][8h + i], i = 0..7
//   B (16 x 32):  lane holds B[8h + i][l % 32]
//   D (32 x 32):  lane holds D[8(j/4) + 4h + j%4][l % 32], j = 0..15
// Inference computes H_out^T = W H_in^T with the batch (cells) along the MFMA columns,
// so a lane keeps one cell through all layers.  The rows of a layer's output that a
// lane holds are exactly the k-slots it must feed into the next layer's B operand once
// the next weight matrix has its columns permuted by
//   pi(16 s + 8 h + i) = 16 s + 8 floor(i/4) + 4 h + i % 4,
// so activations never leave the registers between layers.  The permuted BF16 weights
// are stored fragment-major ([tile][k-step][lane][8]) and live in LDS.
#include "fp_closure_dev.h"

#include <mutex>
#include <string>

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

namespace fpg {

constexpr int NF = 32, NH = 128, NO = 16;
constexpr int OFF_W1 = 0, OFF_B1 = 4096, OFF_W2 = 4224, OFF_B2 = 20608, OFF_W3 = 20736,
              OFF_B3 = 37120, OFF_W4 = 37248, OFF_B4 = 39296, OFF_XM = 39312, OFF_XS = 39344,
              OFF_YM = 39376, OFF_YS = 39392, N_PARAMS = 39408, N_TRAIN = 39312;
// BF16 fragment image
constexpr int IMG_L1 = 0, IMG_L2 = 4096, IMG_L3 = 20480, IMG_L4 = 36864, IMG_BF = 40960;
// FP32 section after the image: b1 b2 b3 b4 x_mean x_std y_mean y_std
constexpr int SEC_B1 = 0, SEC_B2 = 128, SEC_B3 = 256, SEC_B4 = 384, SEC_XM = 400, SEC_XS = 432,
              SEC_YM = 464, SEC_YS = 480, SEC_N = 496;
constexpr int TRAIN_CHUNK = 1024;

__device__ __forceinline__ int perm_k(int K) {
    const int s = K >> 4, h = (K >> 3) & 1, i = K & 7;
    return 16 * s + 8 * (i >> 2) + 4 * h + (i & 3);
}

__device__ __forceinline__ float silu_f(float z) { return z / (1.0f + __expf(-z)); }
// inference: z * sigmoid(z) with the hardware exp2 and reciprocal (about 1 ulp; the
// result is rounded to bfloat16 right after)
__device__ __forceinline__ float silu_fast(float z) {
    constexpr float LOG2E = 1.4426950408889634f;
    return z * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-LOG2E * z));
}
__device__ __forceinline__ float dsilu_f(float z) {
    const float s = 1.0f / (1.0f + __expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

__device__ __forceinline__ f32x16 mfma32(bf16x8 a, bf16x8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------------------
// pack FP32 parameters into the permuted BF16 fragment image + FP32 section
__global__ void nn_pack_kernel(const float* __restrict__ p, __bf16* __restrict__ img,
                               float* __restrict__ sec) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < IMG_BF) {
        int layer, base, ks_n;
        if (t < IMG_L2) { layer = 1; base = IMG_L1; ks_n = 2; }
        else if (t < IMG_L3) { layer = 2; base = IMG_L2; ks_n = 8; }
        else if (t < IMG_L4) { layer = 3; base = IMG_L3; ks_n = 8; }
        else { layer = 4; base = IMG_L4; ks_n = 8; }
        const int e = t - base;
        const int i = e & 7, lane = (e >> 3) & 63, frag = e >> 9;
        const int ks = frag % ks_n, mt = frag / ks_n;
        const int m = mt * 32 + (lane & 31), h = lane >> 5;
        const int K = ks * 16 + 8 * h + i;
        float v = 0.0f;
        if (layer == 1) v = p[OFF_W1 + m * NF + K];
        else if (layer == 2) v = p[OFF_W2 + m * NH + perm_k(K)];
        else if (layer == 3) v = p[OFF_W3 + m * NH + perm_k(K)];
        else v = m < NO ? p[OFF_W4 + m * NH + perm_k(K)] : 0.0f;
        img[t] = (__bf16)v;
    }
    if (t < SEC_N) {
        float v;
        if (t < SEC_B2) v = p[OFF_B1 + t];
        else if (t < SEC_B3) v = p[OFF_B2 + t - SEC_B2];
        else if (t < SEC_B4) v = p[OFF_B3 + t - SEC_B3];
        else if (t < SEC_XM) v = p[OFF_B4 + t - SEC_B4];
        else if (t < SEC_XS) v = p[OFF_XM + t - SEC_XM];
        else if (t < SEC_YM) v = p[OFF_XS + t - SEC_XS];
        else if (t < SEC_YS) v = p[OFF_YM + t - SEC_YM];
        else v = p[OFF_YS + t - SEC_YS];
        sec[t] = v;
    }
}

// features of one cell (FP64 in, FP32 out), index K in 0..31:
// [P/th - I (6), T/th^1.5 (10), R/th^2 - 5 I (6), W/th^2.5 (3), eps_hat, log10 N, 0...]
__device__ __forceinline__ void cell_features(const double* m, double eps_hat, float f[32]) {
    const double th = m[M_TH];
    const double i1 = 1.0 / th, i15 = i1 / sqrt(th), i2 = i1 * i1, i25 = i2 / sqrt(th);
    const double d6[6] = {1, 0, 0, 1, 0, 1};
#pragma unroll
    for (int q = 0; q < 6; ++q) f[q] = (float)(m[M_P + q] * i1 - d6[q]);
#pragma unroll
    for (int q = 0; q < 10; ++q) f[6 + q] = (float)(m[M_T + q] * i15);
#pragma unroll
    for (int q = 0; q < 6; ++q) f[16 + q] = (float)(m[M_R + q] * i2 - 5.0 * d6[q]);
#pragma unroll
    for (int q = 0; q < 3; ++q) f[22 + q] = (float)(m[M_W + q] * i25);
    f[25] = (float)eps_hat;
    f[26] = (float)log10(m[M_N]);
#pragma unroll
    for (int q = 27; q < 32; ++q) f[q] = 0.0f;
}

// the 16 features lane half h feeds into the first layer: f[q] = feature 8h + q (q < 8)
// and 16 + 8h + (q - 8) (q >= 8); the same arithmetic as cell_features, with only the
// moments that half needs loaded (17 of them for h = 0, 11 for h = 1)
__device__ __forceinline__ void half_features(const double* __restrict__ m, int h, double eps_hat,
                                              float f[16]) {
    const double th = m[M_TH];
    const double i1 = 1.0 / th, i15 = i1 / sqrt(th), i2 = i1 * i1, i25 = i2 / sqrt(th);
    // feature K -> (moment index, scale: 0 = 1/th 1 = th^-1.5 2 = th^-2 3 = th^-2.5,
    // offset), for K < 25
    auto fea = [&](int K, bool hi) -> float {
        if (K < 6) return (float)(m[M_P + K] * i1 - ((K == 0 || K == 3 || K == 5) ? 1.0 : 0.0));
        if (K < 16) return (float)(m[M_T + K - 6] * i15);
        if (K < 22) {
            const int q = K - 16;
            return (float)(m[M_R + q] * i2 - ((q == 0 || q == 3 || q == 5) ? 5.0 : 0.0));
        }
        if (K < 25) return (float)(m[M_W + K - 22] * i25);
        if (K == 25) return (float)eps_hat;
        if (K == 26) return hi ? (float)log10(m[M_N]) : 0.0f;
        return 0.0f;
    };
    if (h == 0) {
#pragma unroll
        for (int q = 0; q < 16; ++q) f[q] = fea(q < 8 ? q : 16 + q - 8, false);
    } else {
#pragma unroll
        for (int q = 0; q < 16; ++q) f[q] = fea(q < 8 ? 8 + q : 24 + q - 8, true);
    }
}

// ---------------------------------------------------------------------------------------
// fused inference: standardised outputs y_std[cell][16] (entries 9..15 zero)
// 16 waves per workgroup share one LDS copy of the weights (82 KB: one workgroup per
// CU), i.e. 4 waves per SIMD, so that one wave's SiLU epilogue (VALU) overlaps another's
// MFMAs; every wave keeps at most 128 registers (VGPRs and AGPRs together)
constexpr int NN_BLOCK = 1024;

// Inverted dropout of the hidden activations for the sensitivity probe: activation row u
// of cell k in pass t is kept if word u % 4 of Philox4x32-10 at counter
// (k, t, PURPOSE_DROPOUT, 32 (layer - 1) + u / 4) is at least keep_min (= floor(p 2^32)),
// and then scaled by 1 / (1 - p); no dropout when drop is null.
// DROP: inverted dropout after the SiLU; bit 16 mt + 4 jq + i of keep set <=> the lane's
// output row 32 mt + 8 jq + 4 h + i is kept (and scaled)
template <int KS, bool DROP = false>
__device__ __forceinline__ void nn_layer(const __bf16* __restrict__ img_l, const float* __restrict__ bias,
                                         const bf16x8 (&bin)[8], bf16x8 (&bout)[8], int lane,
                                         uint64_t keep = 0, float scale = 1.0f) {
    const int h = lane >> 5;
    // two of the four 32-row output tiles at a time (32 accumulator registers live)
#pragma unroll
    for (int mp = 0; mp < 4; mp += 2) {
        // accumulators start from the bias: output row u = 32 mt + 8 (j / 4) + 4 h + j % 4,
        // four consecutive rows per 16-byte LDS read
        f32x16 acc[2];
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int jq = 0; jq < 4; ++jq) {
                const float4 bq = *(const float4*)(bias + (mp + t) * 32 + 8 * jq + 4 * h);
                acc[t][4 * jq + 0] = bq.x;
                acc[t][4 * jq + 1] = bq.y;
                acc[t][4 * jq + 2] = bq.z;
                acc[t][4 * jq + 3] = bq.w;
            }
#pragma unroll
        for (int s = 0; s < KS; ++s) {
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const bf16x8 a = *(const bf16x8*)(img_l + (((mp + t) * KS + s) * 64 + lane) * 8);
                acc[t] = mfma32(a, bin[s], acc[t]);
            }
        }
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            if constexpr (DROP) {
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const float a = silu_fast(acc[t][j]);
                    bout[2 * (mp + t) + (j >> 3)][j & 7] =
                        (__bf16)(((keep >> (16 * (mp + t) + j)) & 1) ? a * scale : 0.0f);
                }
            } else {
#pragma unroll
                for (int j = 0; j < 16; ++j)
                    bout[2 * (mp + t) + (j >> 3)][j & 7] = (__bf16)silu_fast(acc[t][j]);
            }
        }
    }
}

__global__ __launch_bounds__(NN_BLOCK) void nn_infer_kernel(int32_t ncell, const double* __restrict__ mom,
                                                             double eps_hat,
                                                             const __bf16* __restrict__ gimg,
                                                             const float* __restrict__ gsec,
                                                             float* __restrict__ yout) {
    __shared__ __attribute__((aligned(16))) __bf16 img[IMG_BF];
    __shared__ __attribute__((aligned(16))) float sec[SEC_N];
    for (int t = threadIdx.x; t < IMG_BF / 8; t += NN_BLOCK)
        ((bf16x8*)img)[t] = ((const bf16x8*)gimg)[t];
    for (int t = threadIdx.x; t < SEC_N; t += NN_BLOCK) sec[t] = gsec[t];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, h = lane >> 5, n = lane & 31;
    const int32_t ntiles = (ncell + 31) / 32;
    for (int32_t tile = blockIdx.x * (NN_BLOCK / 64) + wave; tile < ntiles;
         tile += gridDim.x * (NN_BLOCK / 64)) {
        // the weight fragments are read from LDS inside every tile: keep the compiler from
        // hoisting them out of the loop (80 fragments would not fit in the registers)
        __asm__ volatile("" ::: "memory");
        const int32_t cell = tile * 32 + n;
        const bool valid = cell < ncell;
        float f[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) f[q] = 0.0f;
        if (valid) {
            const double* mr = mom + (int64_t)cell * MOM;
            if (mr[M_N] > 1.0 && mr[M_TH] > 0.0) half_features(mr, h, eps_hat, f);
        }
        bf16x8 b0[8], b1[8];
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int K = 16 * s + 8 * h + i;
                b0[s][i] = (__bf16)((f[8 * s + i] - sec[SEC_XM + K]) / sec[SEC_XS + K]);
            }
        nn_layer<2>(img + IMG_L1, sec + SEC_B1, b0, b1, lane);
        nn_layer<8>(img + IMG_L2, sec + SEC_B2, b1, b0, lane);
        nn_layer<8>(img + IMG_L3, sec + SEC_B3, b0, b1, lane);
        f32x16 acc = f32x16{};
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const bf16x8 a = *(const bf16x8*)(img + IMG_L4 + (s * 64 + lane) * 8);
            acc = mfma32(a, b1[s], acc);
        }
        // rows 0..3 and 8 live in half 0 (j = 0..3, 4), rows 4..7 in half 1 (j = 0..3)
        float o[9];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float mine = acc[j];
            const float other = __shfl_xor(mine, 32, 64);
            o[j] = mine;
            o[4 + j] = other;
        }
        o[8] = acc[4];
        if (valid && h == 0) {
            float* dst = yout + (int64_t)cell * NO;
#pragma unroll
            for (int q = 0; q < 9; ++q) dst[q] = o[q] + sec[SEC_B4 + q];
#pragma unroll
            for (int q = 9; q < 16; ++q) dst[q] = 0.0f;
        }
    }
}

// ---------------------------------------------------------------------------------------
// coefficient-sensitivity probe (Sec. "Heuristic coefficient-sensitivity probe"): npass
// forward passes with inverted dropout on the three hidden layers; per cell the standard
// deviation (1/npass) over the passes of each de-standardised normalised coefficient, and
// sens[cell] = (|sigma_C| over the six stress coefficients, |sigma_Gamma| over the three
// heat-flux ones); cells without features (N <= 1 or theta <= 0) get zeros.  Each wave
// keeps its 32 cells' inputs and runs every pass; the sums of the deviations from the
// first pass are FP64 (no cancellation).
constexpr int SENS_BLOCK = 512;

__global__ __launch_bounds__(SENS_BLOCK) void nn_sense_kernel(int32_t ncell, const double* __restrict__ mom,
                                                              double eps_hat, const __bf16* __restrict__ gimg,
                                                              const float* __restrict__ gsec, int32_t npass,
                                                              uint64_t seed, uint32_t keep_min, float scale,
                                                              double* __restrict__ sens) {
    __shared__ __attribute__((aligned(16))) __bf16 img[IMG_BF];
    __shared__ __attribute__((aligned(16))) float sec[SEC_N];
    for (int t = threadIdx.x; t < IMG_BF / 8; t += SENS_BLOCK)
        ((bf16x8*)img)[t] = ((const bf16x8*)gimg)[t];
    for (int t = threadIdx.x; t < SEC_N; t += SENS_BLOCK) sec[t] = gsec[t];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, h = lane >> 5, n = lane & 31;
    const int32_t ntiles = (ncell + 31) / 32;
    for (int32_t tile = blockIdx.x * (SENS_BLOCK / 64) + wave; tile < ntiles;
         tile += gridDim.x * (SENS_BLOCK / 64)) {
        __asm__ volatile("" ::: "memory");
        const int32_t cell = tile * 32 + n;
        const bool valid = cell < ncell;
        float f[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) f[q] = 0.0f;
        bool feat = false;
        if (valid) {
            const double* mr = mom + (int64_t)cell * MOM;
            feat = mr[M_N] > 1.0 && mr[M_TH] > 0.0;
            if (feat) half_features(mr, h, eps_hat, f);
        }
        bf16x8 bin[2];
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int K = 16 * s + 8 * h + i;
                bin[s][i] = (__bf16)((f[8 * s + i] - sec[SEC_XM + K]) / sec[SEC_XS + K]);
            }
        double y0[9], s1[9], s2[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) y0[q] = s1[q] = s2[q] = 0.0;
        for (int32_t t = 0; t < npass; ++t) {
            __asm__ volatile("" ::: "memory");  // keeps the weight reads inside the pass
            bf16x8 b0[8], b1[8];
            b0[0] = bin[0];
            b0[1] = bin[1];
            // masks of the lane's 64 rows of each hidden layer: row 32 mt + 8 jq + 4 h + i
            // of layer l is decided by word i of the draw with sub 32 (l-1) + 8 mt + 2 jq + h
            uint64_t km[3];
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                uint64_t m = 0;
#pragma unroll 1
                for (int g = 0; g < 16; ++g) {
                    const uint4 r = draw(seed, (uint32_t)cell, (uint32_t)t, PURPOSE_DROPOUT,
                                         32u * (uint32_t)l + 2u * (uint32_t)g + (uint32_t)h);
                    const uint64_t b = (uint64_t)(r.x >= keep_min) | ((uint64_t)(r.y >= keep_min) << 1) |
                                       ((uint64_t)(r.z >= keep_min) << 2) |
                                       ((uint64_t)(r.w >= keep_min) << 3);
                    m |= b << (4 * g);
                }
                km[l] = m;
            }
            nn_layer<2, true>(img + IMG_L1, sec + SEC_B1, b0, b1, lane, km[0], scale);
            nn_layer<8, true>(img + IMG_L2, sec + SEC_B2, b1, b0, lane, km[1], scale);
            nn_layer<8, true>(img + IMG_L3, sec + SEC_B3, b0, b1, lane, km[2], scale);
            f32x16 acc = f32x16{};
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const bf16x8 a = *(const bf16x8*)(img + IMG_L4 + (s * 64 + lane) * 8);
                acc = mfma32(a, b1[s], acc);
            }
            float o[9];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float mine = acc[j];
                const float other = __shfl_xor(mine, 32, 64);
                o[j] = mine;
                o[4 + j] = other;
            }
            o[8] = acc[4];
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                const double y = (double)(o[q] + sec[SEC_B4 + q]) * (double)sec[SEC_YS + q] +
                                 (double)sec[SEC_YM + q];
                if (t == 0) y0[q] = y;
                const double dy = y - y0[q];
                s1[q] += dy;
                s2[q] += dy * dy;
            }
        }
        if (valid && h == 0) {
            double vc = 0.0, vg = 0.0;
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                const double m = s1[q] / (double)npass;
                const double var = fmax(s2[q] / (double)npass - m * m, 0.0);
                if (q < 6) vc += var;
                else vg += var;
            }
            sens[(int64_t)cell * 2] = feat ? sqrt(vc) : 0.0;
            sens[(int64_t)cell * 2 + 1] = feat ? sqrt(vg) : 0.0;
        }
    }
}

// ---------------------------------------------------------------------------------------
// training kernels (batch along the MFMA columns, activations sample-major in HBM)

// H0 = bf16((f - x_mean) / x_std)
__global__ void nn_input_kernel(int64_t B, const float* __restrict__ feats, const float* __restrict__ p,
                                __bf16* __restrict__ H0) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= B * NF) return;
    const int k = (int)(t % NF);
    H0[t] = (__bf16)((feats[t] - p[OFF_XM + k]) / p[OFF_XS + k]);
}

// Z[n][m] = sum_k W[m][k] H[n][k] + b[m]; H_out = bf16(silu(Z)) (hidden) or Y = Z (output)
template <int K, int M, bool ACT>
__global__ __launch_bounds__(64) void nn_fwd_kernel(int64_t B, const float* __restrict__ W,
                                                    const float* __restrict__ bias,
                                                    const __bf16* __restrict__ Hin,
                                                    float* __restrict__ Z, __bf16* __restrict__ Hout) {
    constexpr int MT = M >= 32 ? M / 32 : 1, KS = K / 16;
    const int lane = threadIdx.x, h = lane >> 5, c = lane & 31;
    const int64_t n = (int64_t)blockIdx.x * 32 + c;
    const bool valid = n < B;
    bf16x8 bfr[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
        if (valid) bfr[s] = *(const bf16x8*)(Hin + n * K + 16 * s + 8 * h);
        else bfr[s] = bf16x8{};
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        const int m = mt * 32 + c;
        f32x16 acc = f32x16{};
#pragma unroll
        for (int s = 0; s < KS; ++s) {
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
                    if (ACT) Hout[n * M + mm] = (__bf16)silu_f(z);
                }
            }
        }
    }
}

// loss and dL/dY.  kind 0: mean over samples of sum_o (y_o - t_o)^2 on standardised
// targets.  kind 1: mean of |A y - b|^2 of the normalised closure system with y the
// de-standardised output (sys[n] = A row-major (81) then b (9), FP64).
constexpr int LOSS_BLOCK = 256;
__global__ __launch_bounds__(LOSS_BLOCK) void nn_loss_kernel(int64_t B, int kind, const float* __restrict__ p,
                                                              const float* __restrict__ Y,
                                                              const float* __restrict__ T,
                                                              const float* __restrict__ feats,
                                                              const double* __restrict__ sys,
                                                              float* __restrict__ dY,
                                                              double* __restrict__ lpart) {
    __shared__ double sh[LOSS_BLOCK];
    const int64_t n = (int64_t)blockIdx.x * LOSS_BLOCK + threadIdx.x;
    double l = 0.0;
    if (n < B) {
        const double invB = 1.0 / (double)B;
        float d[NO];
#pragma unroll
        for (int o = 0; o < NO; ++o) d[o] = 0.0f;
        if (kind == 0) {
#pragma unroll
            for (int o = 0; o < 9; ++o) {
                const double t = ((double)T[n * NO + o] - p[OFF_YM + o]) / p[OFF_YS + o];
                const double e = (double)Y[n * NO + o] - t;
                l += e * e;
                d[o] = (float)(2.0 * e * invB);
            }
        } else {
            const double eh = feats[n * NF + 25];
            double y[9];
#pragma unroll
            for (int o = 0; o < 9; ++o) y[o] = (double)Y[n * NO + o] * p[OFF_YS + o] + p[OFF_YM + o];
            y[0] += 5.0 * eh; y[3] += 5.0 * eh; y[5] += 5.0 * eh;
            const double* S = sys + n * 90;
            double r[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                double t = -S[81 + i];
#pragma unroll
                for (int k = 0; k < 9; ++k) t = fma(S[i * 9 + k], y[k], t);
                r[i] = t;
                l += t * t;
            }
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                double g = 0.0;
#pragma unroll
                for (int i = 0; i < 9; ++i) g = fma(S[i * 9 + k], r[i], g);
                d[k] = (float)(2.0 * g * invB * p[OFF_YS + k]);
            }
        }
#pragma unroll
        for (int o = 0; o < NO; ++o) dY[n * NO + o] = d[o];
    }
    sh[threadIdx.x] = l;
    __syncthreads();
    for (int s = LOSS_BLOCK / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) lpart[blockIdx.x] = sh[0];
}

__global__ void nn_loss_final_kernel(int nb, int64_t B, const double* __restrict__ lpart,
                                     float* __restrict__ loss) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < nb; ++i) s += lpart[i];
        *loss = (float)(s / (double)B);
    }
}

// dH[n][k] = sum_m dZ[n][m] W[m][k];  out[n][k] = dH * silu'(Zprev[n][k])
template <int M, int K>
__global__ __launch_bounds__(64) void nn_bwd_kernel(int64_t B, const float* __restrict__ W,
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
#pragma unroll
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
                dZprev[n * K + kk] = acc[j] * dsilu_f(Zprev[n * K + kk]);
            }
        }
    }
}

// partial weight gradient of one chunk of samples: dWp[chunk][m][k] = sum_n dZ[n][m] H[n][k]
template <int M, int K>
__global__ __launch_bounds__(64) void nn_wgrad_kernel(int64_t B, const float* __restrict__ dZ,
                                                      const __bf16* __restrict__ H,
                                                      float* __restrict__ part, int64_t pstride,
                                                      int woff) {
    constexpr int MT = M >= 32 ? M / 32 : 1, KT = K / 32;
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
            b[i] = v ? H[n * K + k] : (__bf16)0.0f;
        }
        acc = mfma32(a, b, acc);
    }
    float* dst = part + (int64_t)chunk * pstride + woff;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int mm = mt * 32 + 8 * (j >> 2) + 4 * h + (j & 3);
        if (mm < M) dst[mm * K + k] = acc[j];
    }
}

// partial bias gradient of one chunk: dbp[chunk][m] = sum_n dZ[n][m] (sequential, FP32)
__global__ void nn_bgrad_kernel(int64_t B, int M, const float* __restrict__ dZ,
                                float* __restrict__ part, int64_t pstride, int boff) {
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
__global__ void nn_reduce_kernel(int nchunk, const float* __restrict__ part, int64_t pstride,
                                 float* __restrict__ grad) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N_TRAIN) return;
    float s = 0.0f;
    for (int c = 0; c < nchunk; ++c) s += part[(int64_t)c * pstride + q];
    grad[q] = s;
}

// Adam (Kingma and Ba) on the trainable prefix, FP32 master weights
__global__ void nn_adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                               float* __restrict__ v, float lr, float b1, float b2, float eps,
                               float c1, float c2) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N_TRAIN) return;
    const float gq = g[q];
    const float mq = b1 * m[q] + (1.0f - b1) * gq;
    const float vq = b2 * v[q] + (1.0f - b2) * gq * gq;
    m[q] = mq;
    v[q] = vq;
    p[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
}

// features of a batch of moment records (raw, unstandardised) for training
__global__ void nn_features_kernel(int64_t n, const double* __restrict__ mom, double eps_hat,
                                   float* __restrict__ feats) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    double m[31];
#pragma unroll
    for (int i = 0; i < 31; ++i) m[i] = mom[c * MOM + i];
    float f[32];
    cell_features(m, eps_hat, f);
#pragma unroll
    for (int q = 0; q < 32; ++q) feats[c * NF + q] = f[q];
}

// normalised targets of a batch of update records
__global__ void nn_targets_kernel(int64_t n, const double* __restrict__ rec, double eps_hat,
                                  float* __restrict__ tg) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const double* r = rec + c * REC;
    const double tau = r[R_TAU], sth = sqrt(r[R_TH]);
    const double d6[6] = {1, 0, 0, 1, 0, 1};
#pragma unroll
    for (int q = 0; q < 6; ++q) tg[c * NO + q] = (float)(r[R_C + q] * tau - 5.0 * eps_hat * d6[q]);
#pragma unroll
    for (int q = 0; q < 3; ++q) tg[c * NO + 6 + q] = (float)(r[R_G + q] * tau * sth);
#pragma unroll
    for (int q = 9; q < NO; ++q) tg[c * NO + q] = 0.0f;
}

// normalised closure system (A row-major, then b) of a batch of moment records
__global__ void nn_system_kernel(int64_t n, const double* __restrict__ mom, double eps_hat,
                                 double* __restrict__ sys) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    double m[31];
#pragma unroll
    for (int i = 0; i < 31; ++i) m[i] = mom[c * MOM + i];
    CellSystem s;
    build_system(m, eps_hat, s);
    double* d = sys + c * 90;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
#pragma unroll
        for (int k = 0; k < 9; ++k) d[i * 9 + k] = s.a[i][k];
        d[81 + i] = s.a[i][9];
    }
}

}  // namespace fpg

// =========================================================================================
using namespace fpg;

struct fp_nn {
    fp_ctx* ctx = nullptr;
    int64_t max_batch = 0;
    __bf16* img = nullptr;
    float* sec = nullptr;
    float* ybuf = nullptr;   // [ncell][16] standardised outputs of the last inference
    // training scratch
    __bf16 *H0 = nullptr, *H1 = nullptr, *H2 = nullptr, *H3 = nullptr;
    float *Z1 = nullptr, *Z2 = nullptr, *Z3 = nullptr, *Y = nullptr, *dY = nullptr;
    float *dZa = nullptr, *dZb = nullptr, *part = nullptr, *grad = nullptr;
    double* lpart = nullptr;
    int nchunk = 0;
};

template <typename T>
static bool nalloc(T** p, size_t count) {
    return hipMalloc((void**)p, sizeof(T) * (count ? count : 1)) == hipSuccess;
}

// ---- scratch of fp_closure_nn_noalloc --------------------------------------------------
// The standardised network outputs pass from the network kernel to the check kernel through
// this file-scope array instead of the handle's buffer: every GPU the library runs on holds
// one copy of FP_NN_NOALLOC_CELLS x 16 floats (16 MiB) until the process ends.  In host code
// the name `scratch` is a host-side stand-in, not a device address: fp_nn_create looks up
// the address of the current device's copy once per device (hipGetSymbolAddress) and keeps
// it in scratch_dev[device]; host code uses only that pointer.
static __device__ __align__(256) float scratch[(size_t)FP_NN_NOALLOC_CELLS * NO];
constexpr int SCRATCH_DEVICES = 64;
static std::mutex scratch_mu;
static float* scratch_dev[SCRATCH_DEVICES] = {};

// With the context's device current: look up that device's copy of the array once.
static int scratch_setup(fp_ctx* c) {
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (c->device < 0 || c->device >= SCRATCH_DEVICES) return FP_EINVAL;
    if (scratch_dev[c->device]) return FP_OK;
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return FP_EDEVICE;
    scratch_dev[c->device] = (float*)ptr;
    return FP_OK;
}

static float* scratch_of(const fp_ctx* c) {
    std::lock_guard<std::mutex> lock(scratch_mu);
    return (c->device >= 0 && c->device < SCRATCH_DEVICES) ? scratch_dev[c->device] : nullptr;
}

extern "C" int fp_nn_create(fp_ctx* c, int64_t max_batch, fp_nn** out) {
    if (!c || !out || max_batch < 0 || max_batch > ((int64_t)1 << 26)) return FP_EINVAL;
    *out = nullptr;
    {
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess) return set_err(c, FP_EDEVICE, "fp_nn_create: hipGetDevice failed");
        if (cur != c->device && hipSetDevice(c->device) != hipSuccess)
            return set_err(c, FP_EDEVICE, "fp_nn_create: hipSetDevice failed");
        const int rc = scratch_setup(c);
        if (cur != c->device) (void)hipSetDevice(cur);
        if (rc) return set_err(c, rc, "fp_nn_create: no address for the no-allocation scratch");
    }
    fp_nn* n = new (std::nothrow) fp_nn();
    if (!n) return FP_ENOMEM;
    n->ctx = c;
    n->max_batch = max_batch;
    const size_t B = (size_t)max_batch;
    n->nchunk = (int)((max_batch + TRAIN_CHUNK - 1) / TRAIN_CHUNK);
    bool ok = nalloc(&n->img, IMG_BF) && nalloc(&n->sec, SEC_N) && nalloc(&n->ybuf, (size_t)c->ncell * NO);
    if (ok && B > 0)
        ok = nalloc(&n->H0, B * NF) && nalloc(&n->H1, B * NH) && nalloc(&n->H2, B * NH) &&
             nalloc(&n->H3, B * NH) && nalloc(&n->Z1, B * NH) && nalloc(&n->Z2, B * NH) &&
             nalloc(&n->Z3, B * NH) && nalloc(&n->Y, B * NO) && nalloc(&n->dY, B * NO) &&
             nalloc(&n->dZa, B * NH) && nalloc(&n->dZb, B * NH) &&
             nalloc(&n->part, (size_t)n->nchunk * N_TRAIN) && nalloc(&n->grad, N_PARAMS) &&
             nalloc(&n->lpart, B / LOSS_BLOCK + 1);
    if (!ok) {
        fp_nn_destroy(n);
        return FP_ENOMEM;
    }
    *out = n;
    return FP_OK;
}

extern "C" void fp_nn_destroy(fp_nn* n) {
    if (!n) return;
    (void)hipDeviceSynchronize();
    for (void* p : {(void*)n->img, (void*)n->sec, (void*)n->ybuf, (void*)n->H0, (void*)n->H1,
                    (void*)n->H2, (void*)n->H3, (void*)n->Z1, (void*)n->Z2, (void*)n->Z3,
                    (void*)n->Y, (void*)n->dY, (void*)n->dZa, (void*)n->dZb, (void*)n->part,
                    (void*)n->grad, (void*)n->lpart})
        (void)hipFree(p);
    delete n;
}

extern "C" int fp_nn_load(fp_ctx* c, fp_nn* n, const float* params, hipStream_t s) {
    if (!c || !n || !params || n->ctx != c) return set_err(c, FP_EINVAL, "fp_nn_load: bad argument");
    hipLaunchKernelGGL(nn_pack_kernel, dim3((IMG_BF + 255) / 256), dim3(256), 0, s, params, n->img,
                       n->sec);
    return check_launch(c, "fp_nn_load");
}

namespace fpg {
int launch_closure_nn(fp_ctx* c, const float* ynn, const float* ysec, double tol_abs,
                      double tol_rel, double relax, const double* mom, double* rec, int32_t* status,
                      hipStream_t s);
}

// network kernel into ybuf ([ncell][16] floats), then the check / de-normalisation kernel
static int closure_nn(fp_ctx* c, const fp_nn* n, const double* mom, double* rec, int32_t* status,
                      double tol_abs, double tol_rel, double relax, float* ybuf, const char* what,
                      hipStream_t s) {
    if (!c || !n || !mom || !rec || !status || n->ctx != c || !(tol_abs >= 0) || !(tol_rel >= 0) ||
        !(relax > 0.0 && relax <= 1.0))
        return set_err(c, FP_EINVAL, std::string(what) + ": bad argument");
    if (c->cfg.moment_order == 3 && tol_abs != INFINITY)
        return set_err(c, FP_EINVAL, std::string(what) + ": the check needs moments through fifth order");
    const int32_t ntiles = (c->ncell + 31) / 32;
    int grid = (ntiles + NN_BLOCK / 64 - 1) / (NN_BLOCK / 64);
    if (grid > 256) grid = 256;   // one workgroup per CU, each loops over its tiles
    hipLaunchKernelGGL(nn_infer_kernel, dim3(grid), dim3(NN_BLOCK), 0, s, c->ncell, mom,
                       c->cfg.eps_hat, (const __bf16*)n->img, (const float*)n->sec, ybuf);
    int rc = check_launch(c, what);
    if (rc) return rc;
    return launch_closure_nn(c, ybuf, n->sec + SEC_YM, tol_abs, tol_rel, relax, mom, rec, status, s);
}

extern "C" int fp_closure_nn(fp_ctx* c, const fp_nn* n, const double* mom, double* rec,
                             int32_t* status, double tol_abs, double tol_rel, double relax,
                             hipStream_t s) {
    if (!c || !n) return set_err(c, FP_EINVAL, "fp_closure_nn: bad argument");
    return closure_nn(c, n, mom, rec, status, tol_abs, tol_rel, relax, n->ybuf, "fp_closure_nn", s);
}

extern "C" int fp_closure_nn_noalloc(fp_ctx* c, const fp_nn* n, const double* mom, double* rec,
                                     int32_t* status, double tol_abs, double tol_rel, double relax,
                                     hipStream_t s) {
    if (!c || !n) return set_err(c, FP_EINVAL, "fp_closure_nn_noalloc: bad argument");
    if (c->ncell > FP_NN_NOALLOC_CELLS)
        return set_err(c, FP_EINVAL, "fp_closure_nn_noalloc: more cells than FP_NN_NOALLOC_CELLS (" +
                                         std::to_string(c->ncell) + " > " +
                                         std::to_string(FP_NN_NOALLOC_CELLS) + ")");
    float* y = scratch_of(c);
    if (!y) return set_err(c, FP_EINVAL, "fp_closure_nn_noalloc: no scratch on this device");
    return closure_nn(c, n, mom, rec, status, tol_abs, tol_rel, relax, y, "fp_closure_nn_noalloc", s);
}

extern "C" int fp_nn_infer(fp_ctx* c, const fp_nn* n, const double* mom, float* y, hipStream_t s) {
    if (!c || !n || !mom || !y || n->ctx != c) return set_err(c, FP_EINVAL, "fp_nn_infer: bad argument");
    if (c->ncell == 0) return FP_OK;
    const int32_t ntiles = (c->ncell + 31) / 32;
    int grid = (ntiles + NN_BLOCK / 64 - 1) / (NN_BLOCK / 64);
    if (grid > 256) grid = 256;
    hipLaunchKernelGGL(nn_infer_kernel, dim3(grid), dim3(NN_BLOCK), 0, s, c->ncell, mom, c->cfg.eps_hat,
                       (const __bf16*)n->img, (const float*)n->sec, y);
    return check_launch(c, "fp_nn_infer");
}

extern "C" int fp_nn_sensitivity(fp_ctx* c, const fp_nn* n, const double* mom, int32_t npass,
                                 double p, uint64_t seed, double* sens, hipStream_t s) {
    if (!c || !n || !mom || !sens || n->ctx != c || npass < 1 || !(p >= 0.0 && p < 1.0))
        return set_err(c, FP_EINVAL, "fp_nn_sensitivity: bad argument");
    const int32_t ntiles = (c->ncell + 31) / 32;
    int grid = (ntiles + SENS_BLOCK / 64 - 1) / (SENS_BLOCK / 64);
    if (grid > 512) grid = 512;
    const uint32_t keep_min = (uint32_t)std::floor(p * 4294967296.0);
    hipLaunchKernelGGL(nn_sense_kernel, dim3(grid), dim3(SENS_BLOCK), 0, s, c->ncell, mom,
                       c->cfg.eps_hat, (const __bf16*)n->img, (const float*)n->sec, npass, seed,
                       keep_min, (float)(1.0 / (1.0 - p)), sens);
    return check_launch(c, "fp_nn_sensitivity");
}

extern "C" int fp_nn_outputs(fp_ctx* c, const fp_nn* n, float* y, hipStream_t s) {
    if (!c || !n || !y) return set_err(c, FP_EINVAL, "fp_nn_outputs: bad argument");
    if (hipMemcpyAsync(y, n->ybuf, sizeof(float) * (size_t)c->ncell * NO, hipMemcpyDeviceToDevice,
                       s) != hipSuccess)
        return set_err(c, FP_EDEVICE, "fp_nn_outputs: copy failed");
    return FP_OK;
}

extern "C" int fp_nn_features(fp_ctx* c, const double* mom, int64_t n, float* feats, hipStream_t s) {
    if (!c || !mom || !feats || n < 0) return set_err(c, FP_EINVAL, "fp_nn_features: bad argument");
    if (n == 0) return FP_OK;
    hipLaunchKernelGGL(nn_features_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, mom,
                       c->cfg.eps_hat, feats);
    return check_launch(c, "fp_nn_features");
}

extern "C" int fp_nn_targets(fp_ctx* c, const double* rec, int64_t n, float* targets, hipStream_t s) {
    if (!c || !rec || !targets || n < 0) return set_err(c, FP_EINVAL, "fp_nn_targets: bad argument");
    if (n == 0) return FP_OK;
    hipLaunchKernelGGL(nn_targets_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, rec,
                       c->cfg.eps_hat, targets);
    return check_launch(c, "fp_nn_targets");
}

extern "C" int fp_closure_build(fp_ctx* c, const double* mom, int64_t n, double* sys, hipStream_t s) {
    if (!c || !mom || !sys || n < 0) return set_err(c, FP_EINVAL, "fp_closure_build: bad argument");
    if (n == 0) return FP_OK;
    hipLaunchKernelGGL(nn_system_kernel, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, s, n, mom,
                       c->cfg.eps_hat, sys);
    return check_launch(c, "fp_closure_build");
}

extern "C" int fp_nn_grad(fp_ctx* c, fp_nn* n, const float* params, const float* feats,
                          const float* targets, const double* sys, int64_t B, int32_t loss_kind,
                          float* grad, float* loss, hipStream_t s) {
    if (!c || !n || !params || !feats || !grad || !loss || B <= 0 || B > n->max_batch ||
        (loss_kind != 0 && loss_kind != 1) || (loss_kind == 0 && !targets) ||
        (loss_kind == 1 && !sys))
        return set_err(c, FP_EINVAL, "fp_nn_grad: bad argument");
    const unsigned g32 = (unsigned)((B + 31) / 32);
    const int nchunk = (int)((B + TRAIN_CHUNK - 1) / TRAIN_CHUNK);
    hipLaunchKernelGGL(nn_input_kernel, dim3((unsigned)((B * NF + 255) / 256)), dim3(256), 0, s, B,
                       feats, params, n->H0);
    hipLaunchKernelGGL((nn_fwd_kernel<NF, NH, true>), dim3(g32), dim3(64), 0, s, B, params + OFF_W1,
                       params + OFF_B1, n->H0, n->Z1, n->H1);
    hipLaunchKernelGGL((nn_fwd_kernel<NH, NH, true>), dim3(g32), dim3(64), 0, s, B, params + OFF_W2,
                       params + OFF_B2, n->H1, n->Z2, n->H2);
    hipLaunchKernelGGL((nn_fwd_kernel<NH, NH, true>), dim3(g32), dim3(64), 0, s, B, params + OFF_W3,
                       params + OFF_B3, n->H2, n->Z3, n->H3);
    hipLaunchKernelGGL((nn_fwd_kernel<NH, NO, false>), dim3(g32), dim3(64), 0, s, B, params + OFF_W4,
                       params + OFF_B4, n->H3, n->Y, (__bf16*)nullptr);
    const int nb = (int)((B + LOSS_BLOCK - 1) / LOSS_BLOCK);
    hipLaunchKernelGGL(nn_loss_kernel, dim3(nb), dim3(LOSS_BLOCK), 0, s, B, (int)loss_kind, params,
                       n->Y, targets, feats, sys, n->dY, n->lpart);
    hipLaunchKernelGGL(nn_loss_final_kernel, dim3(1), dim3(64), 0, s, nb, B, n->lpart, loss);
    const int64_t ps = N_TRAIN;
    // layer 4: dZ4 = dY
    hipLaunchKernelGGL((nn_wgrad_kernel<NO, NH>), dim3(1 * (NH / 32), nchunk), dim3(64), 0, s, B, n->dY,
                       n->H3, n->part, ps, OFF_W4);
    hipLaunchKernelGGL(nn_bgrad_kernel, dim3(nchunk), dim3(128), 0, s, B, NO, n->dY, n->part, ps, OFF_B4);
    hipLaunchKernelGGL((nn_bwd_kernel<NO, NH>), dim3(g32), dim3(64), 0, s, B, params + OFF_W4, n->dY,
                       n->Z3, n->dZa);
    // layer 3
    hipLaunchKernelGGL((nn_wgrad_kernel<NH, NH>), dim3(16, nchunk), dim3(64), 0, s, B, n->dZa, n->H2,
                       n->part, ps, OFF_W3);
    hipLaunchKernelGGL(nn_bgrad_kernel, dim3(nchunk), dim3(128), 0, s, B, NH, n->dZa, n->part, ps, OFF_B3);
    hipLaunchKernelGGL((nn_bwd_kernel<NH, NH>), dim3(g32), dim3(64), 0, s, B, params + OFF_W3, n->dZa,
                       n->Z2, n->dZb);
    // layer 2
    hipLaunchKernelGGL((nn_wgrad_kernel<NH, NH>), dim3(16, nchunk), dim3(64), 0, s, B, n->dZb, n->H1,
                       n->part, ps, OFF_W2);
    hipLaunchKernelGGL(nn_bgrad_kernel, dim3(nchunk), dim3(128), 0, s, B, NH, n->dZb, n->part, ps, OFF_B2);
    hipLaunchKernelGGL((nn_bwd_kernel<NH, NH>), dim3(g32), dim3(64), 0, s, B, params + OFF_W2, n->dZb,
                       n->Z1, n->dZa);
    // layer 1
    hipLaunchKernelGGL((nn_wgrad_kernel<NH, NF>), dim3(4, nchunk), dim3(64), 0, s, B, n->dZa, n->H0,
                       n->part, ps, OFF_W1);
    hipLaunchKernelGGL(nn_bgrad_kernel, dim3(nchunk), dim3(128), 0, s, B, NH, n->dZa, n->part, ps, OFF_B1);
    hipLaunchKernelGGL(nn_reduce_kernel, dim3((N_TRAIN + 255) / 256), dim3(256), 0, s, nchunk, n->part,
                       ps, grad);
    return check_launch(c, "fp_nn_grad");
}

extern "C" int fp_nn_adam(fp_ctx* c, float* params, const float* grad, float* m, float* v,
                          int64_t t, float lr, hipStream_t s) {
    if (!c || !params || !grad || !m || !v || t < 1 || !(lr >= 0.0f))
        return set_err(c, FP_EINVAL, "fp_nn_adam: bad argument");
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = (float)(1.0 - pow(0.9, (double)t)), c2 = (float)(1.0 - pow(0.999, (double)t));
    hipLaunchKernelGGL(nn_adam_kernel, dim3((N_TRAIN + 255) / 256), dim3(256), 0, s, params, grad, m, v,
                       lr, b1, b2, eps, c1, c2);
    return check_launch(c, "fp_nn_adam");
}

extern "C" int fp_nn_train_step(fp_ctx* c, fp_nn* n, float* params, float* m, float* v, int64_t t,
                                float lr, const float* feats, const float* targets, const double* sys,
                                int64_t B, int32_t loss_kind, float* loss, hipStream_t s) {
    if (!n) return set_err(c, FP_EINVAL, "fp_nn_train_step: bad argument");
    int rc = fp_nn_grad(c, n, params, feats, targets, sys, B, loss_kind, n->grad, loss, s);
    if (rc) return rc;
    return fp_nn_adam(c, params, n->grad, m, v, t, lr, s);
}
