// fp_internal.h -- context, layout constants and device helpers of libfpgpu (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>

#include "../../include/fp.h"

namespace fpg {

// ---- record layouts (see include/fp.h) -------------------------------------------------
constexpr int MOM = 32, REC = 16, SAMP = 16, DIAG = 24;
constexpr int AMR_MAX_LEVEL = 4;
enum { M_N = 0, M_U = 1, M_TH = 4, M_P = 5, M_T = 11, M_R = 21, M_W = 27, M_H = 30 };
enum { R_C = 0, R_G = 6, R_TAU = 9, R_TH = 10, R_E = 11, R_EPS2 = 12, R_SIG = 13, R_ST = 14 };
enum { PURPOSE_COLLISION = 3, PURPOSE_WALL = 4, PURPOSE_INJECT = 5, PURPOSE_DROPOUT = 6 };

constexpr double TWO_PI = 6.283185307179586;

}  // namespace fpg

struct fp_ctx {
    fp_config cfg;
    int device = 0;
    int32_t ncell = 0;
    // binning scratch
    int32_t* cnt = nullptr;      // [ncell+1] particles per destination cell
    int32_t* ccnt = nullptr;     // [ncell+1] contribution records per destination cell
    int32_t* coff = nullptr;     // [ncell+1] contribution offsets
    int32_t* ccur = nullptr;     // [ncell+1] contribution cursors
    int32_t* cpair = nullptr;    // [2 (ncell+1)] full sort: per cell the particle count and the
                                 // contribution count, adjacent (one 64-bit atomic adds both)
    int32_t* cwave = nullptr;    // [capacity] contribution: source wave index
    uint64_t* cmask = nullptr;   // [capacity] contribution: lane mask
    int32_t* gidx = nullptr;     // [capacity] slot list for cells too large for LDS
    int32_t* blocksum = nullptr; // scan partials
    int32_t* ncnt = nullptr;     // [ncell*9] re-sort: bucket ends per old cell and direction
    int32_t* bidx = nullptr;     // [capacity] re-sort: source indices bucketed by direction;
                                 // step: per-cell lists of the flights left to flight_rest
    int32_t* farn = nullptr;     // [1] re-sort: length of the list of particles that moved far
    int32_t* pend = nullptr;     // [ncell] step: flights left for flight_rest_kernel per cell
    uint32_t* stepc = nullptr;   // [1] step: the step number collide_kernel read, for flight_rest_kernel
    unsigned long long* errcount = nullptr;  // [2] invalid keys, injection overflows
    // open cylinder domain
    double* vol = nullptr;       // [ncell] gas volume of every cell
    double* nvol = nullptr;      // [ncell] real molecules per particle / gas volume
    int32_t* inj = nullptr;      // [16] per-step counts of the inflow rectangles
    double inj_rect[4][4] = {};  // x_a, x_b, y_a, y_b of the four inflow rectangles
    double inj_lambda[4] = {};   // expected candidates per rectangle and step
    int32_t inj_slot0[5] = {};   // slot prefix: floor(lambda_r) + 1 slots per rectangle
    // surface sampling of the cylinder (fp_wall_sampling): exchange sums of the
    // re-emissions at the body, [wall_nbins][4], caller-owned
    double* wall = nullptr;
    double* wall_edge = nullptr;  // [wall_nbins + 1] cos(k pi / nbins), library-owned
    int32_t wall_nbins = 0;
    // adaptive quadtree (fp_amr_init; the grid of cfg is the finest level): ncell is then
    // the number of leaves and every key is looked up in leafmap
    int32_t amr_L = -1;          // levels below the base grid, -1: no tree
    // leaf numbering generation (fp_amr_init and every fp_amr_adapt advance it) and the one
    // the last fp_bin / fp_rebin sorted by: fp_rebin on a tree needs them equal
    int32_t amr_epoch = 0, sort_epoch = -1;
    int32_t amr_nbx = 0, amr_nby = 0;
    int8_t* amr_state = nullptr; // [nodes] absent / leaf / refined, level-major
    int8_t* amr_flag = nullptr;  // [nodes] 1 split, 2 merge (one adaptation)
    int32_t* amr_age = nullptr;  // [nodes] steps unchanged
    double* amr_sum = nullptr;   // [nodes][8] sums behind the criteria
    int32_t* leafmap = nullptr;  // [nx*ny] leaf of every fine cell
    int32_t* leafmap_old = nullptr;
    int32_t* leaf_node = nullptr;      // [leaves] node of every leaf
    int32_t* leaf_node_old = nullptr;
    int32_t* amr_first = nullptr;      // [nx*ny+1] leaf starts in depth-first order, scanned
    int32_t* amr_part = nullptr;       // scan partials
    double* fine_vol = nullptr;        // [nx*ny] gas volume of the fine cells
    double* vol_old = nullptr;         // [leaves] before the last adaptation
    double* samp_old = nullptr;        // [leaves][16]
    std::string err;
};

namespace fpg {

// ---- error helpers ----------------------------------------------------------------------
int set_err(fp_ctx* c, int code, const std::string& msg);
int check_launch(fp_ctx* c, const char* what);

// ---- Philox4x32-10 (Salmon et al., SC'11) -------------------------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint2 k) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k.x += 0x9E3779B9u;
            k.y += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k.x, (uint32_t)p1,
                       (uint32_t)(p0 >> 32) ^ c.w ^ k.y, (uint32_t)p0);
    }
    return c;
}

__device__ __forceinline__ uint4 draw(uint64_t seed, uint32_t pid, uint32_t step,
                                      uint32_t purpose, uint32_t sub) {
    return philox4x32_10(make_uint4(pid, step, purpose, sub),
                         make_uint2((uint32_t)seed, (uint32_t)(seed >> 32)));
}

// uniform on (0,1): (k + 1/2) 2^-32, exact in double
__device__ __forceinline__ double u01d(uint32_t k) { return ((double)k + 0.5) * 0x1p-32; }
// float version: k rounded to 24 bits, stays in (0, 1]
__device__ __forceinline__ float u01f(uint32_t k) {
    return __builtin_fmaf((float)k, 0x1p-32f, 0x1p-33f);
}

// three standard normals, Box-Muller on (u0,u1) and (u2,u3), double precision
__device__ __forceinline__ void normals3d(uint4 r, double& z0, double& z1, double& z2) {
    const double u0 = u01d(r.x), u1 = u01d(r.y), u2 = u01d(r.z), u3 = u01d(r.w);
    const double r0 = sqrt(-2.0 * log(u0));
    const double r1 = sqrt(-2.0 * log(u2));
    z0 = r0 * cos(TWO_PI * u1);
    z1 = r0 * sin(TWO_PI * u1);
    z2 = r1 * cos(TWO_PI * u3);
}

// -2 ln u for u = (k + 1/2) 2^-32 in single precision (the Box-Muller radius squared).
// Below one half, u01f(k) carries u to 2^-24 relative and its hardware log2 is used
// directly.  Above, u itself is not representable to the precision its logarithm needs: a u
// within 2^-25 of 1 rounds to 1 and would give radius 0 where the exact one reaches 2e-4.
// There t = 1 - u = (~k + 1/2) 2^-32, which FP32 holds to 2^-24 relative, gives
// ln u = ln(1 - t) by the log1p form ln(w) x / (w - 1) with x = -t and w = fl(1 + x)
// (w - 1 is exact for w in [1/2, 1]), and ln u = -t where w rounds to 1.  The result is 0
// never and at least 2.3e-10, never denormal.
__device__ __forceinline__ float m2lnu_f(uint32_t k) {
    constexpr float M2LN2 = -1.3862943611198906f;  // -2 ln 2
    const bool hi = k >= 0x80000000u;
    const float t = __builtin_fmaf((float)(~k), 0x1p-32f, 0x1p-33f);
    const float w = hi ? 1.0f - t : u01f(k);
    const float d = 1.0f - w;
    const float l = M2LN2 * __builtin_amdgcn_logf(w);
    const float f = hi ? t * __builtin_amdgcn_rcpf(d) : 1.0f;
    return (hi && d == 0.0f) ? 2.0f * t : l * f;
}

// single precision: the radius from m2lnu_f, hardware log2 and square root (about 1 ulp;
// the correctly rounded expansion costs a dozen instructions more) and sin/cos of
// revolutions (v_sin/v_cos take x in units of 2 pi, so sin(2 pi u) is one instruction for
// u in (0, 1])
__device__ __forceinline__ void normals3f(uint4 r, float& z0, float& z1, float& z2) {
    const float u1 = u01f(r.y), u3 = u01f(r.w);
    const float r0 = __builtin_amdgcn_sqrtf(m2lnu_f(r.x));
    const float r1 = __builtin_amdgcn_sqrtf(m2lnu_f(r.z));
    z0 = r0 * __builtin_amdgcn_cosf(u1);
    z1 = r0 * __builtin_amdgcn_sinf(u1);
    z2 = r1 * __builtin_amdgcn_cosf(u3);
}

// ---- cell key from a stored position (double, no contraction) --------------------------
__device__ __forceinline__ int32_t axis_cell(double pos, double origin, double inv_h,
                                             int32_t n) {
    const double f = floor(__dmul_rn(__dsub_rn(pos, origin), inv_h));
    if (!(f >= 0.0)) return 0;
    if (f > (double)(n - 1)) return n - 1;
    return (int32_t)f;
}

// ---- cross-lane sums inside aligned groups of G lanes (result in every lane) -----------
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    // every source lane of these row patterns exists, so bound_ctrl changes no value; it
    // lets the compiler drop the copy of the unused "old" operand
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}

template <int G>
__device__ __forceinline__ double group_sum(double v) {
    static_assert(G == 1 || G == 2 || G == 4 || G == 8 || G == 16 || G == 32 || G == 64, "G");
    if constexpr (G >= 2) v += dpp_d<0xB1>(v);   // quad_perm [1,0,3,2]: lane ^ 1
    if constexpr (G >= 4) v += dpp_d<0x4E>(v);   // quad_perm [2,3,0,1]: lane ^ 2
    if constexpr (G >= 8) v += dpp_d<0x141>(v);  // row_half_mirror: other quad of 8
    if constexpr (G >= 16) v += dpp_d<0x140>(v); // row_mirror: other half of 16
    if constexpr (G >= 32) v += __shfl_xor(v, 16, 64);
    if constexpr (G >= 64) v += __shfl_xor(v, 32, 64);
    return v;
}

// Workgroups are handed to the 8 XCDs (each with its own L2) round robin.  xcd_block
// renumbers the first nblocks workgroups so that each XCD gets one contiguous range of
// logical blocks: neighbouring cells, which share destination cache lines in the
// re-sort, then meet in the same L2.  A bijection on [0, nblocks).
constexpr int NUM_XCD = 8;
__device__ __forceinline__ int32_t xcd_block(int32_t bid, int32_t nblocks) {
    const int32_t q = nblocks / NUM_XCD, r = nblocks % NUM_XCD;
    const int32_t x = bid % NUM_XCD, i = bid / NUM_XCD;
    return x * q + min(x, r) + i;
}

template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}

template <int G>
__device__ __forceinline__ int group_sum_i(int v) {
    if constexpr (G >= 2) v += dpp_i<0xB1>(v);
    if constexpr (G >= 4) v += dpp_i<0x4E>(v);
    if constexpr (G >= 8) v += dpp_i<0x141>(v);
    if constexpr (G >= 16) v += dpp_i<0x140>(v);
    if constexpr (G >= 32) v += __shfl_xor(v, 16, 64);
    if constexpr (G >= 64) v += __shfl_xor(v, 32, 64);
    return v;
}

// ---- host-side launch shape of the per-cell kernels -------------------------------------
// Lanes per cell: about ppl particles per lane from the mean occupancy, and at least
// enough lanes that the grid holds min_threads work-items (small grids would leave most
// SIMDs idle); 4..64 lanes.  cfg.lanes > 0 overrides both.
inline int lanes_per_cell(const fp_ctx* c, int64_t n, int64_t min_threads = 0, int ppl = 8) {
    if (c->cfg.lanes > 0) return c->cfg.lanes;
    const double avg = c->ncell > 0 ? (double)n / (double)c->ncell : 0.0;
    int g = 4;
    while (g < 64 && (double)g * ppl < avg * 1.25) g *= 2;
    while (g < 64 && (int64_t)c->ncell * g < min_threads) g *= 2;
    return g;
}
// grid sizes below which the per-cell kernels widen their groups (about four, resp. eight,
// resident waves on each of the 1024 SIMDs)
constexpr int64_t FILL_4 = 1024 * 4 * 64, FILL_8 = 1024 * 8 * 64;

// Element j of a device array as its base plus a 32-bit byte offset: with the base in
// SGPRs (a kernel argument) the compiler uses the global load/store form that takes one
// VGPR for the offset, shared by the arrays of one element size, instead of a 64-bit
// address per array and element.  The context's capacity limit keeps every particle
// array's byte offsets below 2^32.
template <typename T>
__device__ __forceinline__ T ld_off(const T* base, int32_t j) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) +
                                       (uint32_t)j * (uint32_t)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void st_off(T* base, int32_t j, T v) {
    *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + (uint32_t)j * (uint32_t)sizeof(T)) = v;
}

// slots a call's per-particle grid covers: the host count, or with a device count
// (p->n_dev) the capacity of the arrays
inline int64_t slots_of(const fp_particles* p) {
    return p->n_dev ? (p->capacity > 0 ? p->capacity : p->n) : p->n;
}

// ---- launchers implemented in the kernel files -------------------------------------------
int launch_bin(fp_ctx* c, const fp_particles* src, fp_particles* dst, int32_t* offsets,
               int32_t* perm, hipStream_t s);
int launch_diagnostics(fp_ctx* c, const double* samp, double theta_inf, double n_inf,
                       double dg_inf, double* diag, hipStream_t s);
int launch_surface(fp_ctx* c, const double* sums, int32_t nbins, double t_total, double* out,
                   hipStream_t s);
int launch_sample_high(fp_ctx* c, const double* mom, double* hsamp, hipStream_t s);
int launch_high_order(fp_ctx* c, const double* hsamp, double* out, hipStream_t s);
int launch_rebin(fp_ctx* c, const fp_particles* src, const int32_t* src_off, fp_particles* dst,
                 int32_t* offsets, int32_t* perm, double* mom, double* samp, hipStream_t s);
int launch_moments(fp_ctx* c, const fp_particles* p, const int32_t* offsets, double* mom,
                   double* samp0, double* samp1, hipStream_t s);
int launch_closure(fp_ctx* c, const double* mom, double* rec, int32_t* status, hipStream_t s);
int launch_inject(fp_ctx* c, fp_particles* p, int64_t at, uint32_t* pid_next, uint32_t step,
                  const uint32_t* step_dev, uint32_t* advance, hipStream_t s);
int launch_step(fp_ctx* c, fp_particles* p, const int32_t* offsets, const double* mom,
                const double* rec, uint64_t step, uint32_t flags, const uint32_t* step_dev,
                hipStream_t s);
int launch_counter_add(fp_ctx* c, uint32_t* ctr, uint32_t inc, hipStream_t s);
int launch_sample(fp_ctx* c, const double* mom, double* samp, hipStream_t s);

}  // namespace fpg
