// fp_bin.hip -- stable counting sort of particles by cell key.
//
// Particles arrive in the order of the previous sort, so a wave of 64 consecutive
// particles carries only a handful of distinct destination keys.  Each wave folds its
// lanes by key (ballot) into "contributions" (source wave, 64-bit lane mask), one
// integer atomic per distinct key.  A destination cell then orders its contributions
// by source wave, which reproduces the order of a stable counting sort exactly,
// expands them to source indices in LDS and gathers the particle records.  No float
// atomics, no global radix passes; the result is deterministic.
#include "fp_internal.h"

namespace fpg {

constexpr int BIN_BLOCK = 256;

__global__ void bin_zero_kernel(int32_t* __restrict__ cnt, int32_t* __restrict__ ccnt,
                                int32_t* __restrict__ ccur, int32_t len) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) {
        cnt[i] = 0;
        ccnt[i] = 0;
        ccur[i] = 0;
    }
}

// PLACE = false: count particles and contributions per key.
// PLACE = true:  write the contribution records at their slots.
template <bool PLACE>
__global__ __launch_bounds__(BIN_BLOCK) void bin_wave_kernel(
    const int32_t* __restrict__ key, int64_t n, int32_t ncell, int32_t* __restrict__ cnt,
    int32_t* __restrict__ ccnt, int32_t* __restrict__ ccur, const int32_t* __restrict__ coff,
    int32_t* __restrict__ cwave, uint64_t* __restrict__ cmask,
    unsigned long long* __restrict__ errcount) {
    const int64_t p = (int64_t)blockIdx.x * BIN_BLOCK + threadIdx.x;
    const int32_t wave = (int32_t)(p >> 6);
    const int lane = threadIdx.x & 63;
    const bool valid = p < n;
    int32_t k = -1;
    if (valid) {
        k = key[p];
        if (k < 0 || k > ncell) {
            if (!PLACE) atomicAdd(errcount, 1ull);
            k = ncell;  // dropped
        }                // k == ncell: deleted particle, dropped
    }
    uint64_t active = __ballot(valid);
    while (active) {
        const int leader = __builtin_ctzll(active);
        const int32_t kl = __builtin_amdgcn_readlane(k, leader);
        const uint64_t m = __ballot(valid && k == kl);
        if (lane == leader && kl < ncell) {
            if (PLACE) {
                const int32_t slot = coff[kl] + atomicAdd(&ccur[kl], 1);
                cwave[slot] = wave;
                cmask[slot] = m;
            } else {
                atomicAdd(&cnt[kl], __popcll(m));
                atomicAdd(&ccnt[kl], 1);
            }
        }
        active &= ~m;
    }
}

// ---- exclusive scan of two int arrays of length len (ends written at [len]) ------------
constexpr int SCAN_BLOCK = 256, SCAN_ITEMS = 16, SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

__device__ __forceinline__ int32_t block_excl_scan(int32_t v, int32_t* sh, int32_t& total) {
    // Hillis-Steele over the block in shared memory
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < SCAN_BLOCK; off <<= 1) {
        const int32_t add = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    total = sh[SCAN_BLOCK - 1];
    const int32_t incl = sh[t];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(SCAN_BLOCK) void scan_reduce_kernel(
    const int32_t* __restrict__ a, const int32_t* __restrict__ b, int32_t len,
    int32_t* __restrict__ bsum) {
    __shared__ int32_t sh[SCAN_BLOCK];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    int32_t sa = 0, sb = 0;
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        const int64_t j = base + (int64_t)i * SCAN_BLOCK + threadIdx.x;
        if (j < len) {
            sa += a[j];
            sb += b[j];
        }
    }
    int32_t ta, tb;
    block_excl_scan(sa, sh, ta);
    block_excl_scan(sb, sh, tb);
    if (threadIdx.x == 0) {
        bsum[blockIdx.x] = ta;
        bsum[8192 + blockIdx.x] = tb;
    }
}

__global__ __launch_bounds__(SCAN_BLOCK) void scan_blocks_kernel(int32_t* __restrict__ bsum,
                                                                  int32_t nblocks) {
    __shared__ int32_t sh[SCAN_BLOCK];
    for (int arr = 0; arr < 2; ++arr) {
        int32_t* s = bsum + arr * 8192;
        int32_t carry = 0;
        for (int32_t base = 0; base < nblocks; base += SCAN_BLOCK) {
            const int32_t j = base + threadIdx.x;
            const int32_t v = j < nblocks ? s[j] : 0;
            int32_t tot;
            const int32_t ex = block_excl_scan(v, sh, tot);
            if (j < nblocks) s[j] = carry + ex;
            carry += tot;
        }
        if (threadIdx.x == 0) s[nblocks] = carry;
        __syncthreads();
    }
}

// item-contiguous per thread: thread t owns SCAN_ITEMS consecutive elements of the tile
__global__ __launch_bounds__(SCAN_BLOCK) void scan_final_kernel(
    const int32_t* __restrict__ a, const int32_t* __restrict__ b, int32_t len,
    const int32_t* __restrict__ bsum, int32_t nblocks, int32_t* __restrict__ outa,
    int32_t* __restrict__ outb) {
    __shared__ int32_t sh[SCAN_BLOCK];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    int32_t va[SCAN_ITEMS], vb[SCAN_ITEMS];
    int32_t sa = 0, sb = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        const int64_t j = base + i;
        va[i] = j < len ? a[j] : 0;
        vb[i] = j < len ? b[j] : 0;
        sa += va[i];
        sb += vb[i];
    }
    int32_t ta, tb;
    int32_t ea = block_excl_scan(sa, sh, ta) + bsum[blockIdx.x];
    int32_t eb = block_excl_scan(sb, sh, tb) + bsum[8192 + blockIdx.x];
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        const int64_t j = base + i;
        if (j < len) {
            outa[j] = ea;
            outb[j] = eb;
        }
        ea += va[i];
        eb += vb[i];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        outa[len] = bsum[nblocks];
        outb[len] = bsum[8192 + nblocks];
    }
}

// ---- per-cell ordering of contributions and gather --------------------------------------
template <int G>
struct GatherShape {
    static constexpr int GROUPS = BIN_BLOCK / G;
    static constexpr int CAPP = 24 * G;  // particle slots per cell held in LDS
    static constexpr int CAPC = 6 * G;   // contributions per cell held in LDS
};

template <typename T, int G>
__global__ __launch_bounds__(BIN_BLOCK) void bin_gather_kernel(
    int32_t ncell, const int32_t* __restrict__ offsets, const int32_t* __restrict__ coff,
    const int32_t* __restrict__ cwave, const uint64_t* __restrict__ cmask,
    int32_t* __restrict__ gidx, const T* __restrict__ sx, const T* __restrict__ sy,
    const T* __restrict__ svx, const T* __restrict__ svy, const T* __restrict__ svz,
    const uint32_t* __restrict__ spid, T* __restrict__ dx, T* __restrict__ dy,
    T* __restrict__ dvx, T* __restrict__ dvy, T* __restrict__ dvz, uint32_t* __restrict__ dpid,
    int32_t* __restrict__ dkey, int32_t* __restrict__ perm) {
    using S = GatherShape<G>;
    __shared__ int32_t s_w[S::GROUPS][S::CAPC];
    __shared__ uint64_t s_m[S::GROUPS][S::CAPC];
    __shared__ int32_t s_idx[S::GROUPS][S::CAPP];

    const int grp = threadIdx.x / G;
    const int lg = threadIdx.x % G;
    const int32_t cell = blockIdx.x * S::GROUPS + grp;
    const bool in = cell < ncell;
    int32_t b = 0, np = 0, cb = 0, m = 0;
    if (in) {
        b = offsets[cell];
        np = offsets[cell + 1] - b;
        cb = coff[cell];
        m = coff[cell + 1] - cb;
    }
    const bool lds_c = m <= S::CAPC;
    const bool lds_p = np <= S::CAPP;

    // phase A: contributions of this cell into LDS
    if (lds_c)
        for (int32_t j = lg; j < m; j += G) {
            s_w[grp][j] = cwave[cb + j];
            s_m[grp][j] = cmask[cb + j];
        }
    __syncthreads();

    // phase B: slot base of every contribution = particles of contributions from
    // earlier source waves (source waves are unique within a cell); expand lane masks
    int32_t* idx = lds_p ? s_idx[grp] : gidx + b;
    for (int32_t j = lg; j < m; j += G) {
        const int32_t wj = lds_c ? s_w[grp][j] : cwave[cb + j];
        uint64_t mj = lds_c ? s_m[grp][j] : cmask[cb + j];
        int32_t base = 0;
        for (int32_t i = 0; i < m; ++i) {
            const int32_t wi = lds_c ? s_w[grp][i] : cwave[cb + i];
            const uint64_t mi = lds_c ? s_m[grp][i] : cmask[cb + i];
            base += wi < wj ? __popcll(mi) : 0;
        }
        const int32_t src0 = wj << 6;
        while (mj) {
            const int t = __builtin_ctzll(mj);
            idx[base++] = src0 + t;
            mj &= mj - 1;
        }
    }
    __syncthreads();

    // phase C: gather records into the destination slots
    for (int32_t s = lg; s < np; s += G) {
        const int32_t p = idx[s];
        const int32_t d = b + s;
        dx[d] = sx[p];
        if (sy) dy[d] = sy[p];
        dvx[d] = svx[p];
        dvy[d] = svy[p];
        dvz[d] = svz[p];
        dpid[d] = spid[p];
        dkey[d] = cell;
        if (perm) perm[d] = p;
    }
}

template <typename T, int G>
static void gather_launch(fp_ctx* c, const fp_particles* src, fp_particles* dst,
                          const int32_t* offsets, int32_t* perm, hipStream_t s) {
    const int groups = GatherShape<G>::GROUPS;
    const int grid = (c->ncell + groups - 1) / groups;
    const bool two_d = c->cfg.geometry != FP_COUETTE1D;
    hipLaunchKernelGGL((bin_gather_kernel<T, G>), dim3(grid), dim3(BIN_BLOCK), 0, s, c->ncell,
                       offsets, c->coff, c->cwave, c->cmask, c->gidx, (const T*)src->x,
                       two_d ? (const T*)src->y : (const T*)nullptr, (const T*)src->vx,
                       (const T*)src->vy, (const T*)src->vz, src->pid, (T*)dst->x,
                       two_d ? (T*)dst->y : (T*)nullptr, (T*)dst->vx, (T*)dst->vy,
                       (T*)dst->vz, dst->pid, dst->key, perm);
}

template <typename T>
static void gather_dispatch(fp_ctx* c, const fp_particles* src, fp_particles* dst,
                            const int32_t* offsets, int32_t* perm, hipStream_t s) {
    switch (lanes_per_cell(src->n, c->ncell)) {
        case 4: gather_launch<T, 4>(c, src, dst, offsets, perm, s); break;
        case 8: gather_launch<T, 8>(c, src, dst, offsets, perm, s); break;
        case 16: gather_launch<T, 16>(c, src, dst, offsets, perm, s); break;
        case 32: gather_launch<T, 32>(c, src, dst, offsets, perm, s); break;
        default: gather_launch<T, 64>(c, src, dst, offsets, perm, s); break;
    }
}

int launch_bin(fp_ctx* c, const fp_particles* src, fp_particles* dst, int32_t* offsets,
               int32_t* perm, hipStream_t s) {
    const int32_t nc = c->ncell;
    const int64_t n = src->n;
    {
        const int len = nc + 1;
        hipLaunchKernelGGL(bin_zero_kernel, dim3((len + 255) / 256), dim3(256), 0, s, c->cnt,
                           c->ccnt, c->ccur, len);
    }
    const int64_t pgrid = (n + BIN_BLOCK - 1) / BIN_BLOCK;
    if (n > 0)
        hipLaunchKernelGGL(bin_wave_kernel<false>, dim3((unsigned)pgrid), dim3(BIN_BLOCK), 0, s,
                           src->key, n, nc, c->cnt, c->ccnt, c->ccur, (const int32_t*)c->coff,
                           c->cwave, c->cmask, c->errcount);
    const int32_t nblocks = (nc + SCAN_TILE - 1) / SCAN_TILE;
    if (nblocks > 8191) return set_err(c, FP_EINVAL, "fp_bin: too many cells for the scan");
    hipLaunchKernelGGL(scan_reduce_kernel, dim3(nblocks), dim3(SCAN_BLOCK), 0, s, c->cnt,
                       c->ccnt, nc, c->blocksum);
    hipLaunchKernelGGL(scan_blocks_kernel, dim3(1), dim3(SCAN_BLOCK), 0, s, c->blocksum, nblocks);
    hipLaunchKernelGGL(scan_final_kernel, dim3(nblocks), dim3(SCAN_BLOCK), 0, s, c->cnt, c->ccnt,
                       nc, c->blocksum, nblocks, offsets, c->coff);
    if (n > 0)
        hipLaunchKernelGGL(bin_wave_kernel<true>, dim3((unsigned)pgrid), dim3(BIN_BLOCK), 0, s,
                           src->key, n, nc, c->cnt, c->ccnt, c->ccur, (const int32_t*)c->coff,
                           c->cwave, c->cmask, c->errcount);
    if (c->cfg.precision == FP_F32)
        gather_dispatch<float>(c, src, dst, offsets, perm, s);
    else
        gather_dispatch<double>(c, src, dst, offsets, perm, s);
    return check_launch(c, "fp_bin");
}

}  // namespace fpg
