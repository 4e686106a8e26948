// fp_bin.hip -- stable counting sort of particles by cell key.
//
// Particles arrive in the order of the previous sort, so a wave of 64 consecutive
// particles carries only a handful of distinct destination keys.  Each wave folds its
// lanes by key (ballot) into "contributions" (source wave, 64-bit lane mask), one
// integer atomic per distinct key.  A destination cell then orders its contributions
// by source wave, which reproduces the order of a stable counting sort exactly,
// expands them to source indices in LDS and gathers the particle records.  No float
// atomics, no global radix passes; the result is deterministic.
#include "fp_mom_dev.h"
#include "fp_sample_dev.h"

namespace fpg {

constexpr int BIN_BLOCK = 256;

// PLACE = false: count particles and contributions per key: cpair[k] holds both counts
// (particles in its low word, contributions in its high word), so one 64-bit atomic adds
// a contribution.
// PLACE = true:  write the contribution records at their slots.
template <bool PLACE>
__global__ __launch_bounds__(BIN_BLOCK) void bin_wave_kernel(
    const int32_t* __restrict__ key, int64_t n, const int64_t* __restrict__ n_dev, int32_t ncell,
    unsigned long long* __restrict__ cpair, int32_t* __restrict__ ccur,
    const int32_t* __restrict__ coff, int32_t* __restrict__ cwave, uint64_t* __restrict__ cmask,
    unsigned long long* __restrict__ errcount) {
    if (n_dev) n = *n_dev;   // the count kept on the device (the grid covers the slots)
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
    // the lanes of each distinct key: its lowest lane leads and keeps the mask; the leaders'
    // atomics then go out together (one round trip per wave, not one per key in turn)
    uint64_t active = __ballot(valid), mine = 0;
    while (active) {
        const int leader = __builtin_ctzll(active);
        const int32_t kl = __builtin_amdgcn_readlane(k, leader);
        const uint64_t m = __ballot(valid && k == kl);
        if (lane == leader) mine = m;
        active &= ~m;
    }
    if (mine && k < ncell) {
        if (PLACE) {
            const int32_t slot = coff[k] + atomicAdd(&ccur[k], 1);
            cwave[slot] = wave;
            cmask[slot] = mine;
        } else {
            atomicAdd(&cpair[k], (1ull << 32) | (unsigned long long)__popcll(mine));
        }
    }
}

// ---- exclusive scan of two int arrays of length len (ends written at [len]) ------------
constexpr int SCAN_BLOCK = 256, SCAN_ITEMS = 16, SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

__device__ __forceinline__ int32_t block_excl_scan(int32_t v, int32_t* sh, int32_t& total) {
    // wave scans by shuffles, then the SCAN_BLOCK/64 wave totals (sh holds at least
    // SCAN_BLOCK ints; the first SCAN_BLOCK/64 + 1 are used)
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) sh[wv] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t run = 0;
        for (int i = 0; i < SCAN_BLOCK / 64; ++i) {
            const int32_t t = sh[i];
            sh[i] = run;
            run += t;
        }
        sh[SCAN_BLOCK / 64] = run;
    }
    __syncthreads();
    total = sh[SCAN_BLOCK / 64];
    const int32_t r = sh[wv] + x - v;
    __syncthreads();
    return r;
}

// a[j st], b[j st]: two arrays, or (st = 2) the two words of interleaved pairs
__global__ __launch_bounds__(SCAN_BLOCK) void scan_reduce_kernel(
    const int32_t* __restrict__ a, const int32_t* __restrict__ b, int32_t st, int32_t len,
    int32_t* __restrict__ bsum) {
    __shared__ int32_t sh[SCAN_BLOCK];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    int32_t sa = 0, sb = 0;
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        const int64_t j = base + (int64_t)i * SCAN_BLOCK + threadIdx.x;
        if (j < len) {
            sa += a[j * st];
            sb += b[j * st];
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
    const int32_t* __restrict__ a, const int32_t* __restrict__ b, int32_t st, int32_t len,
    const int32_t* __restrict__ bsum, int32_t nblocks, int32_t* __restrict__ outa,
    int32_t* __restrict__ outb) {
    __shared__ int32_t sh[SCAN_BLOCK];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    int32_t va[SCAN_ITEMS], vb[SCAN_ITEMS];
    int32_t sa = 0, sb = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        const int64_t j = base + i;
        va[i] = j < len ? a[j * st] : 0;
        vb[i] = j < len ? b[j * st] : 0;
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
// the general sort's gather runs one wave per workgroup (GBLK lanes; one cell of 64 lanes
// or 64 / G cells): its barriers wait for the wave itself, never for other cells
template <int G>
struct GatherShape {
    static constexpr int BLK = G > 64 ? G : 64;
    static constexpr int GROUPS = BLK / G;
    static constexpr int CAPC = 6 * G;   // contributions per cell held in LDS
};

// position of the r-th set bit (from 0) of a mask with more than r set bits: the half of
// the current window that holds it, by population counts, down to one bit
__device__ __forceinline__ int select_bit(uint64_t m, int r) {
    int pos = 0;
    uint32_t w = (uint32_t)m;
    const int c = __popc(w);
    if (r >= c) {
        r -= c;
        w = (uint32_t)(m >> 32);
        pos = 32;
    }
#pragma unroll
    for (int half = 16; half >= 1; half >>= 1) {
        const int cl = __popc(w & ((1u << half) - 1u));
        if (r >= cl) {
            r -= cl;
            w >>= half;
            pos += half;
        }
    }
    return pos;
}

template <typename T, int G>
__global__ __launch_bounds__(GatherShape<G>::BLK) void bin_gather_kernel(
    int32_t ncell, const int32_t* __restrict__ offsets, const int32_t* __restrict__ coff,
    const int32_t* __restrict__ cwave, const uint64_t* __restrict__ cmask,
    unsigned long long* __restrict__ cpair, int32_t* __restrict__ ccur, int32_t* __restrict__ gidx, const T* __restrict__ sx, const T* __restrict__ sy,
    const T* __restrict__ svx, const T* __restrict__ svy, const T* __restrict__ svz,
    const uint32_t* __restrict__ spid, T* __restrict__ dx, T* __restrict__ dy,
    T* __restrict__ dvx, T* __restrict__ dvy, T* __restrict__ dvz, uint32_t* __restrict__ dpid,
    int32_t* __restrict__ dkey, int32_t* __restrict__ perm, int64_t* __restrict__ kept) {
    if (kept && blockIdx.x == 0 && threadIdx.x == 0) *kept = offsets[ncell];
    using S = GatherShape<G>;
    __shared__ int32_t s_w[S::GROUPS][S::CAPC];
    __shared__ int32_t s_base[S::GROUPS][S::CAPC];
    __shared__ uint64_t s_m[S::GROUPS][S::CAPC];

    // counters of the count and place passes are spent: leave them zero for the next call
    for (int64_t i = (int64_t)blockIdx.x * S::BLK + threadIdx.x; i <= ncell;
         i += (int64_t)gridDim.x * S::BLK) {
        cpair[i] = 0ull;
        ccur[i] = 0;
    }
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

    // phase A: contributions of this cell into LDS
    if (lds_c)
        for (int32_t j = lg; j < m; j += G) {
            s_w[grp][j] = cwave[cb + j];
            s_m[grp][j] = cmask[cb + j];
        }
    __syncthreads();

    // phase B: slot base of every contribution = particles of contributions from earlier
    // source waves (source waves are unique within a cell).  Cells with more
    // contributions than LDS holds expand their masks into a slot list in gidx.
    for (int32_t j = lg; j < m; j += G) {
        const int32_t wj = lds_c ? s_w[grp][j] : cwave[cb + j];
        uint64_t mj = lds_c ? s_m[grp][j] : cmask[cb + j];
        int32_t base = 0;
        for (int32_t i = 0; i < m; ++i) {
            const int32_t wi = lds_c ? s_w[grp][i] : cwave[cb + i];
            const uint64_t mi = lds_c ? s_m[grp][i] : cmask[cb + i];
            base += wi < wj ? __popcll(mi) : 0;
        }
        if (lds_c) {
            s_base[grp][j] = base;
        } else {
            int32_t* idx = gidx + b;
            const int32_t src0 = wj << 6;
            while (mj) {
                const int t = __builtin_ctzll(mj);
                idx[base++] = src0 + t;
                mj &= mj - 1;
            }
        }
    }
    __syncthreads();

    // phase C: every lane takes slots, U per round (slots s0 + u G + lg); the source of slot
    // s is the r-th lane of the contribution whose range [base, base + count) holds s, found
    // for the round's U slots in one pass over the contributions; then all of the round's
    // loads, then its stores
    constexpr int U = 4;
    for (int32_t s0 = 0; s0 < np; s0 += G * U) {
        int32_t src[U];
        if (lds_c) {
            int32_t jj[U], rr[U];
#pragma unroll
            for (int u = 0; u < U; ++u) jj[u] = rr[u] = 0;
            for (int32_t i = 0; i < m; ++i) {
                const int32_t bi = s_base[grp][i], ci = __popcll(s_m[grp][i]);
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int32_t sl = s0 + u * G + lg;
                    if (sl >= bi && sl < bi + ci) {
                        jj[u] = i;
                        rr[u] = sl - bi;
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                src[u] = s0 + u * G + lg < np ? (s_w[grp][jj[u]] << 6) + select_bit(s_m[grp][jj[u]], rr[u]) : -1;
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int32_t sl = s0 + u * G + lg;
                src[u] = sl < np ? gidx[b + sl] : -1;
            }
        }
        T rx[U], ry[U], rvx[U], rvy[U], rvz[U];
        uint32_t rp[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (src[u] < 0) continue;
            const int32_t q = src[u];
            rx[u] = sx[q];
            ry[u] = sy ? sy[q] : (T)0;
            rvx[u] = svx[q];
            rvy[u] = svy[q];
            rvz[u] = svz[q];
            rp[u] = spid[q];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (src[u] < 0) continue;
            const int32_t d = b + s0 + u * G + lg;
            dx[d] = rx[u];
            if (sy) dy[d] = ry[u];
            dvx[d] = rvx[u];
            dvy[d] = rvy[u];
            dvz[d] = rvz[u];
            dpid[d] = rp[u];
            dkey[d] = cell;
            if (perm) perm[d] = src[u];
        }
    }
}

template <typename T, int G>
static void gather_launch(fp_ctx* c, const fp_particles* src, fp_particles* dst,
                          const int32_t* offsets, int32_t* perm, hipStream_t s) {
    const int groups = GatherShape<G>::GROUPS;
    const int grid = (c->ncell + groups - 1) / groups;
    const bool two_d = c->cfg.geometry != FP_COUETTE1D;
    hipLaunchKernelGGL((bin_gather_kernel<T, G>), dim3(grid), dim3(GatherShape<G>::BLK), 0, s, c->ncell,
                       offsets, c->coff, c->cwave, c->cmask, (unsigned long long*)c->cpair, c->ccur, c->gidx,
                       (const T*)src->x,
                       two_d ? (const T*)src->y : (const T*)nullptr, (const T*)src->vx,
                       (const T*)src->vy, (const T*)src->vz, src->pid, (T*)dst->x,
                       two_d ? (T*)dst->y : (T*)nullptr, (T*)dst->vx, (T*)dst->vy,
                       (T*)dst->vz, dst->pid, dst->key, perm, dst->n_dev);
}

template <typename T>
static void gather_dispatch(fp_ctx* c, const fp_particles* src, fp_particles* dst,
                            const int32_t* offsets, int32_t* perm, hipStream_t s) {
    // about one particle per lane, at most 32: the per-cell work (ordering the
    // contributions, expanding their masks) shortens with wider groups (the quadtree
    // cylinder's loop on 7.6e5 leaves of 24 particles: 1.68 ms per step at 32 lanes, 1.70 at
    // 16, 1.91 at 8)
    int g = lanes_per_cell(c, src->n, FILL_8, 1);
    if (c->cfg.lanes <= 0 && g > 32) g = 32;
    switch (g) {
        case 4: gather_launch<T, 4>(c, src, dst, offsets, perm, s); break;
        case 8: gather_launch<T, 8>(c, src, dst, offsets, perm, s); break;
        case 16: gather_launch<T, 16>(c, src, dst, offsets, perm, s); break;
        case 32: gather_launch<T, 32>(c, src, dst, offsets, perm, s); break;
        default: gather_launch<T, 64>(c, src, dst, offsets, perm, s); break;
    }
}

// ---- re-sort of particles that were sorted by cell one step earlier ---------------------
// After a step almost every particle sits in one of the 3 x 3 cells around its old cell.
// Pass 1 (one group per OLD cell) counts the particles bound for each of those nine
// neighbours, and lists the source indices of each direction, in source order, inside
// the old cell's own index range ("buckets": bidx, bucket ends in bend[cell][9]); every
// other particle (moved farther, or after the grouped range) goes to a short far list.
// Every old cell adds its bucket lengths to the counts of the destinations (nine integer
// atomics), far arrivals add one each, and one scan gives the offsets.  Pass 2 (one group per DESTINATION cell)
// concatenates its nine buckets in the order of their old cells -- which is the order of
// source indices, i.e. the stable order -- inserting each far arrival before the buckets
// whose old cell starts after it, and writes its slots contiguously (whole cache lines,
// each written once).  The only global atomics are those of the far list.

// direction 0..8 of key k among the 3 x 3 cells around the old cell (column cx, its row
// starting at cell rs), -1 for any other cell; no division: k's row is told by comparing
// k - rs with 0 and nx
__device__ __forceinline__ int near_dir(int32_t k, int32_t rs, int32_t cx, int32_t nx) {
    const int32_t rel = k - rs;
    const int32_t dy = rel < 0 ? -1 : (rel >= nx ? 1 : 0);
    const int32_t dx = rel - dy * nx - cx;
    if (rel < -nx || rel >= 2 * nx || dx < -1 || dx > 1) return -1;
    return (dy + 1) * 3 + (dx + 1);
}

// inclusive prefix sum over the G consecutive lanes of a group (lane lg of it): steps
// inside rows of 16 lanes by DPP row shifts (lanes before the row start read 0, lanes
// before the group start are masked), then across rows by the row broadcasts
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ uint32_t dpp_u(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xF, true);
}
template <int G>
__device__ __forceinline__ uint32_t group_incl_scan(uint32_t x, int lg) {
    if constexpr (G >= 2) { const uint32_t y = dpp_u<0x111>(x); x += (G >= 16 || lg >= 1) ? y : 0u; }
    if constexpr (G >= 4) { const uint32_t y = dpp_u<0x112>(x); x += (G >= 16 || lg >= 2) ? y : 0u; }
    if constexpr (G >= 8) { const uint32_t y = dpp_u<0x114>(x); x += (G >= 16 || lg >= 4) ? y : 0u; }
    if constexpr (G >= 16) x += dpp_u<0x118>(x);
    if constexpr (G >= 32) x += dpp_u<0x142, 0xA>(x);   // row_bcast:15 into rows 1 and 3
    if constexpr (G >= 64) x += dpp_u<0x143, 0xC>(x);   // row_bcast:31 into rows 2 and 3
    return x;
}

// exclusive prefix sum over a workgroup of BLOCK threads (wave shuffles, then the wave
// totals in LDS); sh holds BLOCK/64 + 1 ints; total receives the sum over the block
template <int BLOCK>
__device__ __forceinline__ int32_t wg_excl_scan(int32_t v, int32_t* sh, int32_t& total) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) sh[wv] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t run = 0;
        for (int i = 0; i < BLOCK / 64; ++i) {
            const int32_t t = sh[i];
            sh[i] = run;
            run += t;
        }
        sh[BLOCK / 64] = run;
    }
    __syncthreads();
    total = sh[BLOCK / 64];
    const int32_t r = sh[wv] + x - v;
    __syncthreads();
    return r;
}

__device__ __forceinline__ void far_put(int32_t k, int32_t j, int64_t slot, int64_t cap,
                                        uint64_t* flist, int32_t* cnt, int32_t* fcnt) {
    if (slot < cap) flist[slot] = ((uint64_t)(uint32_t)k << 32) | (uint32_t)j;
    atomicAdd(&cnt[k], 1);
    atomicAdd(&fcnt[k], 1);
}

// length of the bucket of old cell c for direction d
__device__ __forceinline__ int32_t bucket_len(const int32_t* __restrict__ bend, int32_t c, int d) {
    const int32_t* e = bend + (int64_t)c * 9;
    return e[d] - (d > 0 ? e[d - 1] : 0);
}

// grid: ncell*G lanes for the old cells, then FAR_BLOCKS blocks for the ungrouped tail.
// Far movers are appended to the list with one atomic per block (cells) or per wave
// (tail) on its length: a single counter hit once per particle would serialise.
constexpr int FAR_BLOCKS = 64;

// Order in which the gathers visit destination cells on a 2-D grid: column strips of
// STRIP cells, each strip row by row (a narrower last strip takes the rest).  A
// destination row reads the particles of the three source rows around it; in row-major
// order those rows are a whole grid row apart and their cache lines are evicted from L2
// between the reads, in strip order they are STRIP cells apart.  A bijection on
// [0, nx*ny); the identity for grids no wider than one strip.
constexpr int32_t STRIP = 32;
__device__ __forceinline__ int32_t strip_cell(int32_t t, int32_t nx, int32_t ny) {
    if (nx <= STRIP) return t;
    const int32_t full = nx / STRIP, per = STRIP * ny;
    const int32_t sidx = t / per;
    if (sidx < full) {
        const int32_t r = t - sidx * per;
        return (r / STRIP) * nx + sidx * STRIP + r % STRIP;
    }
    const int32_t w = nx - full * STRIP, r = t - full * per;
    return (r / w) * nx + full * STRIP + r % w;
}

template <int G>
__global__ __launch_bounds__(BIN_BLOCK) void rebin_count_kernel(
    int32_t ncell, int32_t nx, int64_t n, const int64_t* __restrict__ n_dev, int64_t cap,
    int32_t cell_blocks, const int32_t* __restrict__ src_off, const int32_t* __restrict__ key,
    int32_t* __restrict__ bend, int32_t* __restrict__ bidx, int32_t* __restrict__ cnt,
    int32_t* __restrict__ fcnt, int32_t* __restrict__ farn, uint64_t* __restrict__ flist,
    unsigned long long* __restrict__ errcount) {
    if (n_dev) n = *n_dev;
    __shared__ int32_t sh[BIN_BLOCK / 64 + 1];
    __shared__ int32_t s_base;
    __shared__ int32_t s_next[BIN_BLOCK / G][9];
    const int lane = threadIdx.x & 63, grp = threadIdx.x / G;
    const uint64_t below = (1ull << lane) - 1ull;
    if ((int32_t)blockIdx.x >= cell_blocks) {
        // particles after the grouped range: all take the general path
        const int64_t t0 = max((int64_t)src_off[ncell], (int64_t)0);
        const int64_t stride = (int64_t)FAR_BLOCKS * BIN_BLOCK;
        for (int64_t jb = t0 + (int64_t)(blockIdx.x - cell_blocks) * BIN_BLOCK; jb < n;
             jb += stride) {
            const int64_t j = jb + threadIdx.x;
            int32_t k = ncell;
            if (j < n) {
                k = key[j];
                if (k < 0 || k > ncell) {
                    atomicAdd(errcount, 1ull);
                    k = ncell;
                }
            }
            const bool far = k < ncell;
            const uint64_t m = __ballot(far);
            int32_t wbase = 0;
            if (lane == 0 && m) wbase = atomicAdd(farn, (int32_t)__popcll(m));
            wbase = __shfl(wbase, 0, 64);
            if (far) far_put(k, (int32_t)j, (int64_t)wbase + __popcll(m & below), cap, flist, cnt, fcnt);
        }
        return;
    }
    const int64_t gt = (int64_t)blockIdx.x * BIN_BLOCK + threadIdx.x;
    const int32_t cell = (int32_t)(gt / G);
    const int lg = (int)(gt % G);
    int c9[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    int32_t nfar = 0, b = 0, e = 0, cx = 0, rs = 0;
    constexpr int KR = 4;
    int32_t kfirst[KR];   // the keys of the first round, kept for the second pass
#pragma unroll
    for (int u = 0; u < KR; ++u) kfirst[u] = ncell;
    if (cell < ncell) {
        b = max(src_off[cell], 0);
        e = (int32_t)min((int64_t)src_off[cell + 1], n);
        cx = cell % nx;
        rs = cell - cx;
        // branch-free: per round of KR particles the directions are counted in three words
        // of three 10-bit fields (at most KR per field), unpacked once per round
        int32_t nbad = 0;
        for (int32_t j0 = b + lg; j0 < e; j0 += G * KR) {
            int32_t kk[KR];
#pragma unroll
            for (int u = 0; u < KR; ++u) kk[u] = j0 + u * G < e ? key[j0 + u * G] : ncell;
            if (j0 == b + lg)
#pragma unroll
                for (int u = 0; u < KR; ++u) kfirst[u] = kk[u];
            uint32_t w[3] = {0u, 0u, 0u};
#pragma unroll
            for (int u = 0; u < KR; ++u) {
                const int32_t k = kk[u];
                const bool valid = k >= 0 && k < ncell;
                nbad += (!valid && k != ncell) ? 1 : 0;
                const int d = valid ? near_dir(k, rs, cx, nx) : -1;
                nfar += (valid && d < 0) ? 1 : 0;
                const int dw = d < 0 ? 3 : d / 3;
                const uint32_t one = 1u << (10 * (d - 3 * dw));
#pragma unroll
                for (int q = 0; q < 3; ++q) w[q] += dw == q ? one : 0u;
            }
#pragma unroll
            for (int i = 0; i < 9; ++i) c9[i] += (int)((w[i / 3] >> (10 * (i % 3))) & 1023u);
        }
        if (nbad) atomicAdd(errcount, (unsigned long long)nbad);
    }
    // bucket starts inside the cell's range (prefix over directions), same in every lane
    int32_t bst[9];
    {
        int32_t acc = 0;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            c9[i] = group_sum_i<G>(c9[i]);
            bst[i] = acc;
            acc += c9[i];
        }
    }
    if (cell < ncell) {
        if (lg == 0) {
#pragma unroll
            for (int i = 0; i < 9; ++i) bend[(int64_t)cell * 9 + i] = bst[i] + c9[i];
        }
        // this cell's share of the destination counts (integer adds: order-free); lane lg
        // takes directions lg, lg + G, ... (groups may have fewer than 9 lanes)
        for (int q = lg; q < 9; q += G) {
            int32_t cnt_d = 0;
#pragma unroll
            for (int i = 0; i < 9; ++i) cnt_d = q == i ? c9[i] : cnt_d;
            if (cnt_d > 0) atomicAdd(&cnt[cell + (q / 3 - 1) * nx + (q % 3 - 1)], cnt_d);
        }
        // second pass: source indices into the buckets, in source order.  Per round of
        // G particles the rank of a particle among those of its direction is a group
        // prefix sum of one-hot counters (three words of three 10-bit fields; at most
        // G <= 64 per field); the next free position of each direction lives in LDS,
        // advanced after every round by lane lg for directions lg, lg + G, ... (LDS
        // operations of one wave are done in order, so the round's reads see the old
        // value)
        for (int q = lg; q < 9; q += G) {
            int32_t bv = 0;
#pragma unroll
            for (int i = 0; i < 9; ++i) bv = q == i ? bst[i] : bv;
            s_next[grp][q] = bv;
        }
        const int last = lane - lg + G - 1;
        for (int32_t j0 = b; j0 < e; j0 += G * KR) {
            int32_t kk[KR];
            if (j0 == b) {
#pragma unroll
                for (int u = 0; u < KR; ++u) kk[u] = kfirst[u];   // ncell beyond e: no direction
            } else {
#pragma unroll
                for (int u = 0; u < KR; ++u) {
                    const int32_t j = j0 + u * G + lg;
                    kk[u] = j < e ? key[j] : -1;
                }
            }
#pragma unroll
            for (int u = 0; u < KR; ++u) {
                if (j0 + u * G >= e) break;   // group-uniform
                const int32_t k = kk[u];
                int d = -1;
                if (k >= 0 && k < ncell) d = near_dir(k, rs, cx, nx);
                const int dw = d < 0 ? 3 : d / 3, dsh = 10 * (d - 3 * dw);
                const uint32_t w0 = dw == 0 ? 1u << dsh : 0u, w1 = dw == 1 ? 1u << dsh : 0u,
                               w2 = dw == 2 ? 1u << dsh : 0u;
                const uint32_t i0 = group_incl_scan<G>(w0, lg), i1 = group_incl_scan<G>(w1, lg),
                               i2 = group_incl_scan<G>(w2, lg);
                if (d >= 0) {
                    const uint32_t ex = dw == 0 ? i0 - w0 : (dw == 1 ? i1 - w1 : i2 - w2);
                    bidx[b + s_next[grp][d] + (int32_t)((ex >> dsh) & 1023u)] = j0 + u * G + lg;
                }
                const uint32_t t0 = __shfl(i0, last, 64), t1 = __shfl(i1, last, 64),
                               t2 = __shfl(i2, last, 64);
                for (int q = lg; q < 9; q += G) {
                    const int tw = q / 3;
                    const uint32_t tv = tw == 0 ? t0 : (tw == 1 ? t1 : t2);
                    s_next[grp][q] += (int32_t)((tv >> (10 * (q - 3 * tw))) & 1023u);
                }
            }
        }
    }
    int32_t tot;
    const int32_t pre = wg_excl_scan<BIN_BLOCK>(nfar, sh, tot);
    if (tot == 0) return;                      // block-uniform
    if (threadIdx.x == 0) s_base = atomicAdd(farn, tot);
    __syncthreads();
    if (nfar == 0) return;
    int64_t slot = (int64_t)s_base + pre;
    for (int32_t j = b + lg; j < e; j += G) {
        const int32_t k = key[j];
        if (k < 0 || k >= ncell || near_dir(k, rs, cx, nx) >= 0) continue;
        far_put(k, j, slot++, cap, flist, cnt, fcnt);
    }
}

// both exclusive scans for grids of up to SMALL_SCAN_CELLS cells in one launch: each
// workgroup of SSB cells adds up all earlier counts itself (at most a few tens of KB,
// coalesced, one round of loads) instead of waiting for a second pass
constexpr int SSB = 1024, SS_UR = 16;
constexpr int SMALL_SCAN_CELLS = SSB * SS_UR;

// It also splits the far list into per-destination segments for its own cells (every
// workgroup reads the whole list and keeps the entries bound for its range; the slot
// inside a segment comes from an LDS counter, so the order inside a segment is
// arbitrary): no separate far-placement launch on small grids.
__global__ __launch_bounds__(SSB) void rebin_small_scan_kernel(
    int32_t ncell, int64_t cap, const int32_t* __restrict__ cnt, const int32_t* __restrict__ fcnt,
    int32_t* __restrict__ offsets, int32_t* __restrict__ foff, const int32_t* __restrict__ farn,
    const uint64_t* __restrict__ flist, int32_t* __restrict__ fkey, int32_t* __restrict__ fsrc) {
    __shared__ int32_t sh[SSB / 64 + 1];
    __shared__ int32_t s_foff[SSB], s_cur[SSB];
    const int32_t k0 = blockIdx.x * SSB;
    int32_t pa = 0, pb = 0;
#pragma unroll
    for (int u = 0; u < SS_UR; ++u) {
        const int32_t k = u * SSB + threadIdx.x;
        if (k < k0) {
            pa += cnt[k];
            pb += fcnt[k];
        }
    }
    int32_t ta, tb, sa, sb;
    (void)wg_excl_scan<SSB>(pa, sh, ta);
    (void)wg_excl_scan<SSB>(pb, sh, tb);
    const int32_t k = k0 + threadIdx.x;
    const int32_t va = k < ncell ? cnt[k] : 0, vb = k < ncell ? fcnt[k] : 0;
    const int32_t ea = wg_excl_scan<SSB>(va, sh, sa) + ta;
    const int32_t eb = wg_excl_scan<SSB>(vb, sh, sb) + tb;
    if (k < ncell) {
        offsets[k] = ea;
        foff[k] = eb;
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        offsets[ncell] = ta + sa;
        foff[ncell] = tb + sb;
    }
    if (sb == 0) return;    // no far arrivals in this range (block-uniform)
    s_foff[threadIdx.x] = eb;
    s_cur[threadIdx.x] = 0;
    __syncthreads();
    const int64_t nf = min((int64_t)farn[0], cap);
    for (int64_t i = threadIdx.x; i < nf; i += SSB) {
        const uint64_t v = flist[i];
        const int32_t kf = (int32_t)(v >> 32) - k0;
        if (kf < 0 || kf >= SSB) continue;
        const int32_t slot = s_foff[kf] + atomicAdd(&s_cur[kf], 1);
        if (slot < cap) {
            fkey[slot] = kf + k0;
            fsrc[slot] = (int32_t)(uint32_t)v;
        }
    }
}

// far list -> per-destination segments (order inside a segment is arbitrary)
__global__ __launch_bounds__(BIN_BLOCK) void rebin_far_place_kernel(
    int64_t cap, const int32_t* __restrict__ farn, const uint64_t* __restrict__ flist,
    const int32_t* __restrict__ foff, int32_t* __restrict__ fcur, int32_t* __restrict__ fkey,
    int32_t* __restrict__ fsrc) {
    const int64_t nf = min((int64_t)farn[0], cap);
    for (int64_t i = (int64_t)blockIdx.x * BIN_BLOCK + threadIdx.x; i < nf;
         i += (int64_t)gridDim.x * BIN_BLOCK) {
        const uint64_t v = flist[i];
        const int32_t k = (int32_t)(v >> 32), p = (int32_t)(uint32_t)v;
        const int32_t slot = foff[k] + atomicAdd(&fcur[k], 1);
        if (slot < cap) {
            fkey[slot] = k;
            fsrc[slot] = p;
        }
    }
}

template <typename T>
struct Rec {
    const T *sx, *sy, *svx, *svy, *svz;
    const uint32_t* spid;
    T *dx, *dy, *dvx, *dvy, *dvz;
    uint32_t* dpid;
    int32_t *dkey, *perm;
    __device__ __forceinline__ void copy(int32_t p, int32_t d, int32_t k) const {
        dx[d] = sx[p];
        if (sy) dy[d] = sy[p];
        dvx[d] = svx[p];
        dvy[d] = svy[p];
        dvz[d] = svz[p];
        dpid[d] = spid[p];
        dkey[d] = k;
        if (perm) perm[d] = p;
    }
};

// grid: cell blocks (one group of G lanes per destination cell), then FAR_BLOCKS blocks
// for the far arrivals.  Every block also clears a share of fcnt/fcur/farn for the next
// call.
template <typename T, int G>
__global__ __launch_bounds__(BIN_BLOCK) void rebin_gather_kernel(
    int32_t ncell, int32_t nx, int32_t ny, int64_t n, const int64_t* __restrict__ n_dev,
    int64_t* __restrict__ kept, int64_t cap, int32_t cell_blocks,
    const int32_t* __restrict__ src_off, const int32_t* __restrict__ bend,
    const int32_t* __restrict__ bidx, const int32_t* __restrict__ offsets,
    const int32_t* __restrict__ foff, const int32_t* __restrict__ fkey,
    const int32_t* __restrict__ fsrc, int32_t* __restrict__ cnt, int32_t* __restrict__ fcnt,
    int32_t* __restrict__ fcur, int32_t* __restrict__ farn, Rec<T> r) {
    if (n_dev) n = *n_dev;
    if (kept && blockIdx.x == 0 && threadIdx.x == 0) *kept = offsets[ncell];
    constexpr int GROUPS = BIN_BLOCK / G;
    __shared__ int32_t s_run[GROUPS][9][3];   // bucket start in bidx, length, far arrivals before
    for (int64_t i = (int64_t)blockIdx.x * BIN_BLOCK + threadIdx.x; i <= ncell;
         i += (int64_t)gridDim.x * BIN_BLOCK) {
        cnt[i] = 0;
        fcnt[i] = 0;
        fcur[i] = 0;
        if (i == 0) farn[0] = 0;
    }
    const int64_t lim = min((int64_t)offsets[ncell], n);   // slots that exist in dst
    const int32_t fend = (int32_t)min((int64_t)foff[ncell], cap);
    if ((int32_t)blockIdx.x >= cell_blocks) {
        for (int32_t i = (int32_t)(blockIdx.x - cell_blocks) * BIN_BLOCK + threadIdx.x; i < fend;
             i += FAR_BLOCKS * BIN_BLOCK) {
            const int32_t k = fkey[i], p = fsrc[i];
            if (k < 0 || k >= ncell || p < 0 || p >= n) continue;   // only with bad src_off
            const int32_t ky = k / nx, kx = k - ky * nx;
            int32_t slot = offsets[k];
            for (int ey = -1; ey <= 1; ++ey)
                for (int ex = -1; ex <= 1; ++ex) {
                    const int32_t sx = kx - ex, sy = ky - ey;
                    if (sx < 0 || sx >= nx || sy < 0 || sy >= ny) continue;
                    const int32_t c2 = sy * nx + sx;
                    if (src_off[c2] < p) slot += bucket_len(bend, c2, (ey + 1) * 3 + (ex + 1));
                }
            const int32_t f1 = min(foff[k + 1], fend);
            for (int32_t q = foff[k]; q < f1; ++q) slot += fsrc[q] < p ? 1 : 0;
            if (slot >= 0 && slot < lim) r.copy(p, slot, k);
        }
        return;
    }
    const int grp = threadIdx.x / G, lg = threadIdx.x % G;
    const int32_t ord = xcd_block((int32_t)blockIdx.x, cell_blocks) * GROUPS + grp;
    const bool in = ord < ncell;
    const int32_t k = in ? strip_cell(ord, nx, ny) : ord;
    int32_t kx = 0, ky = 0, base = 0;
    if (in) {
        ky = k / nx;
        kx = k - ky * nx;
        base = offsets[k];
    }
    // the nine buckets in the order of their old cells (rows ky-1, ky, ky+1; columns
    // kx-1, kx, kx+1): that is the order of source indices
    for (int q = lg; q < 9; q += G) {
        int32_t st = 0, len = 0, fb = 0;
        const int32_t sy = ky - 1 + q / 3, sx = kx - 1 + q % 3;
        if (in && sx >= 0 && sx < nx && sy >= 0 && sy < ny) {
            const int32_t c2 = sy * nx + sx;
            const int d = (ky - sy + 1) * 3 + (kx - sx + 1);
            const int32_t* e2 = bend + (int64_t)c2 * 9;
            const int32_t b0 = d > 0 ? e2[d - 1] : 0;
            const int32_t s0 = max(src_off[c2], 0);
            st = s0 + b0;
            len = e2[d] - b0;
            const int32_t f1 = min(foff[k + 1], fend);
            for (int32_t f = foff[k]; f < f1; ++f) fb += fsrc[f] < s0 ? 1 : 0;
        }
        s_run[grp][q][0] = st;
        s_run[grp][q][1] = len;
        s_run[grp][q][2] = fb;
    }
    __syncthreads();
    int32_t rs[10], rst[9], rfb[9];
    rs[0] = 0;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        rst[q] = s_run[grp][q][0];
        rs[q + 1] = rs[q] + s_run[grp][q][1];
        rfb[q] = s_run[grp][q][2];
    }
    const int32_t nk = rs[9];
    // position q of the concatenated buckets -> source index, U per lane per round
    constexpr int U = 4;
    for (int32_t q0 = 0; q0 < nk; q0 += G * U) {
        int32_t src[U], dst[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t q = q0 + u * G + lg;
            src[u] = -1;
            dst[u] = -1;
            if (q < nk) {
                int32_t st = rst[0] - rs[0], fb = rfb[0];
#pragma unroll
                for (int t = 1; t < 9; ++t)
                    if (q >= rs[t]) {
                        st = rst[t] - rs[t];
                        fb = rfb[t];
                    }
                src[u] = bidx[st + q];
                dst[u] = base + q + fb;
            }
        }
        T rx[U], ry[U], rvx[U], rvy[U], rvz[U];
        uint32_t rp[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (src[u] >= 0) {
                const int32_t j = src[u];
                rx[u] = r.sx[j];
                ry[u] = r.sy ? r.sy[j] : (T)0;
                rvx[u] = r.svx[j];
                rvy[u] = r.svy[j];
                rvz[u] = r.svz[j];
                rp[u] = r.spid[j];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t d = dst[u];
            if (src[u] >= 0 && d >= 0 && d < lim) {
                r.dx[d] = rx[u];
                if (r.dy) r.dy[d] = ry[u];
                r.dvx[d] = rvx[u];
                r.dvy[d] = rvy[u];
                r.dvz[d] = rvz[u];
                r.dpid[d] = rp[u];
                r.dkey[d] = k;
                if (r.perm) r.perm[d] = src[u];
            }
        }
    }
}

// The gather of one destination cell can also produce the cell's moments (the same
// quantities fp_moments computes from the sorted particles): the group has just written
// every particle of its cell.  In this form the group also places its own far arrivals
// (no separate far blocks) and then reads its fresh slots back (L1/L2-resident) for the
// two moment passes.  Its workgroups are one wave (GM_BLOCK lanes, 64 / G cells, or one
// cell of 64 lanes): the group's barriers (far staging, bucket prefix, slot read-back, the
// moment reduction in LDS) then wait for the wave itself and never for other cells.
constexpr int GM_U = 4;
constexpr int GM_BLOCK = 64;

template <typename T, int G, int NVX, int BLK = GM_BLOCK>
__global__ __launch_bounds__(BLK) void rebin_gather_mom_kernel(
    int32_t ncell, int32_t nx, int32_t ny, int64_t n, const int64_t* __restrict__ n_dev,
    int64_t* __restrict__ kept, int64_t cap,
    const int32_t* __restrict__ src_off, const int32_t* __restrict__ bend,
    const int32_t* __restrict__ bidx, const int32_t* __restrict__ offsets,
    const int32_t* __restrict__ foff, const int32_t* __restrict__ fsrc,
    int32_t* __restrict__ cnt, int32_t* __restrict__ fcnt, int32_t* __restrict__ fcur,
    int32_t* __restrict__ farn, Rec<T> r, double* __restrict__ mom, double* __restrict__ samp) {
    if (n_dev) n = *n_dev;
    if (kept && blockIdx.x == 0 && threadIdx.x == 0) *kept = offsets[ncell];
    constexpr int GROUPS = BLK / G;
    __shared__ int32_t s_run[GROUPS][9][4];   // start in bidx, length, far before, range start
    __shared__ int32_t s_pre[GROUPS][10];     // bucket starts in the cell's concatenation
    __shared__ double s_samp[GROUPS][14];     // the cells' time-average sums
    __shared__ MomShared<BLK, G> sm;
    // far arrivals of a cell staged in LDS, up to FCAP of them (their ranks compare every
    // arrival with all others and with the nine source ranges), in the space of the
    // moment reduction, which is used only after the gather's last barrier: the
    // workgroup's LDS stays below 32 KB (five workgroups per CU)
    constexpr int FCAP = (2048 / GROUPS) < (int)(sizeof(sm.red) / (sizeof(int32_t) * GROUPS))
                             ? (2048 / GROUPS) : (int)(sizeof(sm.red) / (sizeof(int32_t) * GROUPS));
    static_assert(sizeof(int32_t) * GROUPS * FCAP <= sizeof(sm.red), "far staging space");
    int32_t(*s_far)[FCAP] = reinterpret_cast<int32_t(*)[FCAP]>(&sm.red[0][0]);
    for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i <= ncell;
         i += (int64_t)gridDim.x * BLK) {
        cnt[i] = 0;
        fcnt[i] = 0;
        fcur[i] = 0;
        if (i == 0) farn[0] = 0;
    }
    const int64_t lim = min((int64_t)offsets[ncell], n);
    const int32_t fend = (int32_t)min((int64_t)foff[ncell], cap);
    const int grp = threadIdx.x / G, lg = threadIdx.x % G;
    const int32_t ord = xcd_block((int32_t)blockIdx.x, (int32_t)gridDim.x) * GROUPS + grp;
    const bool in = ord < ncell;
    const int32_t k = in ? strip_cell(ord, nx, ny) : ord;
    int32_t kx = 0, ky = 0, base = 0, f0 = 0, f1 = 0;
    if (in) {
        ky = k / nx;
        kx = k - ky * nx;
        base = offsets[k];
        f0 = min(foff[k], fend);
        f1 = min(foff[k + 1], fend);
    }
    // the cell's 14 time-average sums, sum e on lane e % G, loaded now (parked in LDS
    // across the gather and the moments) and updated at the end
    constexpr int SQ = (14 + G - 1) / G;
    const bool samp_cell = samp && in;
    double samp_ld[SQ];
#pragma unroll
    for (int u = 0; u < SQ; ++u) {
        const int e = lg + u * G;
        samp_ld[u] = samp_cell && e < 14 ? samp[(int64_t)k * SAMP + e] : 0.0;
    }
    // the nine buckets' descriptors (bucket start and length in the old cell's range, the
    // range start), loaded before the far staging's barrier
    constexpr int QN = (9 + G - 1) / G;
    int32_t q_st[QN], q_len[QN], q_s0[QN];
#pragma unroll
    for (int u = 0; u < QN; ++u) {
        const int q = lg + u * G;
        q_st[u] = 0;
        q_len[u] = 0;
        q_s0[u] = INT32_MAX;   // a neighbour outside the grid
        const int32_t sy = ky - 1 + q / 3, sx = kx - 1 + q % 3;
        if (q < 9 && in && sx >= 0 && sx < nx && sy >= 0 && sy < ny) {
            const int32_t c2 = sy * nx + sx;
            const int d = (ky - sy + 1) * 3 + (kx - sx + 1);
            const int32_t* e2 = bend + (int64_t)c2 * 9;
            const int32_t b0 = d > 0 ? e2[d - 1] : 0;
            q_s0[u] = max(src_off[c2], 0);
            q_st[u] = q_s0[u] + b0;
            q_len[u] = e2[d] - b0;
        }
    }
    const int32_t nf = f1 - f0;
    const bool far_lds = nf <= FCAP;   // group-uniform
    if (far_lds)
        for (int32_t t = lg; t < nf; t += G) s_far[grp][t] = fsrc[f0 + t];
#pragma unroll
    for (int u = 0; u < SQ; ++u)
        if (samp_cell && lg + u * G < 14) s_samp[grp][lg + u * G] = samp_ld[u];
    __syncthreads();
    auto far_at = [&](int32_t t) __attribute__((always_inline)) {
        return far_lds ? s_far[grp][t] : fsrc[f0 + t];
    };
#pragma unroll
    for (int u = 0; u < QN; ++u) {
        const int q = lg + u * G;
        if (q < 9) {
            int32_t fb = 0;
            if (q_s0[u] != INT32_MAX)
                for (int32_t f = 0; f < nf; ++f) fb += far_at(f) < q_s0[u] ? 1 : 0;
            s_run[grp][q][0] = q_st[u];
            s_run[grp][q][1] = q_len[u];
            s_run[grp][q][2] = fb;
            s_run[grp][q][3] = q_s0[u];
        }
    }
    __syncthreads();
    // bucket starts in the cell's concatenation: lane q adds up the lengths before bucket q
    // (ten lanes at once instead of one lane walking the nine buckets)
    for (int q = lg; q < 10; q += G) {
        int32_t acc = 0;
#pragma unroll
        for (int t = 0; t < 9; ++t) acc += t < q ? s_run[grp][t][1] : 0;
        s_pre[grp][q] = acc;
    }
    __syncthreads();
    int32_t rs[10];
#pragma unroll
    for (int q = 0; q < 10; ++q) rs[q] = s_pre[grp][q];
    const int32_t nk = rs[9];
    // bucket of position q: the number of bucket starts at or before q (the buckets are
    // in order; empty ones share their start), its descriptor read back from LDS
    auto lookup = [&](int32_t q, int32_t& j, int32_t& fb) __attribute__((always_inline)) {
        int t = 0;
#pragma unroll
        for (int tt = 1; tt < 9; ++tt) t += q >= rs[tt] ? 1 : 0;
        fb = s_run[grp][t][2];
        j = ld_off(bidx, s_run[grp][t][0] + q - s_pre[grp][t]);
    };
    // one round: U positions per lane, all loads first; velocities returned
    auto round = [&](int32_t q0, T (&ox)[GM_U], T (&oy)[GM_U], T (&oz)[GM_U])
                     __attribute__((always_inline)) {
        int32_t src[GM_U], dst[GM_U];
#pragma unroll
        for (int u = 0; u < GM_U; ++u) {
            const int32_t q = q0 + u * G + lg;
            src[u] = -1;
            dst[u] = -1;
            if (q < nk) {
                int32_t fb;
                lookup(q, src[u], fb);
                dst[u] = base + q + fb;
            }
        }
        T rx[GM_U], ry[GM_U];
        uint32_t rp[GM_U];
#pragma unroll
        for (int u = 0; u < GM_U; ++u) {
            ox[u] = oy[u] = oz[u] = (T)0;
            if (src[u] >= 0) {
                const int32_t j = src[u];
                rx[u] = ld_off(r.sx, j);
                ry[u] = r.sy ? ld_off(r.sy, j) : (T)0;
                ox[u] = ld_off(r.svx, j);
                oy[u] = ld_off(r.svy, j);
                oz[u] = ld_off(r.svz, j);
                rp[u] = ld_off(r.spid, j);
            }
        }
#pragma unroll
        for (int u = 0; u < GM_U; ++u) {
            const int32_t d = dst[u];
            if (src[u] >= 0 && d >= 0 && d < lim) {
                st_off(r.dx, d, rx[u]);
                if (r.dy) st_off(r.dy, d, ry[u]);
                st_off(r.dvx, d, ox[u]);
                st_off(r.dvy, d, oy[u]);
                st_off(r.dvz, d, oz[u]);
                st_off(r.dpid, d, rp[u]);
                st_off(r.dkey, d, k);
                if (r.perm) st_off(r.perm, d, src[u]);
            }
        }
    };
    // velocities of the first round stay in registers: a cell that one round covers and
    // that has no far arrival takes its moments from them instead of reading its slots back
    T kvx[GM_U], kvy[GM_U], kvz[GM_U];
#pragma unroll
    for (int u = 0; u < GM_U; ++u) kvx[u] = kvy[u] = kvz[u] = (T)0;
    for (int32_t q0 = 0; q0 < nk; q0 += G * GM_U) {
        T tx[GM_U], ty[GM_U], tz[GM_U];
        round(q0, tx, ty, tz);
        if (q0 == 0) {
#pragma unroll
            for (int u = 0; u < GM_U; ++u) {
                kvx[u] = tx[u];
                kvy[u] = ty[u];
                kvz[u] = tz[u];
            }
        }
    }
    // far arrivals of this cell, placed by counting: after every bucket whose old cell
    // starts before it and every arrival with a smaller source index
    for (int32_t i = lg; i < nf; i += G) {
        const int32_t p = far_at(i);
        if (p < 0 || p >= n) continue;   // only with bad src_off
        int32_t slot = base;
#pragma unroll
        for (int q = 0; q < 9; ++q)
            if (s_run[grp][q][3] < p) slot += rs[q + 1] - rs[q];
        for (int32_t f = 0; f < nf; ++f) slot += far_at(f) < p ? 1 : 0;
        if (slot >= 0 && slot < lim) r.copy(p, slot, k);
    }
    // moments of the cell from its sorted slots, in slot order per lane (deterministic:
    // the far arrivals sit in the segment in arbitrary order, their slots do not); the
    // barrier makes the group's writes visible to all of its lanes
    __syncthreads();
    const int32_t ncnt = in ? (int32_t)min((int64_t)nk + (f1 - f0), lim - base) : 0;
    // register path (group-uniform): slot q of the cell is position q, held by lane q % G
    // as round value q / G -- the same values in the same per-lane order as the slots
    const bool regs = nf == 0 && ncnt == nk && nk <= G * GM_U;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    if (regs) {
#pragma unroll
        for (int u = 0; u < GM_U; ++u)
            if (u * G + lg < ncnt) {
                s0 += (double)kvx[u];
                s1 += (double)kvy[u];
                s2 += (double)kvz[u];
            }
    } else {
        for (int32_t q = lg; q < ncnt; q += G) {
            s0 += (double)r.dvx[base + q];
            s1 += (double)r.dvy[base + q];
            s2 += (double)r.dvz[base + q];
        }
    }
    s0 = group_sum<G>(s0);
    s1 = group_sum<G>(s1);
    s2 = group_sum<G>(s2);
    const double inv_n = ncnt > 0 ? 1.0 / (double)ncnt : 0.0;
    const double U0 = s0 * inv_n, U1 = s1 * inv_n, U2 = s2 * inv_n;
    double acc[NVX];
#pragma unroll
    for (int i = 0; i < NVX; ++i) acc[i] = 0.0;
    if (regs) {
#pragma unroll
        for (int u = 0; u < GM_U; ++u)
            if (u * G + lg < ncnt)
                mom_accum<NVX>((double)kvx[u] - U0, (double)kvy[u] - U1, (double)kvz[u] - U2, acc);
    } else {
        for (int32_t q = lg; q < ncnt; q += G)
            mom_accum<NVX>((double)ld_off(r.dvx, base + q) - U0, (double)ld_off(r.dvy, base + q) - U1,
                           (double)ld_off(r.dvz, base + q) - U2, acc);
    }
    mom_finish<BLK, G, NVX>(sm, acc, grp, lg, in, ncnt, U0, U1, U2,
                             mom + (int64_t)(in ? k : 0) * MOM);
    if (samp_cell && lg < 14) {
        // the lane's time-average sums from the record's entries, rebuilt from the final
        // sums in LDS (the values mom_finish stored) instead of reading the record back;
        // every term with a compile-time entry index (no indexed access to m), the lane's
        // own ones kept
        double m[M_T + 10];
#pragma unroll
        for (int e = 0; e < M_T + 10; ++e) m[e] = mom_entry<BLK, G, NVX>(sm, grp, ncnt, U0, U1, U2, e);
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
            if (e < 14) samp[(int64_t)k * SAMP + e] = s_samp[grp][e] + t[u];
        }
    }
}

// Grid of the re-sort's neighbourhoods: the uniform grid, or on the adaptive tree the
// leaves as one row (the leaves just before and after in depth-first order are the side
// buckets; a particle bound for any other leaf takes the far path)
static void rebin_grid(const fp_ctx* c, int32_t& nx, int32_t& ny) {
    nx = c->amr_L >= 0 ? c->ncell : c->cfg.nx;
    ny = c->amr_L >= 0 ? 1 : c->cfg.ny;
}

// pass 1 with G lanes per old cell
template <int G>
static void rebin_count_launch(fp_ctx* c, const fp_particles* src, const int32_t* src_off,
                               hipStream_t s) {
    const int32_t nc = c->ncell;
    int32_t nx, ny;
    rebin_grid(c, nx, ny);
    const int32_t cblocks = (int32_t)(((int64_t)nc * G + BIN_BLOCK - 1) / BIN_BLOCK);
    // cnt, ccnt (far counts), ccur and farn are zero on entry: the previous sort call left
    // them so
    hipLaunchKernelGGL((rebin_count_kernel<G>), dim3(cblocks + FAR_BLOCKS), dim3(BIN_BLOCK), 0, s, nc,
                       nx, src->n, (const int64_t*)src->n_dev, c->cfg.capacity, cblocks, src_off,
                       (const int32_t*)src->key,
                       c->ncnt, c->bidx, c->cnt, c->ccnt, c->farn, c->cmask, c->errcount);
}

// pass 2 with G lanes per destination cell
template <typename T, int G>
static void rebin_gather_launch(fp_ctx* c, const fp_particles* src, const int32_t* src_off,
                                fp_particles* dst, int32_t* offsets, int32_t* perm, double* mom,
                                double* samp, hipStream_t s) {
    const int32_t nc = c->ncell;
    int32_t nx, ny;
    rebin_grid(c, nx, ny);
    const int64_t n = src->n, cap = c->cfg.capacity;
    const bool two_d = c->cfg.geometry != FP_COUETTE1D;
    Rec<T> r{(const T*)src->x,  two_d ? (const T*)src->y : nullptr, (const T*)src->vx,
             (const T*)src->vy, (const T*)src->vz,                   src->pid,
             (T*)dst->x,        two_d ? (T*)dst->y : nullptr,        (T*)dst->vx,
             (T*)dst->vy,       (T*)dst->vz,                         dst->pid,
             dst->key,          perm};
    const int32_t cblocks = (nc + BIN_BLOCK / G - 1) / (BIN_BLOCK / G);
    if (mom) {
        constexpr int BLK = G > GM_BLOCK ? G : GM_BLOCK;
        const int32_t mblocks = (nc + BLK / G - 1) / (BLK / G);
        if (c->cfg.moment_order == 3)
            hipLaunchKernelGGL((rebin_gather_mom_kernel<T, G, NV_LOW, BLK>), dim3(mblocks), dim3(BLK), 0, s,
                               nc, nx, ny, n, (const int64_t*)src->n_dev, dst->n_dev, cap, src_off,
                               (const int32_t*)c->ncnt, (const int32_t*)c->bidx,
                               (const int32_t*)offsets, (const int32_t*)c->coff, (const int32_t*)c->gidx,
                               c->cnt, c->ccnt, c->ccur, c->farn, r, mom, samp);
        else
            hipLaunchKernelGGL((rebin_gather_mom_kernel<T, G, NV, BLK>), dim3(mblocks), dim3(BLK), 0, s,
                               nc, nx, ny, n, (const int64_t*)src->n_dev, dst->n_dev, cap, src_off,
                               (const int32_t*)c->ncnt, (const int32_t*)c->bidx,
                               (const int32_t*)offsets, (const int32_t*)c->coff, (const int32_t*)c->gidx,
                               c->cnt, c->ccnt, c->ccur, c->farn, r, mom, samp);
        return;
    }
    hipLaunchKernelGGL((rebin_gather_kernel<T, G>), dim3(cblocks + FAR_BLOCKS), dim3(BIN_BLOCK),
                       0, s, nc, nx, ny, n, (const int64_t*)src->n_dev, dst->n_dev, cap, cblocks, src_off,
                       (const int32_t*)c->ncnt,
                       (const int32_t*)c->bidx, (const int32_t*)offsets, (const int32_t*)c->coff,
                       (const int32_t*)c->cwave, (const int32_t*)c->gidx, c->cnt, c->ccnt, c->ccur,
                       c->farn, r);
}

template <typename T>
static void rebin_typed(fp_ctx* c, const fp_particles* src, const int32_t* src_off,
                        fp_particles* dst, int32_t* offsets, int32_t* perm, double* mom,
                        double* samp, hipStream_t s) {
    const int32_t nc = c->ncell;
    // count: about 16 particles per lane (its work per particle is a few loads and a key:
    // measured 4 % faster than 8 at 100 per cell); gather: about 4 (its dependent load
    // chains are short per lane), at most 32 (the moment reduction sums G partials per value)
    switch (lanes_per_cell(c, src->n, FILL_4, 16)) {
        case 4: rebin_count_launch<4>(c, src, src_off, s); break;
        case 8: rebin_count_launch<8>(c, src, src_off, s); break;
        case 16: rebin_count_launch<16>(c, src, src_off, s); break;
        case 32: rebin_count_launch<32>(c, src, src_off, s); break;
        default: rebin_count_launch<64>(c, src, src_off, s); break;
    }
    if (nc <= SMALL_SCAN_CELLS) {
        hipLaunchKernelGGL(rebin_small_scan_kernel, dim3((nc + SSB - 1) / SSB), dim3(SSB), 0, s, nc,
                           (int64_t)c->cfg.capacity, (const int32_t*)c->cnt, (const int32_t*)c->ccnt,
                           offsets, c->coff, (const int32_t*)c->farn, (const uint64_t*)c->cmask,
                           c->cwave, c->gidx);
    } else {
        const int32_t nblocks = (nc + SCAN_TILE - 1) / SCAN_TILE;
        hipLaunchKernelGGL(scan_reduce_kernel, dim3(nblocks), dim3(SCAN_BLOCK), 0, s, c->cnt, c->ccnt,
                           1, nc, c->blocksum);
        hipLaunchKernelGGL(scan_blocks_kernel, dim3(1), dim3(SCAN_BLOCK), 0, s, c->blocksum, nblocks);
        hipLaunchKernelGGL(scan_final_kernel, dim3(nblocks), dim3(SCAN_BLOCK), 0, s, c->cnt, c->ccnt, 1, nc,
                           c->blocksum, nblocks, offsets, c->coff);
        hipLaunchKernelGGL(rebin_far_place_kernel, dim3(FAR_BLOCKS), dim3(BIN_BLOCK), 0, s,
                           (int64_t)c->cfg.capacity, (const int32_t*)c->farn, (const uint64_t*)c->cmask,
                           (const int32_t*)c->coff, c->ccur, c->cwave, c->gidx);
    }
    int g = lanes_per_cell(c, src->n, FILL_4, 4);
    if (c->cfg.lanes <= 0 && g > 32) g = 32;
    switch (g) {
        case 4: rebin_gather_launch<T, 4>(c, src, src_off, dst, offsets, perm, mom, samp, s); break;
        case 8: rebin_gather_launch<T, 8>(c, src, src_off, dst, offsets, perm, mom, samp, s); break;
        case 16: rebin_gather_launch<T, 16>(c, src, src_off, dst, offsets, perm, mom, samp, s); break;
        case 32: rebin_gather_launch<T, 32>(c, src, src_off, dst, offsets, perm, mom, samp, s); break;
        default: rebin_gather_launch<T, 64>(c, src, src_off, dst, offsets, perm, mom, samp, s); break;
    }
}

int launch_rebin(fp_ctx* c, const fp_particles* src, const int32_t* src_off, fp_particles* dst,
                 int32_t* offsets, int32_t* perm, double* mom, double* samp, hipStream_t s) {
    if (c->cfg.precision == FP_F32)
        rebin_typed<float>(c, src, src_off, dst, offsets, perm, mom, samp, s);
    else
        rebin_typed<double>(c, src, src_off, dst, offsets, perm, mom, samp, s);
    return check_launch(c, "fp_rebin");
}

int launch_bin(fp_ctx* c, const fp_particles* src, fp_particles* dst, int32_t* offsets,
               int32_t* perm, hipStream_t s) {
    // cpair and ccur are zero on entry (fp_init, and every fp_bin leaves them so)
    const int32_t nc = c->ncell;
    const int64_t n = src->n, slots = slots_of(src);
    const int64_t pgrid = (slots + BIN_BLOCK - 1) / BIN_BLOCK;
    if (slots > 0)
        hipLaunchKernelGGL(bin_wave_kernel<false>, dim3((unsigned)pgrid), dim3(BIN_BLOCK), 0, s,
                           src->key, n, (const int64_t*)src->n_dev, nc, (unsigned long long*)c->cpair,
                           c->ccur, (const int32_t*)c->coff, c->cwave, c->cmask, c->errcount);
    const int32_t nblocks = (nc + SCAN_TILE - 1) / SCAN_TILE;
    if (nblocks > 8191) return set_err(c, FP_EINVAL, "fp_bin: too many cells for the scan");
    hipLaunchKernelGGL(scan_reduce_kernel, dim3(nblocks), dim3(SCAN_BLOCK), 0, s, c->cpair,
                       c->cpair + 1, 2, nc, c->blocksum);
    hipLaunchKernelGGL(scan_blocks_kernel, dim3(1), dim3(SCAN_BLOCK), 0, s, c->blocksum, nblocks);
    hipLaunchKernelGGL(scan_final_kernel, dim3(nblocks), dim3(SCAN_BLOCK), 0, s, c->cpair,
                       c->cpair + 1, 2, nc, c->blocksum, nblocks, offsets, c->coff);
    if (slots > 0)
        hipLaunchKernelGGL(bin_wave_kernel<true>, dim3((unsigned)pgrid), dim3(BIN_BLOCK), 0, s,
                           src->key, n, (const int64_t*)src->n_dev, nc, (unsigned long long*)c->cpair,
                           c->ccur, (const int32_t*)c->coff, c->cwave, c->cmask, c->errcount);
    if (c->cfg.precision == FP_F32)
        gather_dispatch<float>(c, src, dst, offsets, perm, s);
    else
        gather_dispatch<double>(c, src, dst, offsets, perm, s);
    return check_launch(c, "fp_bin");
}

}  // namespace fpg
