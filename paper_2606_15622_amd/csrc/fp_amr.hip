// fp_amr.hip -- adaptive quadtree of the cylinder domain (Sec. "Extension to External
// Aerodynamics", Problem Description).
//
// The context's grid is the finest level; a base grid of (nx >> L) x (ny >> L) cells is
// refined up to L levels.  The tree lives in per-level node arrays (state ABSENT / LEAF /
// REFINED and the age of every node, level-major, row-major inside a level).  Leaves are
// numbered depth first (base cells row-major, children (0,0) (1,0) (0,1) (1,1)), so the
// fine cells of a leaf form one range of the depth-first (Morton) order of the fine
// cells: one flag per fine cell at the start of each leaf and one exclusive scan number
// all leaves, and leafmap[fine cell] gives the key of the particles in it.  Every kernel
// that computes a key from a position looks it up there, so the step, the sort, the
// moments, the closure and the sampling run unchanged on the leaves.
//
// One adaptation: leaf sums (from sampling sums accumulated since the last adaptation)
// -> sums of refined nodes, bottom up -> split flags of leaves -> merge flags of parents
// of four leaves -> new states and ages (each node writes only itself) -> numbering,
// map, leaf volumes -> sampling sums carried over -> particle keys.  The decisions are
// FP64 without contraction, in a fixed order of the sums, so that a plain CPU evaluation
// takes the same ones.
#include "fp_internal.h"

#pragma clang fp contract(off)

namespace fpg {

enum : int8_t { N_ABSENT = 0, N_LEAF = 1, N_REFINED = 2 };
constexpr int AMR_BLOCK = 256;
constexpr int SUMW = 8;   // node sums: S0, S1x, S1y, S1z, S2, V, samples, pad

struct TreeDims {
    int32_t L, nbx, nby, nxf;
    int64_t off[AMR_MAX_LEVEL + 2];   // first node of every level, off[L+1] = node count
};

__device__ __forceinline__ int level_of(const TreeDims& t, int64_t n) {
    int l = 0;
    while (l < t.L && n >= t.off[l + 1]) ++l;
    return l;
}

__device__ __forceinline__ int64_t node_at(const TreeDims& t, int l, int32_t ix, int32_t iy) {
    return t.off[l] + (int64_t)iy * (t.nbx << l) + ix;
}

__device__ __forceinline__ uint32_t morton2(uint32_t lx, uint32_t ly, int bits) {
    uint32_t d = 0;
    for (int k = 0; k < bits; ++k) d |= (((lx >> k) & 1u) << (2 * k)) | (((ly >> k) & 1u) << (2 * k + 1));
    return d;
}

__device__ __forceinline__ void demorton2(uint32_t d, int bits, uint32_t& lx, uint32_t& ly) {
    lx = ly = 0;
    for (int k = 0; k < bits; ++k) {
        lx |= ((d >> (2 * k)) & 1u) << k;
        ly |= ((d >> (2 * k + 1)) & 1u) << k;
    }
}

// the leaf above fine cell (fx, fy): its level and node
__device__ __forceinline__ int64_t leaf_above(const TreeDims& t, const int8_t* __restrict__ state,
                                              int32_t fx, int32_t fy, int& lev) {
    for (int l = 0; l <= t.L; ++l) {
        const int64_t n = node_at(t, l, fx >> (t.L - l), fy >> (t.L - l));
        if (state[n] == N_LEAF) {
            lev = l;
            return n;
        }
    }
    lev = -1;   // not a valid tree
    return -1;
}

__global__ void amr_init_kernel(int64_t nodes, int64_t nbase, int8_t* __restrict__ state,
                                int32_t* __restrict__ age) {
    const int64_t n = (int64_t)blockIdx.x * AMR_BLOCK + threadIdx.x;
    if (n >= nodes) return;
    state[n] = n < nbase ? N_LEAF : N_ABSENT;
    age[n] = 0;
}

// flag[d] = 1 where depth-first fine cell d starts a leaf
__global__ void amr_first_kernel(TreeDims t, const int8_t* __restrict__ state,
                                 int32_t* __restrict__ flag) {
    const int64_t d = (int64_t)blockIdx.x * AMR_BLOCK + threadIdx.x;
    const int64_t total = (int64_t)t.nbx * t.nby << (2 * t.L);
    if (d >= total) return;
    const int64_t base = d >> (2 * t.L);
    uint32_t lx, ly;
    demorton2((uint32_t)(d & (((int64_t)1 << (2 * t.L)) - 1)), t.L, lx, ly);
    const int32_t fx = (int32_t)(base % t.nbx) * (1 << t.L) + (int32_t)lx;
    const int32_t fy = (int32_t)(base / t.nbx) * (1 << t.L) + (int32_t)ly;
    int l;
    leaf_above(t, state, fx, fy, l);
    const int s = 2 * (t.L - (l < 0 ? t.L : l));
    flag[d] = ((d >> s) << s) == d ? 1 : 0;
}

// ---- exclusive scan of n ints in place, total at [n] ------------------------------------
constexpr int ASCAN_ITEMS = 16, ASCAN_TILE = AMR_BLOCK * ASCAN_ITEMS;

__device__ __forceinline__ int32_t block_scan_excl(int32_t v, int32_t& total) {
    __shared__ int32_t wsum[AMR_BLOCK / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    int32_t pre = 0;
    total = 0;
#pragma unroll
    for (int k = 0; k < AMR_BLOCK / 64; ++k) {
        if (k < w) pre += wsum[k];
        total += wsum[k];
    }
    __syncthreads();
    return pre + x - v;
}

__global__ void amr_scan_tiles_kernel(int64_t n, int32_t* __restrict__ a, int32_t* __restrict__ part) {
    const int64_t t0 = (int64_t)blockIdx.x * ASCAN_TILE + (int64_t)threadIdx.x * ASCAN_ITEMS;
    int32_t v[ASCAN_ITEMS], s = 0;
#pragma unroll
    for (int i = 0; i < ASCAN_ITEMS; ++i) {
        v[i] = t0 + i < n ? a[t0 + i] : 0;
        s += v[i];
    }
    int32_t total;
    int32_t run = block_scan_excl(s, total);
#pragma unroll
    for (int i = 0; i < ASCAN_ITEMS; ++i) {
        if (t0 + i < n) a[t0 + i] = run;
        run += v[i];
    }
    if (threadIdx.x == 0) part[blockIdx.x] = total;
}

// one workgroup: exclusive scan of the tile totals, grand total at part[ntiles]
__global__ void amr_scan_parts_kernel(int32_t ntiles, int32_t* __restrict__ part) {
    int32_t carry = 0;
    for (int32_t b = 0; b < ntiles; b += AMR_BLOCK) {
        const int32_t i = b + (int32_t)threadIdx.x;
        const int32_t v = i < ntiles ? part[i] : 0;
        int32_t total;
        const int32_t e = block_scan_excl(v, total);
        if (i < ntiles) part[i] = carry + e;
        carry += total;
    }
    if (threadIdx.x == 0) part[ntiles] = carry;
}

__global__ void amr_scan_add_kernel(int64_t n, int32_t* __restrict__ a, const int32_t* __restrict__ part) {
    const int64_t i = (int64_t)blockIdx.x * AMR_BLOCK + threadIdx.x;
    if (i < n) a[i] += part[i / ASCAN_TILE];
    if (i == 0) a[n] = part[(n + ASCAN_TILE - 1) / ASCAN_TILE];
}

// leafmap[f] (fine cell f row-major) and leaf_node[leaf]
__global__ void amr_map_kernel(TreeDims t, const int8_t* __restrict__ state,
                               const int32_t* __restrict__ first, int32_t* __restrict__ leafmap,
                               int32_t* __restrict__ leaf_node) {
    const int64_t f = (int64_t)blockIdx.x * AMR_BLOCK + threadIdx.x;
    const int64_t total = (int64_t)t.nbx * t.nby << (2 * t.L);
    if (f >= total) return;
    const int32_t fx = (int32_t)(f % t.nxf), fy = (int32_t)(f / t.nxf);
    int l;
    const int64_t node = leaf_above(t, state, fx, fy, l);
    if (node < 0) {
        leafmap[f] = -1;
        return;
    }
    const int32_t mask = (1 << t.L) - 1;
    const int64_t base = (int64_t)(fy >> t.L) * t.nbx + (fx >> t.L);
    const uint32_t m = morton2((uint32_t)(fx & mask), (uint32_t)(fy & mask), t.L);
    const int s = 2 * (t.L - l);
    const int64_t d0 = (base << (2 * t.L)) + ((m >> s) << s);
    const int32_t id = first[d0];
    leafmap[f] = id;
    if (((m >> s) << s) == m) leaf_node[id] = (int32_t)node;
}

__device__ __forceinline__ void node_xy(const TreeDims& t, int64_t node, int& l, int32_t& ix, int32_t& iy) {
    l = level_of(t, node);
    const int64_t r = node - t.off[l];
    ix = (int32_t)(r % (t.nbx << l));
    iy = (int32_t)(r / (t.nbx << l));
}

// gas volume of every leaf (fine cells added depth first) and fnum / volume
__global__ void amr_vol_kernel(TreeDims t, int32_t nleaf, const int32_t* __restrict__ leaf_node,
                               const double* __restrict__ fine_vol, double fnum, double full_fine,
                               double* __restrict__ vol, double* __restrict__ nvol) {
    const int32_t id = (int32_t)(blockIdx.x * AMR_BLOCK + threadIdx.x);
    if (id >= nleaf) return;
    int l;
    int32_t ix, iy;
    node_xy(t, leaf_node[id], l, ix, iy);
    const int s = t.L - l;
    double v = 0.0;
    for (uint32_t d = 0; d < (1u << (2 * s)); ++d) {
        uint32_t lx, ly;
        demorton2(d, s, lx, ly);
        const int64_t f = (int64_t)((iy << s) + (int32_t)ly) * t.nxf + (ix << s) + (int32_t)lx;
        v = v + fine_vol[f];
    }
    const double full = full_fine * (double)(1u << (2 * s));
    vol[id] = v;
    nvol[id] = fnum / (v > 0.0 ? v : full);
}

// node sums of the leaves from their sampling sums (samples: entry 13)
__global__ void amr_leaf_sum_kernel(int32_t nleaf, const int32_t* __restrict__ leaf_node,
                                    const double* __restrict__ acc, const double* __restrict__ vol,
                                    double* __restrict__ sum) {
    const int32_t id = (int32_t)(blockIdx.x * AMR_BLOCK + threadIdx.x);
    if (id >= nleaf) return;
    const double* a = acc + (int64_t)id * SAMP;
    double* o = sum + (int64_t)leaf_node[id] * SUMW;
    o[0] = a[0];
    o[1] = a[1];
    o[2] = a[2];
    o[3] = a[3];
    o[4] = (a[4] + a[7]) + a[9];
    o[5] = vol[id];
    o[6] = a[13];
    o[7] = 0.0;
}

// refined nodes of level l: sums of their four children, in order
__global__ void amr_up_kernel(TreeDims t, int l, const int8_t* __restrict__ state, double* __restrict__ sum) {
    const int64_t r = (int64_t)blockIdx.x * AMR_BLOCK + threadIdx.x;
    const int64_t cnt = (int64_t)(t.nbx << l) * (t.nby << l);
    if (r >= cnt) return;
    const int64_t node = t.off[l] + r;
    if (state[node] != N_REFINED) return;
    const int32_t ix = (int32_t)(r % (t.nbx << l)), iy = (int32_t)(r / (t.nbx << l));
    const double* c0 = sum + node_at(t, l + 1, 2 * ix, 2 * iy) * SUMW;
    double s[6];
    for (int k = 0; k < 6; ++k) s[k] = c0[k];
    for (int c = 1; c < 4; ++c) {
        const double* ch = sum + node_at(t, l + 1, 2 * ix + (c & 1), 2 * iy + (c >> 1)) * SUMW;
        for (int k = 0; k < 6; ++k) s[k] = s[k] + ch[k];
    }
    double* o = sum + node * SUMW;
    for (int k = 0; k < 6; ++k) o[k] = s[k];
    o[6] = c0[6];
    o[7] = 0.0;
}

struct Fields {
    double rho, th, P;
};

__device__ __forceinline__ Fields fields_of(const double* s, double fnum, double mass) {
    const double S0 = s[0], V = s[5], ns = s[6];
    const double u0 = s[1] / S0, u1 = s[2] / S0, u2 = s[3] / S0;
    Fields f;
    f.th = (s[4] / S0 - ((u0 * u0 + u1 * u1) + u2 * u2)) / 3.0;
    f.rho = ((S0 / ns) * fnum) / V;
    f.P = (f.rho * mass) * f.th;
    return f;
}

__device__ __forceinline__ double dev(double a, double b, double eps) {
    return fabs(a - b) / (fabs(a) + eps);
}

__device__ __forceinline__ double max_dev(const Fields& a, const Fields& b, double eps) {
    return fmax(fmax(dev(a.rho, b.rho, eps), dev(a.th, b.th, eps)), dev(a.P, b.P, eps));
}

// split flags of the leaves (flag 1)
__global__ void amr_split_kernel(TreeDims t, int32_t nleaf, const int32_t* __restrict__ leaf_node,
                                 const double* __restrict__ sum, fp_amr_params p, double fnum,
                                 double mass, int8_t* __restrict__ flag) {
    const int32_t id = (int32_t)(blockIdx.x * AMR_BLOCK + threadIdx.x);
    if (id >= nleaf) return;
    const int64_t node = leaf_node[id];
    int l;
    int32_t ix, iy;
    node_xy(t, node, l, ix, iy);
    if (l >= t.L) return;
    const double* s = sum + node * SUMW;
    const double S0 = s[0], V = s[5], ns = s[6];
    if (!(V > 0.0)) return;
    bool split = ns > 0.0 && S0 / ns > p.n_max;
    if (S0 >= p.n_grad) {
        const Fields f = fields_of(s, fnum, mass);
        if (f.P > p.shock_factor * p.p_inf) split = true;
        if (l > 0) {
            const double* sp = sum + node_at(t, l - 1, ix >> 1, iy >> 1) * SUMW;
            if (sp[0] >= p.n_grad && max_dev(f, fields_of(sp, fnum, mass), p.eps) > p.tau_grad) split = true;
        }
    }
    if (split) flag[node] = 1;
}

// merge flags (2) of refined nodes of level l whose four children are leaves
__global__ void amr_merge_kernel(TreeDims t, int l, const int8_t* __restrict__ state,
                                 const int32_t* __restrict__ age, const double* __restrict__ sum,
                                 fp_amr_params p, double fnum, double mass, int8_t* __restrict__ flag) {
    const int64_t r = (int64_t)blockIdx.x * AMR_BLOCK + threadIdx.x;
    const int64_t cnt = (int64_t)(t.nbx << l) * (t.nby << l);
    if (r >= cnt) return;
    const int64_t node = t.off[l] + r;
    if (state[node] != N_REFINED) return;
    const int32_t ix = (int32_t)(r % (t.nbx << l)), iy = (int32_t)(r / (t.nbx << l));
    int64_t kid[4];
    for (int c = 0; c < 4; ++c) {
        kid[c] = node_at(t, l + 1, 2 * ix + (c & 1), 2 * iy + (c >> 1));
        if (state[kid[c]] != N_LEAF) return;
    }
    const double* s = sum + node * SUMW;
    const double S0 = s[0], ns = s[6];
    if (ns > 0.0 && S0 / ns > p.n_max) return;
    const bool has = S0 >= p.n_grad;
    Fields fp{0.0, 0.0, 0.0};
    if (has) {
        fp = fields_of(s, fnum, mass);
        if (fp.P > p.shock_factor * p.p_inf) return;
    }
    for (int c = 0; c < 4; ++c) {
        if (flag[kid[c]] == 1 || age[kid[c]] < p.age_min) return;
        const double* sk = sum + kid[c] * SUMW;
        // a child with n_grad particles makes the parent's count >= n_grad
        if (sk[0] >= p.n_grad && !(max_dev(fields_of(sk, fnum, mass), fp, p.eps) < p.tau_coarse)) return;
    }
    flag[node] = 2;
}

// new state and age of every node; a node writes only itself and reads its parent's flag
__global__ void amr_apply_kernel(TreeDims t, int32_t steps, int8_t* __restrict__ state,
                                 int32_t* __restrict__ age, const int8_t* __restrict__ flag) {
    const int64_t n = (int64_t)blockIdx.x * AMR_BLOCK + threadIdx.x;
    if (n >= t.off[t.L + 1]) return;
    int l;
    int32_t ix, iy;
    node_xy(t, n, l, ix, iy);
    const int8_t pf = l > 0 ? flag[node_at(t, l - 1, ix >> 1, iy >> 1)] : 0;
    const int8_t st = state[n];
    if (st == N_LEAF) {
        if (flag[n] == 1) {
            state[n] = N_REFINED;
        } else if (pf == 2) {
            state[n] = N_ABSENT;
            age[n] = 0;
        } else {
            const int64_t a = (int64_t)age[n] + steps;
            age[n] = (int32_t)(a < 2147483647 ? a : 2147483647);
        }
    } else if (st == N_REFINED) {
        if (flag[n] == 2) {
            state[n] = N_LEAF;
            age[n] = 0;
        }
    } else if (pf == 1) {
        state[n] = N_LEAF;
        age[n] = 0;
    }
}

// sampling sums of the new leaves from the old ones
__global__ void amr_samp_kernel(TreeDims t, int32_t nleaf, const int32_t* __restrict__ leaf_node,
                                const int32_t* __restrict__ leafmap_old,
                                const int32_t* __restrict__ leaf_node_old,
                                const double* __restrict__ samp_old, const double* __restrict__ vol_old,
                                const double* __restrict__ vol, double* __restrict__ samp) {
    const int32_t id = (int32_t)(blockIdx.x * AMR_BLOCK + threadIdx.x);
    if (id >= nleaf) return;
    int l;
    int32_t ix, iy;
    node_xy(t, leaf_node[id], l, ix, iy);
    auto first_fine = [&](int ll, int32_t jx, int32_t jy) -> int64_t {
        const int ss = t.L - ll;
        return (int64_t)(jy << ss) * t.nxf + (jx << ss);
    };
    const int32_t o = leafmap_old[first_fine(l, ix, iy)];
    int lo;
    int32_t ox, oy;
    node_xy(t, leaf_node_old[o], lo, ox, oy);
    double* out = samp + (int64_t)id * SAMP;
    const double* so = samp_old + (int64_t)o * SAMP;
    if (lo == l) {
        for (int k = 0; k < SAMP; ++k) out[k] = so[k];
    } else if (lo < l) {
        const double r = vol[id] / vol_old[o];
        for (int k = 0; k < 13; ++k) out[k] = so[k] * r;
        for (int k = 13; k < SAMP; ++k) out[k] = so[k];
    } else {
        double acc[SAMP];
        for (int k = 0; k < SAMP; ++k) acc[k] = so[k];
        for (int c = 1; c < 4; ++c) {
            const int32_t k2 = leafmap_old[first_fine(l + 1, 2 * ix + (c & 1), 2 * iy + (c >> 1))];
            const double* sk = samp_old + (int64_t)k2 * SAMP;
            for (int k = 0; k < 13; ++k) acc[k] = acc[k] + sk[k];
        }
        for (int k = 0; k < SAMP; ++k) out[k] = acc[k];
    }
}

__global__ void amr_zero_kernel(int64_t n, double* __restrict__ a) {
    const int64_t i = (int64_t)blockIdx.x * AMR_BLOCK + threadIdx.x;
    if (i < n) a[i] = 0.0;
}

__global__ void amr_zero8_kernel(int64_t n, int8_t* __restrict__ a) {
    const int64_t i = (int64_t)blockIdx.x * AMR_BLOCK + threadIdx.x;
    if (i < n) a[i] = 0;
}

// keys of the particles under the new tree; keys outside [0, old_ncell) (deleted or
// unused slots) become new_ncell
template <typename T>
__global__ void amr_rekey_kernel(fp_config g, int64_t n, const int64_t* __restrict__ n_dev,
                                 const T* __restrict__ px, const T* __restrict__ py,
                                 int32_t* __restrict__ key, int32_t old_ncell, int32_t new_ncell,
                                 const int32_t* __restrict__ leafmap) {
    if (n_dev) n = *n_dev;
    const int64_t p = (int64_t)blockIdx.x * AMR_BLOCK + threadIdx.x;
    if (p >= n) return;
    const int32_t k = key[p];
    if (k < 0 || k >= old_ncell) {
        key[p] = new_ncell;
        return;
    }
    const int32_t kx = axis_cell((double)px[p], g.x0, 1.0 / g.dx, g.nx);
    const int32_t ky = axis_cell((double)py[p], g.y0, 1.0 / g.dy, g.ny);
    key[p] = leafmap[ky * g.nx + kx];
}

static inline int blocks(int64_t n) { return (int)((n + AMR_BLOCK - 1) / AMR_BLOCK); }

static TreeDims dims(const fp_ctx* c) {
    TreeDims t{};
    t.L = c->amr_L;
    t.nbx = c->amr_nbx;
    t.nby = c->amr_nby;
    t.nxf = c->cfg.nx;
    int64_t o = 0;
    for (int l = 0; l <= t.L; ++l) {
        t.off[l] = o;
        o += ((int64_t)t.nbx << l) * ((int64_t)t.nby << l);
    }
    t.off[t.L + 1] = o;
    return t;
}

// numbering, map and volumes of the current tree; sets c->ncell (synchronous)
static int renumber(fp_ctx* c, hipStream_t s) {
    const TreeDims t = dims(c);
    const int64_t nfine = (int64_t)c->cfg.nx * c->cfg.ny;
    hipLaunchKernelGGL(amr_first_kernel, dim3(blocks(nfine)), dim3(AMR_BLOCK), 0, s, t,
                       (const int8_t*)c->amr_state, c->amr_first);
    const int32_t ntiles = (int32_t)((nfine + ASCAN_TILE - 1) / ASCAN_TILE);
    hipLaunchKernelGGL(amr_scan_tiles_kernel, dim3(ntiles), dim3(AMR_BLOCK), 0, s, nfine, c->amr_first,
                       c->amr_part);
    hipLaunchKernelGGL(amr_scan_parts_kernel, dim3(1), dim3(AMR_BLOCK), 0, s, ntiles, c->amr_part);
    hipLaunchKernelGGL(amr_scan_add_kernel, dim3(blocks(nfine)), dim3(AMR_BLOCK), 0, s, nfine,
                       c->amr_first, (const int32_t*)c->amr_part);
    hipLaunchKernelGGL(amr_map_kernel, dim3(blocks(nfine)), dim3(AMR_BLOCK), 0, s, t,
                       (const int8_t*)c->amr_state, (const int32_t*)c->amr_first, c->leafmap,
                       c->leaf_node);
    int32_t nleaf = 0;
    if (hipMemcpyAsync(&nleaf, c->amr_first + nfine, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return set_err(c, FP_EDEVICE, "fp_amr: leaf count read-back failed");
    if (nleaf < 1 || nleaf > nfine) return set_err(c, FP_EDEVICE, "fp_amr: invalid tree");
    const double full_fine = c->cfg.dx * c->cfg.dy * c->cfg.depth;
    hipLaunchKernelGGL(amr_vol_kernel, dim3(blocks(nleaf)), dim3(AMR_BLOCK), 0, s, t, nleaf,
                       (const int32_t*)c->leaf_node, (const double*)c->fine_vol, c->cfg.fnum,
                       full_fine, c->vol, c->nvol);
    c->ncell = nleaf;
    return check_launch(c, "fp_amr");
}

}  // namespace fpg

using namespace fpg;

extern "C" int fp_amr_init(fp_ctx* c, int32_t max_level) {
    if (!c) return FP_EINVAL;
    if (c->cfg.geometry != FP_CYLINDER2D)
        return set_err(c, FP_EINVAL, "fp_amr_init: the adaptive tree needs the cylinder domain");
    if (c->amr_L >= 0) return set_err(c, FP_EINVAL, "fp_amr_init: the context already has a tree");
    if (max_level < 0 || max_level > AMR_MAX_LEVEL)
        return set_err(c, FP_EINVAL, "fp_amr_init: max_level outside [0, 4]");
    const int32_t m = 1 << max_level;
    if (c->cfg.nx % m != 0 || c->cfg.ny % m != 0)
        return set_err(c, FP_EINVAL, "fp_amr_init: nx and ny must be multiples of 2^max_level");
    c->amr_L = max_level;
    ++c->amr_epoch;
    c->amr_nbx = c->cfg.nx / m;
    c->amr_nby = c->cfg.ny / m;
    const TreeDims t = dims(c);
    const int64_t nodes = t.off[t.L + 1];
    const int64_t nfine = (int64_t)c->cfg.nx * c->cfg.ny;
    const int64_t ntiles = (nfine + ASCAN_TILE - 1) / ASCAN_TILE;
    auto al = [](auto** p, size_t n) { return hipMalloc((void**)p, sizeof(**p) * (n ? n : 1)) == hipSuccess; };
    bool ok = al(&c->amr_state, nodes) && al(&c->amr_flag, nodes) && al(&c->amr_age, nodes) &&
              al(&c->amr_sum, nodes * SUMW) && al(&c->leafmap, nfine) && al(&c->leafmap_old, nfine) &&
              al(&c->leaf_node, nfine) && al(&c->leaf_node_old, nfine) && al(&c->amr_first, nfine + 1) &&
              al(&c->amr_part, ntiles + 1) && al(&c->fine_vol, nfine) && al(&c->vol_old, nfine) &&
              al(&c->samp_old, nfine * SAMP);
    if (!ok) {
        c->amr_L = -1;
        return set_err(c, FP_ENOMEM, "fp_amr_init: allocation failed");
    }
    hipStream_t s = 0;
    // the context's cell volumes are those of the fine grid until now
    if (hipMemcpyAsync(c->fine_vol, c->vol, sizeof(double) * nfine, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return set_err(c, FP_EDEVICE, "fp_amr_init: copy failed");
    hipLaunchKernelGGL(amr_init_kernel, dim3(blocks(nodes)), dim3(AMR_BLOCK), 0, s, nodes,
                       (int64_t)c->amr_nbx * c->amr_nby, c->amr_state, c->amr_age);
    hipLaunchKernelGGL(amr_zero8_kernel, dim3(blocks(nodes)), dim3(AMR_BLOCK), 0, s, nodes, c->amr_flag);
    const int rc = renumber(c, s);
    if (rc != FP_OK) return rc;
    return hipStreamSynchronize(s) == hipSuccess ? FP_OK : set_err(c, FP_EDEVICE, "fp_amr_init: sync failed");
}

extern "C" int fp_amr_adapt(fp_ctx* c, const fp_amr_params* prm, double* acc, double* samp,
                            fp_particles* p, int32_t steps, hipStream_t s) {
    if (!c || !prm || !acc || steps < 0 || prm->reserved != 0)
        return set_err(c, FP_EINVAL, "fp_amr_adapt: bad argument");
    if (c->amr_L < 0) return set_err(c, FP_EINVAL, "fp_amr_adapt: no tree (fp_amr_init)");
    if (p && (!p->x || !p->y || !p->key || p->n < 0 || p->n > c->cfg.capacity ||
              (p->n_dev && (p->capacity < p->n || p->capacity > c->cfg.capacity))))
        return set_err(c, FP_EINVAL, "fp_amr_adapt: bad particles");
    const TreeDims t = dims(c);
    const int64_t nodes = t.off[t.L + 1];
    const int64_t nfine = (int64_t)c->cfg.nx * c->cfg.ny;
    const int32_t old_ncell = c->ncell;
    ++c->amr_epoch;   // the leaves are renumbered: the next sort must be a full fp_bin
    const double fnum = c->cfg.fnum, mass = c->cfg.mass;
    // decisions on the tree as it is
    hipLaunchKernelGGL(amr_zero8_kernel, dim3(blocks(nodes)), dim3(AMR_BLOCK), 0, s, nodes, c->amr_flag);
    hipLaunchKernelGGL(amr_leaf_sum_kernel, dim3(blocks(old_ncell)), dim3(AMR_BLOCK), 0, s, old_ncell,
                       (const int32_t*)c->leaf_node, (const double*)acc, (const double*)c->vol, c->amr_sum);
    for (int l = t.L - 1; l >= 0; --l) {
        const int64_t cnt = ((int64_t)t.nbx << l) * ((int64_t)t.nby << l);
        hipLaunchKernelGGL(amr_up_kernel, dim3(blocks(cnt)), dim3(AMR_BLOCK), 0, s, t, l,
                           (const int8_t*)c->amr_state, c->amr_sum);
    }
    hipLaunchKernelGGL(amr_split_kernel, dim3(blocks(old_ncell)), dim3(AMR_BLOCK), 0, s, t, old_ncell,
                       (const int32_t*)c->leaf_node, (const double*)c->amr_sum, *prm, fnum, mass,
                       c->amr_flag);
    for (int l = 0; l < t.L; ++l) {
        const int64_t cnt = ((int64_t)t.nbx << l) * ((int64_t)t.nby << l);
        hipLaunchKernelGGL(amr_merge_kernel, dim3(blocks(cnt)), dim3(AMR_BLOCK), 0, s, t, l,
                           (const int8_t*)c->amr_state, (const int32_t*)c->amr_age,
                           (const double*)c->amr_sum, *prm, fnum, mass, c->amr_flag);
    }
    // keep the old numbering for the sums and keys, then the new tree
    bool ok = hipMemcpyAsync(c->leafmap_old, c->leafmap, sizeof(int32_t) * nfine, hipMemcpyDeviceToDevice, s) == hipSuccess &&
              hipMemcpyAsync(c->leaf_node_old, c->leaf_node, sizeof(int32_t) * old_ncell, hipMemcpyDeviceToDevice, s) == hipSuccess &&
              hipMemcpyAsync(c->vol_old, c->vol, sizeof(double) * old_ncell, hipMemcpyDeviceToDevice, s) == hipSuccess;
    if (ok && samp)
        ok = hipMemcpyAsync(c->samp_old, samp, sizeof(double) * SAMP * (size_t)old_ncell, hipMemcpyDeviceToDevice, s) == hipSuccess;
    if (!ok) return set_err(c, FP_EDEVICE, "fp_amr_adapt: copy failed");
    hipLaunchKernelGGL(amr_apply_kernel, dim3(blocks(nodes)), dim3(AMR_BLOCK), 0, s, t, steps, c->amr_state,
                       c->amr_age, (const int8_t*)c->amr_flag);
    const int rc = renumber(c, s);
    if (rc != FP_OK) return rc;
    const int32_t nleaf = c->ncell;
    if (samp)
        hipLaunchKernelGGL(amr_samp_kernel, dim3(blocks(nleaf)), dim3(AMR_BLOCK), 0, s, t, nleaf,
                           (const int32_t*)c->leaf_node, (const int32_t*)c->leafmap_old,
                           (const int32_t*)c->leaf_node_old, (const double*)c->samp_old,
                           (const double*)c->vol_old, (const double*)c->vol, samp);
    hipLaunchKernelGGL(amr_zero_kernel, dim3(blocks((int64_t)nleaf * SAMP)), dim3(AMR_BLOCK), 0, s,
                       (int64_t)nleaf * SAMP, acc);
    if (p && slots_of(p) > 0) {
        if (c->cfg.precision == FP_F32)
            hipLaunchKernelGGL(amr_rekey_kernel<float>, dim3(blocks(slots_of(p))), dim3(AMR_BLOCK), 0, s,
                               c->cfg, p->n, (const int64_t*)p->n_dev, (const float*)p->x, (const float*)p->y, p->key, old_ncell, nleaf,
                               (const int32_t*)c->leafmap);
        else
            hipLaunchKernelGGL(amr_rekey_kernel<double>, dim3(blocks(slots_of(p))), dim3(AMR_BLOCK), 0, s,
                               c->cfg, p->n, (const int64_t*)p->n_dev, (const double*)p->x, (const double*)p->y, p->key, old_ncell, nleaf,
                               (const int32_t*)c->leafmap);
    }
    return check_launch(c, "fp_amr_adapt");
}

extern "C" int32_t fp_ncell(const fp_ctx* c) { return c ? c->ncell : -1; }

extern "C" int64_t fp_amr_nodes(const fp_ctx* c) {
    if (!c || c->amr_L < 0) return 0;
    return dims(c).off[c->amr_L + 1];
}

extern "C" int fp_amr_tree(fp_ctx* c, int8_t* state, int32_t* age, int32_t* leafmap,
                           int32_t* leaf_node, hipStream_t s) {
    if (!c || c->amr_L < 0) return set_err(c, FP_EINVAL, "fp_amr_tree: no tree");
    const int64_t nodes = fp_amr_nodes(c), nfine = (int64_t)c->cfg.nx * c->cfg.ny;
    bool ok = true;
    if (state) ok = ok && hipMemcpyAsync(state, c->amr_state, nodes, hipMemcpyDeviceToDevice, s) == hipSuccess;
    if (age) ok = ok && hipMemcpyAsync(age, c->amr_age, sizeof(int32_t) * nodes, hipMemcpyDeviceToDevice, s) == hipSuccess;
    if (leafmap) ok = ok && hipMemcpyAsync(leafmap, c->leafmap, sizeof(int32_t) * nfine, hipMemcpyDeviceToDevice, s) == hipSuccess;
    if (leaf_node)
        ok = ok && hipMemcpyAsync(leaf_node, c->leaf_node, sizeof(int32_t) * c->ncell, hipMemcpyDeviceToDevice, s) == hipSuccess;
    return ok ? FP_OK : set_err(c, FP_EDEVICE, "fp_amr_tree: copy failed");
}
