// fp_step.hip -- velocity update with per-cell conservation, free flight, diffuse walls.
//
// Collision (G lanes per cell): for every particle, c = v - U,
//   N  = Ct c + G (|c|^2 - 3 theta) - eps2 (c |c|^2 - S)            (eq. update_N)
//   c* = c E + (1 - E) tau N + sigma xi,  xi ~ N(0, I) from Philox    (eq. update_vel)
// then the cell is recentred on U and its energy restored, exactly (EXACT) or with the
// factor alpha of eq. update_alpha (PAPER).  c* of up to K particles per lane stays in
// registers between the sum pass and the write pass; beyond that it waits in the
// particle's own velocity slots.  Per-particle arithmetic is in the storage
// precision; the cell sums and the rescale factor are FP64.
// Flight (eq. update_pos) and the wall interactions are FP64 without contraction, so a
// stored position and the wall decisions are the same numbers on any IEEE machine.
#include "fp_internal.h"

namespace fpg {

constexpr int ST_BLOCK = 256;
constexpr int ST_K = 2;   // register-cached particles per lane in collide_kernel

struct Walls {
    double lo[2], hi[2];
    double RT[4];   // R T_w per wall
    double sRT[4];  // sqrt(R T_w)
};

__device__ __forceinline__ double st_round(double v, bool f32) {
    return f32 ? (double)__double2float_rn(v) : v;
}

// diffuse re-emission from wall w (0: x lo, 1: x hi, 2: y lo, 3: y hi): inward normal
// speed with density ~ v exp(-v^2/(2 R T_w)), Gaussian tangential velocity about u_w
// value of wall w among four, by selects (a dynamic index would put the array in scratch)
__device__ __forceinline__ double pick4(int w, double a0, double a1, double a2, double a3) {
    return w == 0 ? a0 : (w == 1 ? a1 : (w == 2 ? a2 : a3));
}

__device__ __forceinline__ void wall_emit(const fp_config& g, const Walls& W, int w,
                                          uint32_t pid, uint32_t step, uint32_t bounce,
                                          double v[3]) {
    const uint4 r = draw(g.seed, pid, step, PURPOSE_WALL, bounce);
    const double u0 = u01d(r.x), u1 = u01d(r.y), u2 = u01d(r.z);
    const double RT = pick4(w, W.RT[0], W.RT[1], W.RT[2], W.RT[3]);
    const double vn = sqrt(-2.0 * RT * log(u0));
    const double rr = sqrt(-2.0 * log(u1));
    const double za = rr * cos(TWO_PI * u2);
    const double zb = rr * sin(TWO_PI * u2);
    const double s = pick4(w, W.sRT[0], W.sRT[1], W.sRT[2], W.sRT[3]);
    const double uw0 = pick4(w, g.u_wall[0][0], g.u_wall[1][0], g.u_wall[2][0], g.u_wall[3][0]);
    const double uw1 = pick4(w, g.u_wall[0][1], g.u_wall[1][1], g.u_wall[2][1], g.u_wall[3][1]);
    const double uw2 = pick4(w, g.u_wall[0][2], g.u_wall[1][2], g.u_wall[2][2], g.u_wall[3][2]);
    if (w < 2) {
        v[0] = (w == 0) ? vn : -vn;
        v[1] = uw1 + s * za;
        v[2] = uw2 + s * zb;
    } else {
        v[1] = (w == 2) ? vn : -vn;
        v[0] = uw0 + s * za;
        v[2] = uw2 + s * zb;
    }
}

// free flight over dt with wall interactions; pos/v updated in place (FP64)
template <bool TWO_D>
__device__ __forceinline__ void fly(const fp_config& g, const Walls& W, double pos[2],
                                    double v[3], uint32_t pid, uint32_t step, bool f32) {
    double trem = g.dt;
    for (int bounce = 0;; ++bounce) {
        const double ex = __dadd_rn(pos[0], __dmul_rn(v[0], trem));
        const double ey = TWO_D ? __dadd_rn(pos[1], __dmul_rn(v[1], trem)) : 0.0;
        int wall = -1;
        double th = 0.0;
        if (ex < W.lo[0] && v[0] < 0.0) {
            double t = __ddiv_rn(__dsub_rn(W.lo[0], pos[0]), v[0]);
            t = t < 0.0 ? 0.0 : t;
            wall = 0;
            th = t;
        }
        if (ex > W.hi[0] && v[0] > 0.0) {
            double t = __ddiv_rn(__dsub_rn(W.hi[0], pos[0]), v[0]);
            t = t < 0.0 ? 0.0 : t;
            if (wall < 0 || t < th) { wall = 1; th = t; }
        }
        if (TWO_D) {
            if (ey < W.lo[1] && v[1] < 0.0) {
                double t = __ddiv_rn(__dsub_rn(W.lo[1], pos[1]), v[1]);
                t = t < 0.0 ? 0.0 : t;
                if (wall < 0 || t < th) { wall = 2; th = t; }
            }
            if (ey > W.hi[1] && v[1] > 0.0) {
                double t = __ddiv_rn(__dsub_rn(W.hi[1], pos[1]), v[1]);
                t = t < 0.0 ? 0.0 : t;
                if (wall < 0 || t < th) { wall = 3; th = t; }
            }
        }
        if (wall < 0) {
            pos[0] = ex;
            if (TWO_D) pos[1] = ey;
            break;
        }
        if (bounce == g.max_bounces) {
            pos[0] = fmin(fmax(ex, W.lo[0]), W.hi[0]);
            if (TWO_D) pos[1] = fmin(fmax(ey, W.lo[1]), W.hi[1]);
            break;
        }
        th = th > trem ? trem : th;
        if (wall < 2) {
            pos[0] = wall == 0 ? W.lo[0] : W.hi[0];
            if (TWO_D) pos[1] = __dadd_rn(pos[1], __dmul_rn(v[1], th));
        } else {
            pos[0] = __dadd_rn(pos[0], __dmul_rn(v[0], th));
            pos[1] = wall == 2 ? W.lo[1] : W.hi[1];
        }
        wall_emit(g, W, wall, pid, step, (uint32_t)bounce, v);
        v[0] = st_round(v[0], f32);
        v[1] = st_round(v[1], f32);
        v[2] = st_round(v[2], f32);
        trem = __dsub_rn(trem, th);
    }
    pos[0] = st_round(pos[0], f32);
    if (TWO_D) pos[1] = st_round(pos[1], f32);
}

// diffuse re-emission from the cylinder surface at (px, py): normal n = (p - c)/R into the
// gas, speed along n ~ v exp(-v^2/(2 R T_body)), Gaussian along the tangent (-n_y, n_x)
// and along z; the body is at rest
__device__ __forceinline__ void circle_emit(const fp_config& g, double px, double py, uint32_t pid,
                                            uint32_t step, uint32_t bounce, double v[3]) {
    const uint4 r = draw(g.seed, pid, step, PURPOSE_WALL, bounce);
    const double u0 = u01d(r.x), u1 = u01d(r.y), u2 = u01d(r.z);
    const double RT = g.kB / g.mass * g.T_body;
    const double vn = sqrt(-2.0 * RT * log(u0));
    const double rr = sqrt(-2.0 * log(u1));
    const double za = rr * cos(TWO_PI * u2);
    const double zb = rr * sin(TWO_PI * u2);
    const double s = sqrt(RT);
    const double nx = (px - g.circle[0]) / g.circle[2];
    const double ny = (py - g.circle[1]) / g.circle[2];
    const double vt = s * za;
    v[0] = vn * nx - vt * ny;
    v[1] = vn * ny + vt * nx;
    v[2] = s * zb;
}

// exchange of one re-emission at the body, per unit molecular mass, into the bin of the
// surface angle theta (0 at the rear point, pi at the front) with cos theta = n_x: bin b
// holds edge[b + 1] < n_x <= edge[b], edge[k] = cos(k pi / nbins) (host cosines, found by
// bisection): hits, normal momentum v_out.n - v_in.n, tangential momentum towards the
// rear (v_in - v_out).t (t the unit tangent along decreasing theta), energy
// (|v_in|^2 - |v_out|^2) / 2
__device__ __forceinline__ void wall_record(const fp_config& g, double px, double py, const double vin[3],
                                            const double vout[3], double* __restrict__ wall,
                                            const double* __restrict__ edge, int32_t nbins) {
    const double nx = (px - g.circle[0]) / g.circle[2];
    const double ny = (py - g.circle[1]) / g.circle[2];
    int32_t lo = 0, hi = nbins;   // nx <= edge[lo] (edge[0] = 1), nx > edge[hi] unless hi = nbins
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (nx <= edge[mid]) lo = mid;
        else hi = mid;
    }
    const double sg = ny >= 0.0 ? 1.0 : -1.0;
    const double tx = sg * ny, ty = -sg * nx;
    double* w = wall + 4 * (int64_t)lo;
    unsafeAtomicAdd(w, 1.0);
    unsafeAtomicAdd(w + 1, (vout[0] * nx + vout[1] * ny) - (vin[0] * nx + vin[1] * ny));
    unsafeAtomicAdd(w + 2, (vin[0] * tx + vin[1] * ty) - (vout[0] * tx + vout[1] * ty));
    unsafeAtomicAdd(w + 3, 0.5 * ((vin[0] * vin[0] + vin[1] * vin[1] + vin[2] * vin[2]) -
                                  (vout[0] * vout[0] + vout[1] * vout[1] + vout[2] * vout[2])));
}

// free flight in the open cylinder domain: straight segments between diffuse hits on the
// circle; returns true if the particle ends outside the box (deleted).  wall (optional):
// exchange sums of the re-emissions, nbins bins of the surface angle
template <bool REC = false>
__device__ __forceinline__ bool fly_open(const fp_config& g, double pos[2], double v[3],
                                         uint32_t pid, uint32_t step, bool f32,
                                         double* __restrict__ wall = nullptr,
                                         const double* __restrict__ edge = nullptr, int32_t nbins = 0) {
    const double cx = g.circle[0], cy = g.circle[1], R = g.circle[2];
    double trem = g.dt;
    for (int bounce = 0;; ++bounce) {
        const double dxc = pos[0] - cx, dyc = pos[1] - cy;
        const double a = v[0] * v[0] + v[1] * v[1];
        const double b = dxc * v[0] + dyc * v[1];
        const double c = dxc * dxc + dyc * dyc - R * R;
        bool hit = false;
        double th = 0.0;
        if (c < 0.0) {
            if (b < 0.0) {   // inside by rounding and moving in: hit at once
                const double d = sqrt(dxc * dxc + dyc * dyc);
                if (d > 0.0) {
                    pos[0] = cx + R * (dxc / d);
                    pos[1] = cy + R * (dyc / d);
                }
                hit = true;
            }
        } else if (b < 0.0 && a > 0.0) {
            const double disc = b * b - a * c;
            if (disc >= 0.0) {
                const double q = -b + sqrt(disc);
                const double t = c / q;
                if (t <= trem) {
                    hit = true;
                    th = t;
                    pos[0] = pos[0] + v[0] * th;
                    pos[1] = pos[1] + v[1] * th;
                }
            }
        }
        if (!hit) {
            pos[0] = pos[0] + v[0] * trem;
            pos[1] = pos[1] + v[1] * trem;
            break;
        }
        if (bounce == g.max_bounces) return false;   // stop on the surface
        [[maybe_unused]] const double vin[3] = {v[0], v[1], v[2]};
        circle_emit(g, pos[0], pos[1], pid, step, (uint32_t)bounce, v);
        v[0] = st_round(v[0], f32);
        v[1] = st_round(v[1], f32);
        v[2] = st_round(v[2], f32);
        if constexpr (REC) wall_record(g, pos[0], pos[1], vin, v, wall, edge, nbins);
        trem = trem - th;
    }
    const double x1 = g.x0 + g.lx, y1 = g.y0 + g.ly;
    return pos[0] < g.x0 || pos[0] > x1 || pos[1] < g.y0 || pos[1] > y1;
}

// kmap (adaptive tree): the leaf of every cell of the grid, else NULL
template <bool TWO_D>
__device__ __forceinline__ int32_t cell_key(const fp_config& g, double x, double y, double inv_dx,
                                            double inv_dy, const int32_t* __restrict__ kmap) {
    const int32_t kx = axis_cell(x, g.x0, inv_dx, g.nx);
    const int32_t ky = TWO_D ? axis_cell(y, g.y0, inv_dy, g.ny) : 0;
    const int32_t k = ky * g.nx + kx;
    return kmap ? kmap[k] : k;
}

__host__ __device__ inline Walls make_walls(const fp_config& g) {
    Walls W;
    W.lo[0] = g.x0;
    W.lo[1] = g.y0;
    W.hi[0] = g.x0 + g.lx;
    W.hi[1] = g.y0 + g.ly;
    for (int w = 0; w < 4; ++w) {
        W.RT[w] = g.kB / g.mass * g.T_wall[w];
        W.sRT[w] = sqrt(W.RT[w]);
    }
    return W;
}

// ---- per-particle collision arithmetic in the storage precision -----------------------
template <typename T>
struct CellCoef {
    T U[3], C[6], G[3], S[3], th3, E, k1, sig, eps2;
};

template <typename T>
__device__ __forceinline__ void collide_one(const CellCoef<T>& q, T v0, T v1, T v2, uint4 r,
                                            T cs[3], T& nn, T& cn);

template <>
__device__ __forceinline__ void collide_one<float>(const CellCoef<float>& q, float v0, float v1,
                                                   float v2, uint4 r, float cs[3], float& nn,
                                                   float& cn) {
    const float c0 = v0 - q.U[0], c1 = v1 - q.U[1], c2 = v2 - q.U[2];
    const float cc = __builtin_fmaf(c0, c0, __builtin_fmaf(c1, c1, c2 * c2));
    const float a = cc - q.th3;
    const float N0 = __builtin_fmaf(q.C[0], c0, __builtin_fmaf(q.C[1], c1, __builtin_fmaf(q.C[2], c2,
                     __builtin_fmaf(q.G[0], a, -q.eps2 * __builtin_fmaf(c0, cc, -q.S[0])))));
    const float N1 = __builtin_fmaf(q.C[1], c0, __builtin_fmaf(q.C[3], c1, __builtin_fmaf(q.C[4], c2,
                     __builtin_fmaf(q.G[1], a, -q.eps2 * __builtin_fmaf(c1, cc, -q.S[1])))));
    const float N2 = __builtin_fmaf(q.C[2], c0, __builtin_fmaf(q.C[4], c1, __builtin_fmaf(q.C[5], c2,
                     __builtin_fmaf(q.G[2], a, -q.eps2 * __builtin_fmaf(c2, cc, -q.S[2])))));
    float z0, z1, z2;
    normals3f(r, z0, z1, z2);
    cs[0] = __builtin_fmaf(c0, q.E, __builtin_fmaf(q.k1, N0, q.sig * z0));
    cs[1] = __builtin_fmaf(c1, q.E, __builtin_fmaf(q.k1, N1, q.sig * z1));
    cs[2] = __builtin_fmaf(c2, q.E, __builtin_fmaf(q.k1, N2, q.sig * z2));
    nn = __builtin_fmaf(N0, N0, __builtin_fmaf(N1, N1, N2 * N2));
    cn = __builtin_fmaf(c0, N0, __builtin_fmaf(c1, N1, c2 * N2));
}

template <>
__device__ __forceinline__ void collide_one<double>(const CellCoef<double>& q, double v0,
                                                    double v1, double v2, uint4 r, double cs[3],
                                                    double& nn, double& cn) {
    const double c0 = v0 - q.U[0], c1 = v1 - q.U[1], c2 = v2 - q.U[2];
    const double cc = fma(c0, c0, fma(c1, c1, c2 * c2));
    const double a = cc - q.th3;
    const double N0 = fma(q.C[0], c0, fma(q.C[1], c1, fma(q.C[2], c2,
                      fma(q.G[0], a, -q.eps2 * fma(c0, cc, -q.S[0])))));
    const double N1 = fma(q.C[1], c0, fma(q.C[3], c1, fma(q.C[4], c2,
                      fma(q.G[1], a, -q.eps2 * fma(c1, cc, -q.S[1])))));
    const double N2 = fma(q.C[2], c0, fma(q.C[4], c1, fma(q.C[5], c2,
                      fma(q.G[2], a, -q.eps2 * fma(c2, cc, -q.S[2])))));
    double z0, z1, z2;
    normals3d(r, z0, z1, z2);
    cs[0] = fma(c0, q.E, fma(q.k1, N0, q.sig * z0));
    cs[1] = fma(c1, q.E, fma(q.k1, N1, q.sig * z1));
    cs[2] = fma(c2, q.E, fma(q.k1, N2, q.sig * z2));
    nn = fma(N0, N0, fma(N1, N1, N2 * N2));
    cn = fma(c0, N0, fma(c1, N1, c2 * N2));
}

template <typename T, int G, int K, int GEOM>
__global__ __launch_bounds__(ST_BLOCK) void collide_kernel(
    fp_config g, int32_t ncell, const int32_t* __restrict__ offsets,
    const double* __restrict__ mom, const double* __restrict__ rec, T* __restrict__ px,
    T* __restrict__ py, T* __restrict__ pvx, T* __restrict__ pvy, T* __restrict__ pvz,
    const uint32_t* __restrict__ ppid, int32_t* __restrict__ pkey, uint32_t step_arg, int move,
    const uint32_t* __restrict__ stepp, int32_t* __restrict__ pend, int32_t* __restrict__ plist,
    uint32_t* __restrict__ stepc, const int32_t* __restrict__ kmap) {
    const uint32_t step = stepp ? stepp[0] : step_arg;
    if (stepc && blockIdx.x == 0 && threadIdx.x == 0) stepc[0] = step;   // for flight_rest
    const int64_t gt = (int64_t)blockIdx.x * ST_BLOCK + threadIdx.x;
    // with a whole wave per cell the cell is wave-uniform: its coefficients load into
    // scalar registers
    const int32_t cell = G == 64 ? __builtin_amdgcn_readfirstlane((int32_t)(gt / G)) : (int32_t)(gt / G);
    const int lg = (int)(gt % G);
    const bool in = cell < ncell;
    const bool f32 = sizeof(T) == 4;
    int32_t b = 0, n = 0;
    bool active = false;
    CellCoef<T> q;
    double Ud[3] = {0, 0, 0}, theta = 0, tau = 0, E = 1;
    if (in) {
        b = offsets[cell];
        n = offsets[cell + 1] - b;
        const double* r = rec + (int64_t)cell * REC;
        const int st = (int)r[R_ST];
        active = n > 0 && st != FP_CELL_EMPTY && st != FP_CELL_NONFINITE;
        if (active) {
            const double* m = mom + (int64_t)cell * MOM;
            Ud[0] = m[M_U]; Ud[1] = m[M_U + 1]; Ud[2] = m[M_U + 2];
            tau = r[R_TAU]; theta = r[R_TH]; E = r[R_E];
            for (int i = 0; i < 3; ++i) q.U[i] = (T)Ud[i];
            for (int i = 0; i < 6; ++i) q.C[i] = (T)r[R_C + i];
            for (int i = 0; i < 3; ++i) q.G[i] = (T)r[R_G + i];
            q.S[0] = (T)(m[M_T + 0] + m[M_T + 3] + m[M_T + 5]);
            q.S[1] = (T)(m[M_T + 1] + m[M_T + 6] + m[M_T + 8]);
            q.S[2] = (T)(m[M_T + 2] + m[M_T + 7] + m[M_T + 9]);
            q.th3 = (T)(3.0 * theta);
            q.E = (T)E;
            q.k1 = (T)((1.0 - E) * tau);
            q.sig = (T)r[R_SIG];
            q.eps2 = (T)r[R_EPS2];
        }
    }
    const int32_t na = active ? n : 0;
    constexpr bool TWO_D = GEOM != FP_COUETTE1D;

    // pass A: c* and cell sums; the positions of the register-cached particles are loaded
    // here too, so that pass B, after the group sums, does not wait for them
    T cs0[K], cs1[K], cs2[K], xk[K], yk[K];
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0, s4 = 0;
    const bool exact = g.conserve == FP_EXACT;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int32_t j = lg + k * G;
        if (j < na) {
            const int32_t p = b + j;
            if (move) {
                xk[k] = px[p];
                yk[k] = TWO_D ? py[p] : (T)0;
            }
            T cs[3], nn, cn;
            collide_one<T>(q, pvx[p], pvy[p], pvz[p], draw(g.seed, ppid[p], step, PURPOSE_COLLISION, 0),
                           cs, nn, cn);
            cs0[k] = cs[0]; cs1[k] = cs[1]; cs2[k] = cs[2];
            const double d0 = cs[0], d1 = cs[1], d2 = cs[2];
            s0 += d0; s1 += d1; s2 += d2;
            if (exact) s3 = fma(d0, d0, fma(d1, d1, fma(d2, d2, s3)));
            else { s3 += (double)nn; s4 += (double)cn; }
        }
    }
    // beyond the register cache, c* waits in the velocity arrays (same lane, same slot)
    for (int32_t j = lg + K * G; j < na; j += G) {
        const int32_t p = b + j;
        T cs[3], nn, cn;
        collide_one<T>(q, pvx[p], pvy[p], pvz[p], draw(g.seed, ppid[p], step, PURPOSE_COLLISION, 0),
                       cs, nn, cn);
        pvx[p] = cs[0]; pvy[p] = cs[1]; pvz[p] = cs[2];
        const double d0 = cs[0], d1 = cs[1], d2 = cs[2];
        s0 += d0; s1 += d1; s2 += d2;
        if (exact) s3 = fma(d0, d0, fma(d1, d1, fma(d2, d2, s3)));
        else { s3 += (double)nn; s4 += (double)cn; }
    }
    s0 = group_sum<G>(s0);
    s1 = group_sum<G>(s1);
    s2 = group_sum<G>(s2);
    s3 = group_sum<G>(s3);
    s4 = group_sum<G>(s4);

    T cb[3] = {0, 0, 0}, sc = 1;
    if (active) {
        const double in_ = 1.0 / (double)n;
        const double c0 = s0 * in_, c1 = s1 * in_, c2 = s2 * in_;
        double scale;
        if (exact) {
            const double e2 = s3 * in_ - (c0 * c0 + c1 * c1 + c2 * c2);
            scale = sqrt(3.0 * theta / e2);
        } else {
            const double a2 = 1.0 + tau / (3.0 * theta) *
                                        (tau * (1.0 - E) * (1.0 - E) * (s3 * in_) +
                                         2.0 * (E - E * E) * (s4 * in_));
            scale = 1.0 / sqrt(a2);
        }
        if (!isfinite(scale) || !(scale > 0.0)) scale = 1.0;
        cb[0] = (T)c0; cb[1] = (T)c1; cb[2] = (T)c2;
        sc = (T)scale;
    }

    // pass B: final velocity, then flight and key.  The common flight (straight, no wall
    // or body in reach) is decided here; a particle that may meet a wall or the body gets
    // its new velocity stored and takes the full flight in flight_rest_kernel, which keeps
    // the FP64 re-emission code (and its registers) out of this kernel.
    const Walls W = make_walls(g);
    const double inv_dx = 1.0 / g.dx, inv_dy = 1.0 / g.dy;
    auto store_done = [&](int32_t p, double x, double y, T v0, T v1, T v2, bool gone) {
        px[p] = (T)x;
        if (TWO_D) py[p] = (T)y;
        pvx[p] = v0; pvy[p] = v1; pvz[p] = v2;
        pkey[p] = gone ? ncell : cell_key<TWO_D>(g, x, y, inv_dx, inv_dy, kmap);
    };
    // returns false when the full flight is still to do (velocity already stored)
    auto finish_fast = [&](int32_t p, T v0, T v1, T v2, T xo, T yo) -> bool {
        if (!move) {
            pvx[p] = v0; pvy[p] = v1; pvz[p] = v2;
            return true;
        }
        const double x0 = (double)xo, y0 = TWO_D ? (double)yo : 0.0;
        const double w0 = (double)v0, w1 = (double)v1;
        const double ex = __dadd_rn(x0, __dmul_rn(w0, g.dt));
        const double ey = TWO_D ? __dadd_rn(y0, __dmul_rn(w1, g.dt)) : 0.0;
        bool plain, gone = false;
        if constexpr (GEOM == FP_CYLINDER2D) {
            // no hit is possible when the body is out of reach by a wide margin
            const double dxc = x0 - g.circle[0], dyc = y0 - g.circle[1];
            const double reach = g.circle[2] + sqrt(w0 * w0 + w1 * w1) * g.dt;
            plain = dxc * dxc + dyc * dyc > reach * reach * (1.0 + 1e-6) + 1e-300;
            gone = ex < g.x0 || ex > g.x0 + g.lx || ey < g.y0 || ey > g.y0 + g.ly;
        } else {
            plain = !((ex < W.lo[0] && w0 < 0.0) || (ex > W.hi[0] && w0 > 0.0) ||
                      (TWO_D && ((ey < W.lo[1] && w1 < 0.0) || (ey > W.hi[1] && w1 > 0.0))));
        }
        if (!plain) {
            pvx[p] = v0; pvy[p] = v1; pvz[p] = v2;
            return false;
        }
        store_done(p, st_round(ex, f32), TWO_D ? st_round(ey, f32) : 0.0, v0, v1, v2, gone);
        return true;
    };
    auto newv = [&](T c, int i) -> T {
        return __builtin_fma(c - cb[i], sc, q.U[i]);
    };
    // a particle that may meet a wall or the body keeps its new velocity and its index
    // goes to the cell's list (plist[b ..], inside the cell's own range; a group ballot
    // gives each one a distinct place); flight_rest_kernel flies the listed particles
    const int lane = threadIdx.x & 63;
    const uint64_t gmask = G == 64 ? ~0ull : (((1ull << G) - 1ull) << (lane - lg));
    const uint64_t below = (1ull << lane) - 1ull;
    int32_t npend = 0;   // listed so far by the group (same in every lane still working)
    auto finish = [&](int32_t p, T v0, T v1, T v2, T xo, T yo) {
        const bool done = finish_fast(p, v0, v1, v2, xo, yo);
        const uint64_t m = __ballot(!done) & gmask;
        if (!done) plist[b + npend + __popcll(m & below)] = p;
        npend += __popcll(m);
    };
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int32_t j = lg + k * G;
        if (j < n) {
            const int32_t p = b + j;
            // the inactive cells' particles (na = 0) were not prefetched
            const T xo = !move ? (T)0 : (active ? xk[k] : px[p]);
            const T yo = !move || !TWO_D ? (T)0 : (active ? yk[k] : py[p]);
            if (active) finish(p, newv(cs0[k], 0), newv(cs1[k], 1), newv(cs2[k], 2), xo, yo);
            else finish(p, pvx[p], pvy[p], pvz[p], xo, yo);
        }
    }
    for (int32_t j = lg + K * G; j < n; j += G) {
        const int32_t p = b + j;
        const T xo = move ? px[p] : (T)0;
        const T yo = move && TWO_D ? py[p] : (T)0;
        if (active) finish(p, newv(pvx[p], 0), newv(pvy[p], 1), newv(pvz[p], 2), xo, yo);
        else finish(p, pvx[p], pvy[p], pvz[p], xo, yo);
    }
    if (move && in && lg == 0) pend[cell] = npend;   // lane 0 takes part in every round
}

// the flights collide_kernel left: the particles listed for cells with pend > 0 fly from
// their stored position with their stored (new) velocity, through walls / past the body.
// One wave per FR cells: it reads their list lengths at once and spreads the listed
// particles of all of them over its 64 lanes (only cells in reach of a wall or the body
// have any, so most waves end after one load).  The flights of the cells along a wall
// are the kernel's critical path: FR = 2 on small grids keeps them to one flight per
// lane (a wave per 64 cells serialised whole wall rows), FR = 4 on large grids halves
// the number of waves.  With adv non-null the step number is the one collide_kernel
// saved in stepc, and one lane sets *adv (the caller's step counter, read by nothing else
// in this kernel) to the next step number.
constexpr int FR_BLOCK = 256;

template <typename T, int GEOM, int FR, bool REC = false>
__global__ __launch_bounds__(FR_BLOCK) void flight_rest_kernel(
    fp_config g, int32_t ncell, const int32_t* __restrict__ offsets,
    const int32_t* __restrict__ pend, const int32_t* __restrict__ plist, T* __restrict__ px,
    T* __restrict__ py, T* __restrict__ pvx, T* __restrict__ pvy, T* __restrict__ pvz,
    const uint32_t* __restrict__ ppid, int32_t* __restrict__ pkey, uint32_t step_arg,
    const uint32_t* stepp, uint32_t* adv, const uint32_t* __restrict__ stepc,
    const int32_t* __restrict__ kmap, double* __restrict__ wall, const double* __restrict__ wall_edge,
    int32_t wall_nbins) {
    constexpr int FR_CELLS = FR;
    if (adv && blockIdx.x == 0 && threadIdx.x == 0) adv[0] = stepc[0] + 1u;
    const int lane = threadIdx.x & 63;
    const int32_t c0 = (int32_t)((blockIdx.x * (FR_BLOCK / 64) + (threadIdx.x >> 6)) * FR_CELLS);
    int32_t np = 0, b = 0;
    if (lane < FR_CELLS && c0 + lane < ncell) np = pend[c0 + lane];
    if (__ballot(np > 0) == 0) return;
    if (np > 0) b = offsets[c0 + lane];
    int32_t pre[FR_CELLS + 1], bs[FR_CELLS];
    pre[0] = 0;
#pragma unroll
    for (int c = 0; c < FR_CELLS; ++c) {
        pre[c + 1] = pre[c] + __shfl(np, c, 64);
        bs[c] = __shfl(b, c, 64);
    }
    const uint32_t step = adv ? stepc[0] : (stepp ? stepp[0] : step_arg);
    const bool f32 = sizeof(T) == 4;
    constexpr bool TWO_D = GEOM != FP_COUETTE1D;
    const Walls W = make_walls(g);
    const double inv_dx = 1.0 / g.dx, inv_dy = 1.0 / g.dy;
    for (int32_t i = lane; i < pre[FR_CELLS]; i += 64) {
        int32_t at = bs[0] + i;
#pragma unroll
        for (int c = 1; c < FR_CELLS; ++c)
            if (i >= pre[c]) at = bs[c] + (i - pre[c]);
        const int32_t p = plist[at];
        double pos[2] = {(double)px[p], TWO_D ? (double)py[p] : 0.0};
        double v[3] = {(double)pvx[p], (double)pvy[p], (double)pvz[p]};
        bool gone = false;
        if constexpr (GEOM == FP_CYLINDER2D) {
            gone = fly_open<REC>(g, pos, v, ppid[p], step, f32, wall, wall_edge, wall_nbins);
            pos[0] = st_round(pos[0], f32);
            pos[1] = st_round(pos[1], f32);
        } else {
            fly<TWO_D>(g, W, pos, v, ppid[p], step, f32);
        }
        px[p] = (T)pos[0];
        if (TWO_D) py[p] = (T)pos[1];
        pvx[p] = (T)v[0]; pvy[p] = (T)v[1]; pvz[p] = (T)v[2];
        pkey[p] = gone ? ncell : cell_key<TWO_D>(g, pos[0], pos[1], inv_dx, inv_dy, kmap);
    }
}

// flight (or key recomputation) without a collision: one thread per particle
template <typename T, int GEOM, bool REC = false>
__global__ __launch_bounds__(ST_BLOCK) void move_kernel(fp_config g, int64_t n,
                                                         const int64_t* __restrict__ n_dev, T* __restrict__ px,
                                                         T* __restrict__ py, T* __restrict__ pvx,
                                                         T* __restrict__ pvy, T* __restrict__ pvz,
                                                         const uint32_t* __restrict__ ppid,
                                                         int32_t* __restrict__ pkey, uint32_t step_arg,
                                                         int keys_only, const uint32_t* __restrict__ stepp,
                                                         int32_t ncell, const int32_t* __restrict__ kmap,
                                                         double* __restrict__ wall,
                                                         const double* __restrict__ wall_edge, int32_t wall_nbins) {
    const uint32_t step = stepp ? stepp[0] : step_arg;
    if (n_dev) n = *n_dev;
    constexpr bool TWO_D = GEOM != FP_COUETTE1D;
    const int64_t p = (int64_t)blockIdx.x * ST_BLOCK + threadIdx.x;
    if (p >= n) return;
    const double inv_dx = 1.0 / g.dx, inv_dy = 1.0 / g.dy;
    double pos[2] = {(double)px[p], TWO_D ? (double)py[p] : 0.0};
    bool gone = false;
    if (!keys_only) {
        const bool f32 = sizeof(T) == 4;
        double v[3] = {(double)pvx[p], (double)pvy[p], (double)pvz[p]};
        if constexpr (GEOM == FP_CYLINDER2D) {
            gone = fly_open<REC>(g, pos, v, ppid[p], step, f32, wall, wall_edge, wall_nbins);
            pos[0] = st_round(pos[0], f32);
            pos[1] = st_round(pos[1], f32);
        } else {
            const Walls W = make_walls(g);
            fly<TWO_D>(g, W, pos, v, ppid[p], step, f32);
        }
        px[p] = (T)pos[0];
        if (TWO_D) py[p] = (T)pos[1];
        pvx[p] = (T)v[0]; pvy[p] = (T)v[1]; pvz[p] = (T)v[2];
    }
    pkey[p] = gone ? ncell : cell_key<TWO_D>(g, pos[0], pos[1], inv_dx, inv_dy, kmap);
}

template <typename T, int G, int GEOM>
static void collide_launch(fp_ctx* c, fp_particles* p, const int32_t* off, const double* mom,
                           const double* rec, uint32_t step, int move, const uint32_t* stepp,
                           uint32_t* adv, hipStream_t s) {
    const int64_t threads = (int64_t)c->ncell * G;
    const unsigned grid = (unsigned)((threads + ST_BLOCK - 1) / ST_BLOCK);
    // register cache of c* (and of the positions): ST_K particles per lane, as many as the
    // lane widths of collide_dispatch give a lane on average; particles beyond it keep c* in
    // the velocity arrays.  A larger cache costs registers and resident waves (8 per lane
    // on the quadtree's 24-particle leaves at 16 lanes: 1.88 against 1.81 ms per step)
    constexpr int K = ST_K;
    hipLaunchKernelGGL((collide_kernel<T, G, K, GEOM>), dim3(grid), dim3(ST_BLOCK), 0, s,
                       c->cfg, c->ncell, off, mom, rec, (T*)p->x, (T*)p->y, (T*)p->vx, (T*)p->vy,
                       (T*)p->vz, p->pid, p->key, step, move, stepp, c->pend, c->bidx,
                       adv ? c->stepc : nullptr, (const int32_t*)c->leafmap);
    if (move) {
        const int fr = c->ncell <= 65536 ? 2 : 4;
        const int32_t per_block = FR_BLOCK / 64 * fr;
        const dim3 fgrid((c->ncell + per_block - 1) / per_block);
        // surface sampling: a variant with the exchange records (their registers stay out
        // of the plain kernel)
        auto fr_launch = [&](auto kern) {
            hipLaunchKernelGGL(kern, fgrid, dim3(FR_BLOCK), 0, s, c->cfg, c->ncell, off,
                               (const int32_t*)c->pend, (const int32_t*)c->bidx, (T*)p->x, (T*)p->y,
                               (T*)p->vx, (T*)p->vy, (T*)p->vz, p->pid, p->key, step, stepp, adv,
                               (const uint32_t*)c->stepc, (const int32_t*)c->leafmap, c->wall,
                               (const double*)c->wall_edge, c->wall_nbins);
        };
        const bool rec = GEOM == FP_CYLINDER2D && c->wall != nullptr;
        if (fr == 2) {
            if (rec) fr_launch(flight_rest_kernel<T, GEOM, 2, GEOM == FP_CYLINDER2D>);
            else fr_launch(flight_rest_kernel<T, GEOM, 2, false>);
        } else {
            if (rec) fr_launch(flight_rest_kernel<T, GEOM, 4, GEOM == FP_CYLINDER2D>);
            else fr_launch(flight_rest_kernel<T, GEOM, 4, false>);
        }
    }
}

template <typename T, int GEOM>
static void collide_dispatch(fp_ctx* c, fp_particles* p, const int32_t* off, const double* mom,
                             const double* rec, uint32_t step, int move, const uint32_t* sp,
                             uint32_t* adv, hipStream_t s) {
    // about two particles per lane: at 100 particles per cell a whole wave per cell (its
    // coefficients wave-uniform, in scalar registers; 74 VGPRs, 6 waves per SIMD) was
    // measured 4 % faster than 32 lanes (82 VGPRs, 5 waves) and 9 % faster than 16
    switch (lanes_per_cell(c, p->n, FILL_4, 2)) {
        case 4: collide_launch<T, 4, GEOM>(c, p, off, mom, rec, step, move, sp, adv, s); break;
        case 8: collide_launch<T, 8, GEOM>(c, p, off, mom, rec, step, move, sp, adv, s); break;
        case 16: collide_launch<T, 16, GEOM>(c, p, off, mom, rec, step, move, sp, adv, s); break;
        case 32: collide_launch<T, 32, GEOM>(c, p, off, mom, rec, step, move, sp, adv, s); break;
        default: collide_launch<T, 64, GEOM>(c, p, off, mom, rec, step, move, sp, adv, s); break;
    }
}

template <typename T>
static void step_typed(fp_ctx* c, fp_particles* p, const int32_t* off, const double* mom,
                       const double* rec, uint32_t step, uint32_t flags, const uint32_t* sp,
                       hipStream_t s) {
    const int geom = c->cfg.geometry;
    const int move = (flags & FP_STEP_MOVE) ? 1 : 0;
    if ((flags & FP_STEP_COLLIDE) && move) {
        // the counter advance rides on the last kernel of the step
        uint32_t* adv = (flags & FP_STEP_ADVANCE) ? const_cast<uint32_t*>(sp) : nullptr;
        if (geom == FP_CAVITY2D) collide_dispatch<T, FP_CAVITY2D>(c, p, off, mom, rec, step, move, sp, adv, s);
        else if (geom == FP_CYLINDER2D)
            collide_dispatch<T, FP_CYLINDER2D>(c, p, off, mom, rec, step, move, sp, adv, s);
        else collide_dispatch<T, FP_COUETTE1D>(c, p, off, mom, rec, step, move, sp, adv, s);
        return;
    }
    if (flags & FP_STEP_ADVANCE) {
        // the other forms end with a kernel of their own for it
        step_typed<T>(c, p, off, mom, rec, step, flags & ~FP_STEP_ADVANCE, sp, s);
        launch_counter_add(c, const_cast<uint32_t*>(sp), 1u, s);
        return;
    }
    if (flags & FP_STEP_COLLIDE) {
        if (geom == FP_CAVITY2D) collide_dispatch<T, FP_CAVITY2D>(c, p, off, mom, rec, step, 0, sp, nullptr, s);
        else if (geom == FP_CYLINDER2D)
            collide_dispatch<T, FP_CYLINDER2D>(c, p, off, mom, rec, step, 0, sp, nullptr, s);
        else collide_dispatch<T, FP_COUETTE1D>(c, p, off, mom, rec, step, 0, sp, nullptr, s);
        return;
    }
    const int64_t slots = slots_of(p);
    if (slots == 0) return;
    const unsigned grid = (unsigned)((slots + ST_BLOCK - 1) / ST_BLOCK);
    const int64_t* nd = p->n_dev;
    const int keys_only = (flags & FP_STEP_KEYS) ? 1 : 0;
    if (geom == FP_CAVITY2D)
        hipLaunchKernelGGL((move_kernel<T, FP_CAVITY2D>), dim3(grid), dim3(ST_BLOCK), 0, s, c->cfg,
                           p->n, nd, (T*)p->x, (T*)p->y, (T*)p->vx, (T*)p->vy, (T*)p->vz, p->pid, p->key,
                           step, keys_only, sp, c->ncell, (const int32_t*)c->leafmap, c->wall,
                           (const double*)c->wall_edge, c->wall_nbins);
    else if (geom == FP_CYLINDER2D && c->wall)
        hipLaunchKernelGGL((move_kernel<T, FP_CYLINDER2D, true>), dim3(grid), dim3(ST_BLOCK), 0, s, c->cfg,
                           p->n, nd, (T*)p->x, (T*)p->y, (T*)p->vx, (T*)p->vy, (T*)p->vz, p->pid, p->key,
                           step, keys_only, sp, c->ncell, (const int32_t*)c->leafmap, c->wall,
                           (const double*)c->wall_edge, c->wall_nbins);
    else if (geom == FP_CYLINDER2D)
        hipLaunchKernelGGL((move_kernel<T, FP_CYLINDER2D>), dim3(grid), dim3(ST_BLOCK), 0, s, c->cfg,
                           p->n, nd, (T*)p->x, (T*)p->y, (T*)p->vx, (T*)p->vy, (T*)p->vz, p->pid, p->key,
                           step, keys_only, sp, c->ncell, (const int32_t*)c->leafmap, c->wall,
                           (const double*)c->wall_edge, c->wall_nbins);
    else
        hipLaunchKernelGGL((move_kernel<T, FP_COUETTE1D>), dim3(grid), dim3(ST_BLOCK), 0, s, c->cfg,
                           p->n, nd, (T*)p->x, (T*)nullptr, (T*)p->vx, (T*)p->vy, (T*)p->vz, p->pid,
                           p->key, step, keys_only, sp, c->ncell, (const int32_t*)c->leafmap, c->wall,
                           (const double*)c->wall_edge, c->wall_nbins);
}


// ---- free-stream inflow of the open domain ------------------------------------------------
// counts of the four rectangles: floor(lambda_r) + Bernoulli(lambda_r - floor(lambda_r))
// with the uniform of counter (r, step, 5, 1); cnt[0..3] counts, cnt[4..8] prefix, cnt[9]
// the first slot (the host's at, or *n_dev; -1 when the slots do not fit below cap, which
// is counted in *ovf), cnt[10] the step number (the host's, or *step_dev)
__global__ void inject_count_kernel(fp_config g, double l0, double l1, double l2, double l3,
                                    uint32_t step, const uint32_t* __restrict__ step_dev,
                                    int64_t at, const int64_t* __restrict__ n_dev, int64_t cap,
                                    int32_t slots, int32_t* __restrict__ cnt,
                                    unsigned long long* __restrict__ ovf) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (step_dev) step = *step_dev;
    if (n_dev) {
        at = *n_dev;
        if (at < 0 || at + slots > cap) {
            at = -1;
            atomicAdd(ovf, 1ull);
        }
    }
    cnt[9] = (int32_t)at;
    cnt[10] = (int32_t)step;
    const double lam[4] = {l0, l1, l2, l3};
    int32_t pre = 0;
    cnt[4] = 0;
    for (int r = 0; r < 4; ++r) {
        const double base = floor(lam[r]);
        const uint4 d = draw(g.seed, (uint32_t)r, step, PURPOSE_INJECT, 1);
        const int32_t k = (int32_t)base + (u01d(d.x) < lam[r] - base ? 1 : 0);
        cnt[r] = k;
        pre += k;
        cnt[5 + r] = pre;
    }
}

struct InjectGeom {
    double rect[4][4];
    int32_t slot0[5];
};

template <typename T>
__global__ __launch_bounds__(ST_BLOCK) void inject_kernel(fp_config g, InjectGeom ig,
                                                          const int32_t* __restrict__ cnt,
                                                          const uint32_t* __restrict__ pid_next,
                                                          T* __restrict__ px, T* __restrict__ py,
                                                          T* __restrict__ pvx, T* __restrict__ pvy,
                                                          T* __restrict__ pvz, uint32_t* __restrict__ ppid,
                                                          int32_t* __restrict__ pkey, int32_t ncell,
                                                          const int32_t* __restrict__ kmap) {
    const int32_t at = cnt[9];
    const uint32_t step = (uint32_t)cnt[10];
    if (at < 0) return;   // no room: nothing is written
    const int32_t k0 = blockIdx.x * ST_BLOCK + threadIdx.x;   // slot of the call
    if (k0 >= ig.slot0[4]) return;
    const int64_t slot = (int64_t)at + k0;
    int r = 0;
    while (r < 3 && k0 >= ig.slot0[r + 1]) ++r;
    const int32_t k = k0 - ig.slot0[r];
    const bool f32 = sizeof(T) == 4;
    if (k >= cnt[r]) {
        pkey[slot] = ncell;   // unused slot
        return;
    }
    const int32_t gidx = (r == 0 ? 0 : cnt[4 + r]) + k;
    const uint32_t id = pid_next[0] + (uint32_t)gidx;
    const double xa = ig.rect[r][0], xb = ig.rect[r][1], ya = ig.rect[r][2], yb = ig.rect[r][3];
    const uint4 d0 = draw(g.seed, id, step, PURPOSE_INJECT, 0);
    const uint4 d1 = draw(g.seed, id, step, PURPOSE_INJECT, 2);
    const double RT = g.kB / g.mass * g.T_inf;
    const double s = sqrt(RT);
    const double x = xa + u01d(d0.x) * (xb - xa);
    const double y = ya + u01d(d0.y) * (yb - ya);
    const double r0 = sqrt(-2.0 * log(u01d(d0.z)));
    const double v0 = g.u_inf[0] + s * (r0 * cos(TWO_PI * u01d(d0.w)));
    const double v1 = g.u_inf[1] + s * (r0 * sin(TWO_PI * u01d(d0.w)));
    const double v2 = g.u_inf[2] + s * (sqrt(-2.0 * log(u01d(d1.x))) * cos(TWO_PI * u01d(d1.y)));
    const double ex = x + v0 * g.dt;
    const double ey = y + v1 * g.dt;
    const double x1 = g.x0 + g.lx, y1 = g.y0 + g.ly;
    if (!(ex >= g.x0 && ex <= x1 && ey >= g.y0 && ey <= y1)) {
        pkey[slot] = ncell;   // did not enter
        return;
    }
    const double sx = st_round(ex, f32), sy = st_round(ey, f32);
    px[slot] = (T)sx;
    py[slot] = (T)sy;
    pvx[slot] = (T)v0;
    pvy[slot] = (T)v1;
    pvz[slot] = (T)v2;
    ppid[slot] = id;
    pkey[slot] = cell_key<true>(g, sx, sy, 1.0 / g.dx, 1.0 / g.dy, kmap);
}

// after the slots are written: ids advance by the candidates drawn, the device count (if
// any) by the slots, the step counter (if asked) by one
__global__ void inject_advance_kernel(const int32_t* __restrict__ cnt, uint32_t* __restrict__ pid_next,
                                      int64_t* __restrict__ n_dev, int32_t slots,
                                      uint32_t* __restrict__ adv) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (cnt[9] >= 0) {
        pid_next[0] += (uint32_t)cnt[8];
        if (n_dev) n_dev[0] = (int64_t)cnt[9] + slots;
    }
    if (adv) adv[0] += 1u;
}

template <typename T>
static void inject_typed(fp_ctx* c, fp_particles* p, int64_t at, uint32_t* pid_next, uint32_t step,
                         const uint32_t* step_dev, uint32_t* adv, hipStream_t s) {
    InjectGeom ig;
    for (int r = 0; r < 4; ++r)
        for (int k = 0; k < 4; ++k) ig.rect[r][k] = c->inj_rect[r][k];
    for (int r = 0; r < 5; ++r) ig.slot0[r] = c->inj_slot0[r];
    const int32_t slots = ig.slot0[4];
    // at < 0: the first slot is the device count (fp_inject_dev)
    int64_t* n_dev = at < 0 ? p->n_dev : nullptr;
    hipLaunchKernelGGL(inject_count_kernel, dim3(1), dim3(64), 0, s, c->cfg, c->inj_lambda[0],
                       c->inj_lambda[1], c->inj_lambda[2], c->inj_lambda[3], step, step_dev, at,
                       (const int64_t*)n_dev, (int64_t)p->capacity, slots, c->inj, c->errcount + 1);
    if (slots > 0)
        hipLaunchKernelGGL((inject_kernel<T>), dim3((slots + ST_BLOCK - 1) / ST_BLOCK), dim3(ST_BLOCK),
                           0, s, c->cfg, ig, (const int32_t*)c->inj, (const uint32_t*)pid_next,
                           (T*)p->x, (T*)p->y, (T*)p->vx, (T*)p->vy, (T*)p->vz, p->pid, p->key, c->ncell,
                           (const int32_t*)c->leafmap);
    hipLaunchKernelGGL(inject_advance_kernel, dim3(1), dim3(64), 0, s, (const int32_t*)c->inj, pid_next,
                       n_dev, slots, adv);
}

int launch_inject(fp_ctx* c, fp_particles* p, int64_t at, uint32_t* pid_next, uint32_t step,
                  const uint32_t* step_dev, uint32_t* adv, hipStream_t s) {
    if (c->cfg.precision == FP_F32) inject_typed<float>(c, p, at, pid_next, step, step_dev, adv, s);
    else inject_typed<double>(c, p, at, pid_next, step, step_dev, adv, s);
    return check_launch(c, "fp_inject");
}

int launch_step(fp_ctx* c, fp_particles* p, const int32_t* offsets, const double* mom,
                const double* rec, uint64_t step, uint32_t flags, const uint32_t* step_dev,
                hipStream_t s) {
    if (c->cfg.precision == FP_F32)
        step_typed<float>(c, p, offsets, mom, rec, (uint32_t)step, flags, step_dev, s);
    else
        step_typed<double>(c, p, offsets, mom, rec, (uint32_t)step, flags, step_dev, s);
    return check_launch(c, "fp_step");
}

__global__ void counter_add_kernel(uint32_t* __restrict__ ctr, uint32_t inc) {
    if (threadIdx.x == 0 && blockIdx.x == 0) ctr[0] += inc;
}

int launch_counter_add(fp_ctx* c, uint32_t* ctr, uint32_t inc, hipStream_t s) {
    hipLaunchKernelGGL(counter_add_kernel, dim3(1), dim3(64), 0, s, ctr, inc);
    return check_launch(c, "fp_counter_add");
}

}  // namespace fpg
