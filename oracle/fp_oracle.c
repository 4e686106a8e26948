/*
 * fp_oracle.c -- plain FP64 CPU oracle of the cubic Fokker-Planck particle step.
 *
 * TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark are the only users.  No GPU code includes or links this file.
 *
 * Every function follows one passage of the paper (Roohi, "Accelerating Kinetic
 * Fokker-Planck Simulations via a GPU-Native Deep Neural Network Surrogate"):
 *   or_moments        central velocity moments entering the closure (Sec. "The Moment-
 *                     Matching Closure"; moment definition below eq. system9x9)
 *   or_closure_system the moment-matching conditions (eq. moment_match) for the test
 *                     functions c_i c_j and c_i |c|^2 under the cubic drift (eq.
 *                     cubic_drift) and isotropic noise (eqs. cubic_diffusion, sde_vel),
 *                     with the stress relaxing at 2/tau and the heat flux at 4/(3 tau)
 *                     (tau = 2 mu / p, eq. tau; Pr = 2/3).  Its V and W blocks are
 *                     Table matrix_system with the second-order moments P_ij in V.
 *   or_update         eqs. update_vel, update_N, update_alpha
 *   or_move           eq. update_pos with diffuse isothermal walls
 *   or_run            the order of Algorithm "Baseline Physics Simulation Loop"
 * Plain loops, no blocking or fusion; sums run in particle order.  Loops whose every
 * output belongs to one iteration (a cell, a particle) may be split across threads
 * (OpenMP); the arithmetic of each output is unchanged, so no result depends on the
 * number of threads.
 */
#include "fp_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* threads of the parallel loops (n <= 0: the OpenMP default); returns the count in use */
int or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

#define OR_PI 3.14159265358979323846

/* ------------------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2,
 * 3", SC'11): ten rounds of two 32x32->64 multiplies with the Weyl key schedule.        */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

void or_uniforms(uint64_t seed, uint32_t pid, uint32_t step, uint32_t purpose, uint32_t sub,
                 double u[4])
{
    uint32_t ctr[4] = {pid, step, purpose, sub};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t r[4];
    or_philox4x32_10(ctr, key, r);
    for (int i = 0; i < 4; ++i) u[i] = ((double)r[i] + 0.5) * 0x1p-32;
}

/* Box-Muller: the paper asks for standard normal variates (list under eq. update_vel) */
void or_normals3(uint64_t seed, uint32_t pid, uint32_t step, uint32_t purpose, uint32_t sub,
                 double z[3])
{
    double u[4];
    or_uniforms(seed, pid, step, purpose, sub, u);
    double r0 = sqrt(-2.0 * log(u[0]));
    double r1 = sqrt(-2.0 * log(u[2]));
    z[0] = r0 * cos(2.0 * OR_PI * u[1]);
    z[1] = r0 * sin(2.0 * OR_PI * u[1]);
    z[2] = r1 * cos(2.0 * OR_PI * u[3]);
}

/* ------------------------------------------------------------------------------------ */
static int32_t axis_index(double pos, double origin, double inv_h, int32_t ncell)
{
    double f = floor((pos - origin) * inv_h);
    if (!(f >= 0.0)) return 0;               /* also catches NaN */
    if (f > (double)(ncell - 1)) return ncell - 1;
    return (int32_t)f;
}

void or_keys(const or_config* cfg, int64_t n, const double* x, const double* y, int32_t* key)
{
    double inv_dx = 1.0 / cfg->dx;
    double inv_dy = 1.0 / cfg->dy;
    #pragma omp parallel for schedule(static) if (n > 4096)
    for (int64_t p = 0; p < n; ++p) {
        int32_t kx = axis_index(x[p], cfg->x0, inv_dx, cfg->nx);
        int32_t ky = 0;
        if (cfg->geometry != OR_COUETTE1D) ky = axis_index(y[p], cfg->y0, inv_dy, cfg->ny);
        key[p] = ky * cfg->nx + kx;
    }
}

/* Stable counting sort (sort step of the loop): slot order within a cell is the
 * previous order of the particles.  Particles with key == ncell (deleted) or a key
 * outside [0, ncell] are dropped. */
void or_bin(int32_t ncell, int64_t n, const int32_t* key, int64_t* perm, int32_t* offsets)
{
    for (int32_t c = 0; c <= ncell; ++c) offsets[c] = 0;
    /* key == ncell marks a deleted particle; keys outside [0, ncell] name no cell: both
       take no part in the sort */
    for (int64_t p = 0; p < n; ++p)
        if (key[p] >= 0 && key[p] < ncell) offsets[key[p] + 1] += 1;
    for (int32_t c = 0; c < ncell; ++c) offsets[c + 1] += offsets[c];
    int32_t* cursor = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ncell > 0 ? ncell : 1));
    for (int32_t c = 0; c < ncell; ++c) cursor[c] = offsets[c];
    for (int64_t p = 0; p < n; ++p)
        if (key[p] >= 0 && key[p] < ncell) perm[cursor[key[p]]++] = p;
    free(cursor);
}

/* ------------------------------------------------------------------------------------ */
/* index of the symmetric pair (i,j) in the order 11 12 13 22 23 33 */
static int sym2(int i, int j)
{
    if (i > j) { int t = i; i = j; j = t; }
    static const int tab[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
    return tab[i][j];
}
/* index of the symmetric triple (i,j,k) in the order 111 112 113 122 123 133 222 223 233 333 */
static int sym3(int i, int j, int k)
{
    int a[3] = {i, j, k};
    for (int s = 0; s < 2; ++s)
        for (int t = 0; t < 2 - s; ++t)
            if (a[t] > a[t + 1]) { int q = a[t]; a[t] = a[t + 1]; a[t + 1] = q; }
    static const int tab[3][3][3] = {
        {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}},
        {{1, 3, 4}, {3, 6, 7}, {4, 7, 8}},
        {{2, 4, 5}, {4, 7, 8}, {5, 8, 9}}};
    return tab[a[0]][a[1]][a[2]];
}

enum { M_N = 0, M_U = 1, M_TH = 4, M_P = 5, M_T = 11, M_R = 21, M_W = 27, M_H = 30 };

void or_moments(int32_t ncell, const int32_t* offsets, const double* vx, const double* vy,
                const double* vz, double* mom)
{
    #pragma omp parallel for schedule(dynamic, 16) if (ncell > 64)
    for (int32_t cell = 0; cell < ncell; ++cell) {
        double* m = mom + (int64_t)cell * OR_MOM_STRIDE;
        for (int i = 0; i < OR_MOM_STRIDE; ++i) m[i] = 0.0;
        int32_t b = offsets[cell], e = offsets[cell + 1];
        int32_t n = e - b;
        m[M_N] = (double)n;
        if (n == 0) continue;
        double U[3] = {0.0, 0.0, 0.0};
        for (int32_t p = b; p < e; ++p) { U[0] += vx[p]; U[1] += vy[p]; U[2] += vz[p]; }
        for (int i = 0; i < 3; ++i) U[i] /= (double)n;
        double P[6] = {0}, T[10] = {0}, R[6] = {0}, W[3] = {0}, H = 0.0;
        for (int32_t p = b; p < e; ++p) {
            double c[3] = {vx[p] - U[0], vy[p] - U[1], vz[p] - U[2]};
            double c2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
            for (int i = 0; i < 3; ++i)
                for (int j = i; j < 3; ++j) {
                    P[sym2(i, j)] += c[i] * c[j];
                    R[sym2(i, j)] += c[i] * c[j] * c2;
                    for (int k = j; k < 3; ++k) T[sym3(i, j, k)] += c[i] * c[j] * c[k];
                }
            for (int i = 0; i < 3; ++i) W[i] += c[i] * c2 * c2;
            H += c2 * c2 * c2;
        }
        for (int i = 0; i < 3; ++i) m[M_U + i] = U[i];
        for (int i = 0; i < 6; ++i) m[M_P + i] = P[i] / (double)n;
        for (int i = 0; i < 10; ++i) m[M_T + i] = T[i] / (double)n;
        for (int i = 0; i < 6; ++i) m[M_R + i] = R[i] / (double)n;
        for (int i = 0; i < 3; ++i) m[M_W + i] = W[i] / (double)n;
        m[M_H] = H / (double)n;
        m[M_TH] = (m[M_P + 0] + m[M_P + 3] + m[M_P + 5]) / 3.0;
    }
}

/* ------------------------------------------------------------------------------------ */
/* Collision time tau = 2 mu / p (eq. tau) with the VHS law for mu, and the cubic
 * stabiliser eps^2 = eps_hat / (theta tau).                                           */
void or_cell_params(const or_config* cfg, const double* m, double nvol, double* tau,
                    double* eps2)
{
    double theta = m[M_TH];
    double T = theta * cfg->mass / cfg->kB;
    double ndens = m[M_N] * nvol;
    double p = ndens * cfg->kB * T;
    double mu = cfg->mu_ref * pow(T / cfg->T_ref, cfg->omega);
    *tau = 2.0 * mu / p;
    *eps2 = cfg->eps_hat / (theta * (*tau));
}

/* Normalised moment-matching system of one cell.  Unknowns y = (Ch11 Ch12 Ch13 Ch22
 * Ch23 Ch33, Gh1 Gh2 Gh3) with Ch = tau Ct, Gh = tau sqrt(theta) Gamma, where the drift
 * is A = -c/tau + N and N = Ct c + Gamma (|c|^2 - 3 theta) - eps^2 (c |c|^2 - S) (eqs.
 * cubic_drift, update_N).  Moments are scaled by powers of theta (P/theta, T/theta^1.5,
 * R/theta^2, W/theta^2.5) and eps_hat = eps^2 theta tau.
 *   rows (ij):  sum_k (Ch_ik P_kj + Ch_jk P_ki) + Gh_i S_j + Gh_j S_i = 2 eps_hat R_ij
 *   rows (i):   sum_j Ch_ij S_j + 2 sum_jk Ch_jk T_ijk + Gh_i (Q - 9)
 *               + 2 sum_k Gh_k (R_ik - 3 P_ik) = 5/3 S_i + eps_hat (3 W_i - 3 S_i - 2 P_ik S_k)
 * with S_i = T_ikk and Q = R_kk.  Each equation is written out term by term; symmetric
 * unknowns collect the contributions of both index orders.                           */
void or_closure_system(const double* m, double eps_hat, double* A, double* b)
{
    double th = m[M_TH];
    double s15 = th * sqrt(th);
    double Ph[3][3], Th[3][3][3], Rh[3][3], Wh[3], Sh[3], Qh = 0.0;
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) {
            Ph[i][j] = m[M_P + sym2(i, j)] / th;
            Rh[i][j] = m[M_R + sym2(i, j)] / (th * th);
            for (int k = 0; k < 3; ++k) Th[i][j][k] = m[M_T + sym3(i, j, k)] / s15;
        }
        Wh[i] = m[M_W + i] / (th * th * sqrt(th));
    }
    for (int i = 0; i < 3; ++i) {
        Sh[i] = 0.0;
        for (int k = 0; k < 3; ++k) Sh[i] += Th[i][k][k];
        Qh += Rh[i][i];
    }
    for (int r = 0; r < 81; ++r) A[r] = 0.0;
    for (int r = 0; r < 9; ++r) b[r] = 0.0;
    /* stress rows */
    for (int i = 0; i < 3; ++i)
        for (int j = i; j < 3; ++j) {
            int r = sym2(i, j);
            for (int k = 0; k < 3; ++k) {
                A[r * 9 + sym2(i, k)] += Ph[k][j];
                A[r * 9 + sym2(j, k)] += Ph[k][i];
            }
            A[r * 9 + 6 + i] += Sh[j];
            A[r * 9 + 6 + j] += Sh[i];
            b[r] = 2.0 * eps_hat * Rh[i][j];
        }
    /* heat-flux rows */
    for (int i = 0; i < 3; ++i) {
        int r = 6 + i;
        for (int j = 0; j < 3; ++j) A[r * 9 + sym2(i, j)] += Sh[j];
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k) A[r * 9 + sym2(j, k)] += 2.0 * Th[i][j][k];
        A[r * 9 + 6 + i] += Qh - 9.0;
        for (int k = 0; k < 3; ++k) A[r * 9 + 6 + k] += 2.0 * (Rh[i][k] - 3.0 * Ph[i][k]);
        double PS = 0.0;
        for (int k = 0; k < 3; ++k) PS += Ph[i][k] * Sh[k];
        b[r] = 5.0 / 3.0 * Sh[i] + eps_hat * (3.0 * Wh[i] - 3.0 * Sh[i] - 2.0 * PS);
    }
}

/* Gaussian elimination with partial pivoting; returns 0, or 1 if a pivot is below tol */
static int solve9(double* A, double* b, double* y, double tol)
{
    for (int k = 0; k < 9; ++k) {
        int piv = k;
        double best = fabs(A[k * 9 + k]);
        for (int r = k + 1; r < 9; ++r)
            if (fabs(A[r * 9 + k]) > best) { best = fabs(A[r * 9 + k]); piv = r; }
        if (!(best >= tol)) return 1;
        if (piv != k) {
            for (int c = 0; c < 9; ++c) {
                double t = A[k * 9 + c]; A[k * 9 + c] = A[piv * 9 + c]; A[piv * 9 + c] = t;
            }
            double t = b[k]; b[k] = b[piv]; b[piv] = t;
        }
        for (int r = k + 1; r < 9; ++r) {
            double f = A[r * 9 + k] / A[k * 9 + k];
            for (int c = k; c < 9; ++c) A[r * 9 + c] -= f * A[k * 9 + c];
            b[r] -= f * b[k];
        }
    }
    for (int k = 8; k >= 0; --k) {
        double s = b[k];
        for (int c = k + 1; c < 9; ++c) s -= A[k * 9 + c] * y[c];
        y[k] = s / A[k * 9 + k];
    }
    return 0;
}

void or_closure(const or_config* cfg, int32_t ncell, const double* mom, const double* nvol,
                double* rec, int32_t* status)
{
    #pragma omp parallel for schedule(dynamic, 16) if (ncell > 64)
    for (int32_t cell = 0; cell < ncell; ++cell) {
        const double* m = mom + (int64_t)cell * OR_MOM_STRIDE;
        double* r = rec + (int64_t)cell * OR_REC_STRIDE;
        for (int i = 0; i < OR_REC_STRIDE; ++i) r[i] = 0.0;
        int st = OR_OK;
        int finite = 1;
        for (int i = 0; i < 31; ++i) if (!isfinite(m[i])) finite = 0;
        double theta = m[M_TH];
        if (m[M_N] <= 1.0) st = OR_EMPTY;
        else if (!finite) st = OR_NONFINITE;
        else if (!(theta > 0.0)) st = OR_EMPTY;
        if (st != OR_OK) {
            r[11] = 1.0;                         /* E: no relaxation */
            r[10] = finite ? theta : 0.0;
            r[14] = (double)st;
            status[cell] = st;
            continue;
        }
        double tau, eps2;
        or_cell_params(cfg, m, nvol ? nvol[cell] : cfg->fnum_over_vol, &tau, &eps2);
        double E = exp(-cfg->dt / tau);
        double sigma = sqrt(theta * (1.0 - exp(-2.0 * cfg->dt / tau)));
        double y[9] = {0};
        if (m[M_N] < (double)cfg->n_min) {
            st = OR_FEW;
        } else {
            double A[81], b[9];
            or_closure_system(m, cfg->eps_hat, A, b);
            if (solve9(A, b, y, cfg->pivot_tol) != 0) st = OR_SINGULAR;
            for (int i = 0; i < 9 && st == OR_OK; ++i) if (!isfinite(y[i])) st = OR_SINGULAR;
        }
        if (st == OR_OK) {
            for (int i = 0; i < 6; ++i) r[i] = y[i] / tau;
            for (int i = 0; i < 3; ++i) r[6 + i] = y[6 + i] / (tau * sqrt(theta));
            r[12] = eps2;
        } else {
            r[12] = 0.0;                         /* Langevin: N = 0 */
        }
        r[9] = tau; r[10] = theta; r[11] = E; r[13] = sigma; r[14] = (double)st;
        status[cell] = st;
    }
}


/* ------------------------------------------------------------------------------------ */
/* Gas volume of the cells.  The part of a cell covered by the circle is integrated over
 * x = cx + R sin(phi) (dx = R cos(phi) dphi, chord half-height R cos(phi)), split at the
 * angles where the chord ends cross the cell's horizontal edges, with 24-point
 * Gauss-Legendre on every smooth piece; the nodes are found by Newton iteration on the
 * Legendre polynomial. */
static void gauss_legendre(int n, double* xs, double* ws)
{
    for (int i = 0; i < n; ++i) {
        double x = cos(OR_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = p2;
            }
            double dp = n * (x * p1 - p0) / (x * x - 1.0);
            double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        double p0 = 1.0, p1 = x;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
            p0 = p1; p1 = p2;
        }
        double dp = n * (x * p1 - p0) / (x * x - 1.0);
        xs[i] = x;
        ws[i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
}

static double chord_in_cell(double phi, double cx, double cy, double R, double ya, double yb)
{
    (void)cx;
    double h = R * cos(phi);
    double lo = cy - h > ya ? cy - h : ya;
    double hi = cy + h < yb ? cy + h : yb;
    return hi > lo ? (hi - lo) * R * cos(phi) : 0.0;
}

static double covered_area(double cx, double cy, double R, double xa, double xb, double ya,
                           double yb, const double* gx, const double* gw, int ng)
{
    double lo = xa > cx - R ? xa : cx - R;
    double hi = xb < cx + R ? xb : cx + R;
    if (!(lo < hi)) return 0.0;
    double br[6];
    int nb = 0;
    br[nb++] = asin((lo - cx) / R);
    br[nb++] = asin((hi - cx) / R);
    double ys[2] = {ya, yb};
    for (int k = 0; k < 2; ++k) {
        double d = ys[k] - cy;
        if (fabs(d) < R) {
            double a = acos(fabs(d) / R);     /* chord end crosses y at x - cx = +-R sin(a) */
            for (int sg = -1; sg <= 1; sg += 2) {
                double ph = sg * a;
                if (ph > br[0] && ph < br[1]) br[nb++] = ph;
            }
        }
    }
    for (int i = 1; i < nb; ++i)
        for (int j = i; j > 0 && br[j] < br[j - 1]; --j) { double t = br[j]; br[j] = br[j - 1]; br[j - 1] = t; }
    double area = 0.0;
    for (int k = 0; k + 1 < nb; ++k) {
        double a = br[k], b = br[k + 1];
        if (!(b > a)) continue;
        double s = 0.0;
        for (int i = 0; i < ng; ++i) {
            double ph = 0.5 * (a + b) + 0.5 * (b - a) * gx[i];
            s += gw[i] * chord_in_cell(ph, cx, cy, R, ya, yb);
        }
        area += 0.5 * (b - a) * s;
    }
    return area;
}

void or_cell_volumes(const or_config* cfg, double* vol)
{
    double gx[24], gw[24];
    gauss_legendre(24, gx, gw);
    for (int32_t ky = 0; ky < cfg->ny; ++ky)
        for (int32_t kx = 0; kx < cfg->nx; ++kx) {
            double xa = cfg->x0 + kx * cfg->dx, xb = xa + cfg->dx;
            double ya = cfg->y0 + ky * cfg->dy, yb = ya + cfg->dy;
            double full = cfg->dx * cfg->dy;
            double v = full;
            if (cfg->geometry == OR_CYLINDER2D) {
                v = full - covered_area(cfg->circle[0], cfg->circle[1], cfg->circle[2], xa, xb, ya,
                                        yb, gx, gw, 24);
                if (v < 1e-12 * full) v = 0.0;     /* covered cells (up to rounding) */
                v *= cfg->depth;
            }
            vol[ky * cfg->nx + kx] = v;
        }
}

/* ------------------------------------------------------------------------------------ */
static double store(const or_config* cfg, double v)
{
    return cfg->precision == OR_F32 ? (double)(float)v : v;
}

/* Velocity update (eq. update_vel) with the nonlinear drift N (eq. update_N) and the
 * Ornstein-Uhlenbeck part integrated exactly.  After the step every cell is recentred
 * on its mean velocity (momentum); its energy is restored either exactly (EXACT) or by
 * the factor alpha of eq. update_alpha (PAPER).                                         */
void or_update(const or_config* cfg, int32_t ncell, const int32_t* offsets, double* vx,
               double* vy, double* vz, const uint32_t* pid, const double* mom,
               const double* rec, uint32_t step)
{
    int64_t n = offsets[ncell];
    double* cs = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    #pragma omp parallel for schedule(dynamic, 16) if (ncell > 64)
    for (int32_t cell = 0; cell < ncell; ++cell) {
        const double* m = mom + (int64_t)cell * OR_MOM_STRIDE;
        const double* r = rec + (int64_t)cell * OR_REC_STRIDE;
        int st = (int)r[14];
        if (st == OR_EMPTY || st == OR_NONFINITE) continue;
        int32_t b = offsets[cell], e = offsets[cell + 1];
        int32_t np = e - b;
        double U[3] = {m[M_U], m[M_U + 1], m[M_U + 2]};
        double Ct[3][3], G[3], S[3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) Ct[i][j] = r[sym2(i, j)];
        for (int i = 0; i < 3; ++i) {
            G[i] = r[6 + i];
            S[i] = 0.0;
            for (int k = 0; k < 3; ++k) S[i] += m[M_T + sym3(i, k, k)];
        }
        double tau = r[9], theta = r[10], E = r[11], eps2 = r[12], sigma = r[13];
        double sum_cs[3] = {0, 0, 0}, sum_NN = 0.0, sum_cN = 0.0;
        for (int32_t p = b; p < e; ++p) {
            double c[3] = {vx[p] - U[0], vy[p] - U[1], vz[p] - U[2]};
            double c2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
            double N[3];
            for (int i = 0; i < 3; ++i) {
                N[i] = 0.0;
                for (int j = 0; j < 3; ++j) N[i] += Ct[i][j] * c[j];
                N[i] += G[i] * (c2 - 3.0 * theta);
                N[i] -= eps2 * (c[i] * c2 - S[i]);
            }
            double xi[3];
            or_normals3(cfg->seed, pid[p], step, OR_PURPOSE_COLLISION, 0, xi);
            for (int i = 0; i < 3; ++i) {
                double v = c[i] * E + (1.0 - E) * tau * N[i] + sigma * xi[i];
                cs[3 * (int64_t)p + i] = v;
                sum_cs[i] += v;
                sum_NN += N[i] * N[i];
                sum_cN += c[i] * N[i];
            }
        }
        double cbar[3] = {sum_cs[0] / np, sum_cs[1] / np, sum_cs[2] / np};
        double scale = 1.0;
        if (cfg->conserve == OR_EXACT) {
            double e2 = 0.0;
            for (int32_t p = b; p < e; ++p)
                for (int i = 0; i < 3; ++i) {
                    double d = cs[3 * (int64_t)p + i] - cbar[i];
                    e2 += d * d;
                }
            e2 /= np;
            scale = sqrt(3.0 * theta / e2);
        } else {
            double NN = sum_NN / np, cN = sum_cN / np;
            double a2 = 1.0 + tau / (3.0 * theta) *
                                  (tau * (1.0 - E) * (1.0 - E) * NN + 2.0 * (E - E * E) * cN);
            scale = 1.0 / sqrt(a2);
        }
        if (!isfinite(scale) || !(scale > 0.0)) scale = 1.0;
        for (int32_t p = b; p < e; ++p) {
            vx[p] = store(cfg, (cs[3 * (int64_t)p + 0] - cbar[0]) * scale + U[0]);
            vy[p] = store(cfg, (cs[3 * (int64_t)p + 1] - cbar[1]) * scale + U[1]);
            vz[p] = store(cfg, (cs[3 * (int64_t)p + 2] - cbar[2]) * scale + U[2]);
        }
    }
    free(cs);
}

/* ------------------------------------------------------------------------------------ */
/* Diffuse re-emission from wall w (0: x_lo, 1: x_hi, 2: y_lo, 3: y_hi) at temperature
 * T_w moving with u_w: the inward normal speed has density proportional to
 * v exp(-v^2 / (2 R T_w)), the tangential components are Gaussian about u_w.           */
static void emit(const or_config* cfg, int w, uint32_t pid, uint32_t step, uint32_t bounce,
                 double v[3])
{
    double u[4];
    or_uniforms(cfg->seed, pid, step, OR_PURPOSE_WALL, bounce, u);
    double RT = cfg->kB / cfg->mass * cfg->T_wall[w];
    double vn = sqrt(-2.0 * RT * log(u[0]));
    double rr = sqrt(-2.0 * log(u[1]));
    double za = rr * cos(2.0 * OR_PI * u[2]);
    double zb = rr * sin(2.0 * OR_PI * u[2]);
    double s = sqrt(RT);
    int nax = w / 2;                    /* normal axis */
    double sign = (w % 2 == 0) ? 1.0 : -1.0;
    int ta = (nax == 0) ? 1 : 0;        /* first tangential axis */
    int tb = 2;                         /* second tangential axis */
    v[nax] = sign * vn;
    v[ta] = cfg->u_wall[w][ta] + s * za;
    v[tb] = cfg->u_wall[w][tb] + s * zb;
}

/* Diffuse re-emission from the cylinder surface at (px, py): normal n = (p - c)/R points
 * into the gas; speed along n ~ v exp(-v^2/(2 R T_body)), Gaussian along the in-plane
 * tangent (-n_y, n_x) and along z; the body is at rest. */
static void emit_circle(const or_config* cfg, double px, double py, uint32_t pid, uint32_t step,
                        uint32_t bounce, double v[3])
{
    double u[4];
    or_uniforms(cfg->seed, pid, step, OR_PURPOSE_WALL, bounce, u);
    double RT = cfg->kB / cfg->mass * cfg->T_body;
    double vn = sqrt(-2.0 * RT * log(u[0]));
    double rr = sqrt(-2.0 * log(u[1]));
    double za = rr * cos(2.0 * OR_PI * u[2]);
    double zb = rr * sin(2.0 * OR_PI * u[2]);
    double s = sqrt(RT);
    double nx = (px - cfg->circle[0]) / cfg->circle[2];
    double ny = (py - cfg->circle[1]) / cfg->circle[2];
    double vt = s * za;
    v[0] = vn * nx - vt * ny;
    v[1] = vn * ny + vt * nx;
    v[2] = s * zb;
}

/* Free flight in the open cylinder domain: straight segments between diffuse hits on
 * the circle |p - c| = R; a particle whose end point lies outside the box is deleted.
 * Returns 1 if deleted. */
/* Exchange of one diffuse re-emission at the cylinder, per unit molecular mass, into the
 * bin of the surface angle theta (0 at the rear point, pi at the front; cos theta = n_x):
 * bin b holds the points with cos((b+1) pi / nbins) < n_x <= cos(b pi / nbins), i.e. b is
 * the number of interior edges k = 1 .. nbins-1 with n_x <= cos(k pi / nbins).  Recorded:
 * hits, normal momentum given to the wall v_out.n - v_in.n, tangential momentum given to
 * the wall towards the rear (v_in - v_out).t with t the unit tangent along decreasing
 * theta, energy given to the wall (|v_in|^2 - |v_out|^2) / 2. */
static void wall_record(const or_config* cfg, double px, double py, const double vin[3],
                        const double vout[3], double* wall, int32_t nbins)
{
    double nx = (px - cfg->circle[0]) / cfg->circle[2];
    double ny = (py - cfg->circle[1]) / cfg->circle[2];
    int32_t bin = 0;
    for (int32_t k = 1; k < nbins; ++k)
        if (nx <= cos((double)k * OR_PI / (double)nbins)) bin = k;
    double sgn = ny >= 0.0 ? 1.0 : -1.0;
    double tx = sgn * ny, ty = -sgn * nx;
    double* w = wall + 4 * (int64_t)bin;
    w[0] += 1.0;
    w[1] += (vout[0] * nx + vout[1] * ny) - (vin[0] * nx + vin[1] * ny);
    w[2] += (vin[0] * tx + vin[1] * ty) - (vout[0] * tx + vout[1] * ty);
    w[3] += 0.5 * ((vin[0] * vin[0] + vin[1] * vin[1] + vin[2] * vin[2]) -
                   (vout[0] * vout[0] + vout[1] * vout[1] + vout[2] * vout[2]));
}

static int fly_cylinder(const or_config* cfg, double pos[2], double v[3], uint32_t pid,
                        uint32_t step, double* wall, int32_t nbins)
{
    const double cx = cfg->circle[0], cy = cfg->circle[1], R = cfg->circle[2];
    double trem = cfg->dt;
    for (int bounce = 0;; ++bounce) {
        double dxc = pos[0] - cx, dyc = pos[1] - cy;
        double a = v[0] * v[0] + v[1] * v[1];
        double b = dxc * v[0] + dyc * v[1];
        double c = dxc * dxc + dyc * dyc - R * R;
        int hit = 0;
        double th = 0.0;
        if (c < 0.0) {
            if (b < 0.0) {                    /* inside (rounding) and moving in: hit now */
                double d = sqrt(dxc * dxc + dyc * dyc);
                if (d > 0.0) {
                    pos[0] = cx + R * (dxc / d);
                    pos[1] = cy + R * (dyc / d);
                }
                hit = 1;
            }
        } else if (b < 0.0 && a > 0.0) {
            double disc = b * b - a * c;
            if (disc >= 0.0) {
                double q = -b + sqrt(disc);
                double t = c / q;
                if (t <= trem) {
                    hit = 1;
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
        if (bounce == cfg->max_bounces) return 0;      /* stop on the surface */
        double vin[3] = {v[0], v[1], v[2]};
        emit_circle(cfg, pos[0], pos[1], pid, step, (uint32_t)bounce, v);
        for (int i = 0; i < 3; ++i) v[i] = store(cfg, v[i]);
        if (wall) wall_record(cfg, pos[0], pos[1], vin, v, wall, nbins);
        trem = trem - th;
    }
    double x1 = cfg->x0 + cfg->lx, y1 = cfg->y0 + cfg->ly;
    return (pos[0] < cfg->x0 || pos[0] > x1 || pos[1] < cfg->y0 || pos[1] > y1) ? 1 : 0;
}

void or_move(const or_config* cfg, int64_t n, double* x, double* y, double* vx, double* vy,
             double* vz, const uint32_t* pid, int32_t* key, uint32_t step)
{
    or_move_wall(cfg, n, x, y, vx, vy, vz, pid, key, step, NULL, 0);
}

void or_move_wall(const or_config* cfg, int64_t n, double* x, double* y, double* vx,
                  double* vy, double* vz, const uint32_t* pid, int32_t* key, uint32_t step,
                  double* wall, int32_t nbins)
{
    if (cfg->geometry == OR_CYLINDER2D) {
        int32_t ncell = cfg->nx * cfg->ny;
        for (int64_t p = 0; p < n; ++p) {
            double pos[2] = {x[p], y[p]};
            double v[3] = {vx[p], vy[p], vz[p]};
            int gone = fly_cylinder(cfg, pos, v, pid[p], step, wall, nbins);
            x[p] = store(cfg, pos[0]);
            y[p] = store(cfg, pos[1]);
            vx[p] = v[0]; vy[p] = v[1]; vz[p] = v[2];
            or_keys(cfg, 1, &x[p], &y[p], &key[p]);
            if (gone) key[p] = ncell;
        }
        return;
    }
    int two_d = (cfg->geometry == OR_CAVITY2D);
    double lo[2] = {cfg->x0, cfg->y0};
    double hi[2] = {cfg->x0 + cfg->lx, cfg->y0 + cfg->ly};
#pragma omp parallel for schedule(static) if (n > 4096)
    for (int64_t p = 0; p < n; ++p) {
        double pos[2] = {x[p], two_d ? y[p] : 0.0};
        double v[3] = {vx[p], vy[p], vz[p]};
        double trem = cfg->dt;
        int nax = two_d ? 2 : 1;
        for (int bounce = 0;; ++bounce) {
            double end[2] = {pos[0] + v[0] * trem, pos[1] + v[1] * trem};
            int wall = -1;
            double th = 0.0;
            for (int a = 0; a < nax; ++a) {
                if (end[a] < lo[a] && v[a] < 0.0) {
                    double t = (lo[a] - pos[a]) / v[a];
                    if (t < 0.0) t = 0.0;
                    if (wall < 0 || t < th) { wall = 2 * a; th = t; }
                }
                if (end[a] > hi[a] && v[a] > 0.0) {
                    double t = (hi[a] - pos[a]) / v[a];
                    if (t < 0.0) t = 0.0;
                    if (wall < 0 || t < th) { wall = 2 * a + 1; th = t; }
                }
            }
            if (wall < 0) {
                for (int a = 0; a < nax; ++a) pos[a] = end[a];
                break;
            }
            if (bounce == cfg->max_bounces) {
                for (int a = 0; a < nax; ++a) {
                    pos[a] = end[a];
                    if (pos[a] < lo[a]) pos[a] = lo[a];
                    if (pos[a] > hi[a]) pos[a] = hi[a];
                }
                break;
            }
            if (th > trem) th = trem;
            int wa = wall / 2;
            for (int a = 0; a < nax; ++a)
                pos[a] = (a == wa) ? ((wall % 2 == 0) ? lo[a] : hi[a]) : pos[a] + v[a] * th;
            emit(cfg, wall, pid[p], step, (uint32_t)bounce, v);
            for (int i = 0; i < 3; ++i) v[i] = store(cfg, v[i]);
            trem = trem - th;
        }
        x[p] = store(cfg, pos[0]);
        if (two_d) y[p] = store(cfg, pos[1]);
        vx[p] = v[0]; vy[p] = v[1]; vz[p] = v[2];
    }
    or_keys(cfg, n, x, y, key);
}


/* ------------------------------------------------------------------------------------ */
int64_t or_inject(const or_config* cfg, uint32_t step, uint32_t* pid_next, int64_t room,
                  double* x, double* y, double* vx, double* vy, double* vz, uint32_t* pid,
                  int32_t* key)
{
    double RT = cfg->kB / cfg->mass * cfg->T_inf;
    double umag = sqrt(cfg->u_inf[0] * cfg->u_inf[0] + cfg->u_inf[1] * cfg->u_inf[1] +
                       cfg->u_inf[2] * cfg->u_inf[2]);
    double w = (umag + 4.0 * sqrt(2.0 * RT)) * cfg->dt;
    double x0 = cfg->x0, y0 = cfg->y0, x1 = cfg->x0 + cfg->lx, y1 = cfg->y0 + cfg->ly;
    double reg[4][4] = {{x0 - w, x0, y0 - w, y1 + w}, {x1, x1 + w, y0 - w, y1 + w},
                        {x0, x1, y0 - w, y0}, {x0, x1, y1, y1 + w}};
    double s = sqrt(RT);
    int64_t total = 0, out = 0;
    for (int r = 0; r < 4; ++r) {
        double xa = reg[r][0], xb = reg[r][1], ya = reg[r][2], yb = reg[r][3];
        double lam = cfg->n_inf * ((xb - xa) * (yb - ya)) * cfg->depth / cfg->fnum;
        double base = floor(lam);
        double uc[4];
        or_uniforms(cfg->seed, (uint32_t)r, step, OR_PURPOSE_INJECT, 1, uc);
        int64_t K = (int64_t)base + (uc[0] < lam - base ? 1 : 0);
        for (int64_t k = 0; k < K; ++k) {
            uint32_t id = *pid_next + (uint32_t)(total + k);
            double d0[4], d1[4];
            or_uniforms(cfg->seed, id, step, OR_PURPOSE_INJECT, 0, d0);
            or_uniforms(cfg->seed, id, step, OR_PURPOSE_INJECT, 2, d1);
            double px = xa + d0[0] * (xb - xa);
            double py = ya + d0[1] * (yb - ya);
            double r0 = sqrt(-2.0 * log(d0[2]));
            double v0 = cfg->u_inf[0] + s * (r0 * cos(2.0 * OR_PI * d0[3]));
            double v1 = cfg->u_inf[1] + s * (r0 * sin(2.0 * OR_PI * d0[3]));
            double v2 = cfg->u_inf[2] + s * (sqrt(-2.0 * log(d1[0])) * cos(2.0 * OR_PI * d1[1]));
            double ex = px + v0 * cfg->dt;
            double ey = py + v1 * cfg->dt;
            if (ex >= x0 && ex <= x1 && ey >= y0 && ey <= y1) {
                if (out >= room) return -1;
                x[out] = store(cfg, ex);
                y[out] = store(cfg, ey);
                vx[out] = store(cfg, v0);
                vy[out] = store(cfg, v1);
                vz[out] = store(cfg, v2);
                pid[out] = id;
                or_keys(cfg, 1, &x[out], &y[out], &key[out]);
                ++out;
            }
        }
        total += K;
    }
    *pid_next += (uint32_t)total;
    return out;
}

/* ------------------------------------------------------------------------------------ */
void or_sample(int32_t ncell, const int32_t* offsets, const double* vx, const double* vy,
               const double* vz, double* samp)
{
    #pragma omp parallel for schedule(dynamic, 16) if (ncell > 64)
    for (int32_t cell = 0; cell < ncell; ++cell) {
        double* s = samp + (int64_t)cell * OR_SAMP_STRIDE;
        for (int32_t p = offsets[cell]; p < offsets[cell + 1]; ++p) {
            double v[3] = {vx[p], vy[p], vz[p]};
            double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
            s[0] += 1.0;
            for (int i = 0; i < 3; ++i) s[1 + i] += v[i];
            for (int i = 0; i < 3; ++i)
                for (int j = i; j < 3; ++j) s[4 + sym2(i, j)] += v[i] * v[j];
            for (int i = 0; i < 3; ++i) s[10 + i] += v[i] * v2;
        }
        s[13] += 1.0;
    }
}

/* ------------------------------------------------------------------------------------ */
static void permute_d(double* a, const int64_t* perm, int64_t n, double* tmp)
{
#pragma omp parallel for schedule(static) if (n > 4096)
    for (int64_t j = 0; j < n; ++j) tmp[j] = a[perm[j]];
    memcpy(a, tmp, sizeof(double) * (size_t)n);
}

int or_run(const or_config* cfg, int64_t n, double* x, double* y, double* vx, double* vy,
           double* vz, uint32_t* pid, int32_t* key, uint32_t step0, int32_t nsteps,
           uint32_t n_skip, double* mom, double* rec, int32_t* status, double* samp)
{
    int32_t ncell = cfg->nx * cfg->ny;
    int64_t* perm = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int32_t* offsets = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ncell + 1));
    double* tmp = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    uint32_t* tmpu = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    if (!perm || !offsets || !tmp || !tmpu) {
        free(perm); free(offsets); free(tmp); free(tmpu);
        return -1;
    }
    for (int32_t s = 0; s < nsteps; ++s) {
        uint32_t step = step0 + (uint32_t)s;
        or_bin(ncell, n, key, perm, offsets);
        permute_d(x, perm, n, tmp);
        if (cfg->geometry == OR_CAVITY2D) permute_d(y, perm, n, tmp);
        permute_d(vx, perm, n, tmp);
        permute_d(vy, perm, n, tmp);
        permute_d(vz, perm, n, tmp);
        for (int64_t j = 0; j < n; ++j) tmpu[j] = pid[perm[j]];
        memcpy(pid, tmpu, sizeof(uint32_t) * (size_t)n);
        or_moments(ncell, offsets, vx, vy, vz, mom);
        if (step >= n_skip && samp) or_sample(ncell, offsets, vx, vy, vz, samp);
        or_closure(cfg, ncell, mom, NULL, rec, status);
        or_update(cfg, ncell, offsets, vx, vy, vz, pid, mom, rec, step);
        or_move(cfg, n, x, y, vx, vy, vz, pid, key, step);
    }
    free(perm); free(offsets); free(tmp); free(tmpu);
    return 0;
}

int or_run_open(const or_config* cfg, int64_t capacity, int64_t* n, double* x, double* y,
                double* vx, double* vy, double* vz, uint32_t* pid, int32_t* key,
                uint32_t* pid_next, uint32_t step0, int32_t nsteps, uint32_t n_skip,
                double* mom, double* rec, int32_t* status, double* samp)
{
    int32_t ncell = cfg->nx * cfg->ny;
    size_t cap = (size_t)(capacity > 0 ? capacity : 1);
    int64_t* perm = (int64_t*)malloc(sizeof(int64_t) * cap);
    int32_t* offsets = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ncell + 1));
    double* tmp = (double*)malloc(sizeof(double) * cap);
    uint32_t* tmpu = (uint32_t*)malloc(sizeof(uint32_t) * cap);
    double* vol = (double*)malloc(sizeof(double) * (size_t)ncell);
    double* nvol = (double*)malloc(sizeof(double) * (size_t)ncell);
    if (!perm || !offsets || !tmp || !tmpu || !vol || !nvol) {
        free(perm); free(offsets); free(tmp); free(tmpu); free(vol); free(nvol);
        return -1;
    }
    or_cell_volumes(cfg, vol);
    double full = cfg->dx * cfg->dy * cfg->depth;
    for (int32_t c = 0; c < ncell; ++c) nvol[c] = cfg->fnum / (vol[c] > 0.0 ? vol[c] : full);
    int rc = 0;
    for (int32_t s = 0; s < nsteps && rc == 0; ++s) {
        uint32_t step = step0 + (uint32_t)s;
        or_bin(ncell, *n, key, perm, offsets);
        int64_t live = offsets[ncell];
        double* arrs[5] = {x, y, vx, vy, vz};
        for (int a = 0; a < 5; ++a) {
            for (int64_t j = 0; j < live; ++j) tmp[j] = arrs[a][perm[j]];
            memcpy(arrs[a], tmp, sizeof(double) * (size_t)live);
        }
        for (int64_t j = 0; j < live; ++j) tmpu[j] = pid[perm[j]];
        memcpy(pid, tmpu, sizeof(uint32_t) * (size_t)live);
        *n = live;
        or_moments(ncell, offsets, vx, vy, vz, mom);
        if (step >= n_skip && samp) or_sample(ncell, offsets, vx, vy, vz, samp);
        or_closure(cfg, ncell, mom, nvol, rec, status);
        or_update(cfg, ncell, offsets, vx, vy, vz, pid, mom, rec, step);
        or_move(cfg, live, x, y, vx, vy, vz, pid, key, step);
        int64_t add = or_inject(cfg, step, pid_next, capacity - live, x + live, y + live,
                                vx + live, vy + live, vz + live, pid + live, key + live);
        if (add < 0) rc = -2;
        else *n = live + add;
    }
    free(perm); free(offsets); free(tmp); free(tmpu); free(vol); free(nvol);
    return rc;
}
