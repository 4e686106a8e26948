// fp_api.hip -- context management and argument checking of the C ABI (include/fp.h).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <new>
#include <vector>

#include "fp_internal.h"

namespace fpg {

int set_err(fp_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    return code;
}

int check_launch(fp_ctx* c, const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return set_err(c, FP_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return FP_OK;
}

}  // namespace fpg

using namespace fpg;

static bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

static int validate(const fp_config* g, std::string& why) {
    if (g->geometry != FP_COUETTE1D && g->geometry != FP_CAVITY2D && g->geometry != FP_CYLINDER2D)
        return why = "geometry", 0;
    if (g->precision != FP_F32 && g->precision != FP_F64) return why = "precision", 0;
    if (g->conserve != FP_EXACT && g->conserve != FP_PAPER) return why = "conserve", 0;
    if (g->nx < 1 || g->ny < 1 || (int64_t)g->nx * g->ny > (1 << 28)) return why = "grid", 0;
    if (g->geometry == FP_COUETTE1D && g->ny != 1) return why = "1-D grid needs ny = 1", 0;
    // at most 2^29 - 64 slots: byte offsets into the FP64 particle arrays stay below 2^32
    if (g->capacity < 0 || g->capacity > ((int64_t)1 << 29) - 64) return why = "capacity", 0;
    if (g->max_bounces < 0 || g->max_bounces > 1000) return why = "max_bounces", 0;
    if (g->lanes != 0 && g->lanes != 4 && g->lanes != 8 && g->lanes != 16 && g->lanes != 32 &&
        g->lanes != 64)
        return why = "lanes", 0;
    if ((g->moment_order != 0 && g->moment_order != 3 && g->moment_order != 5) || g->reserved0 != 0)
        return why = "moment_order", 0;
    if (!finite_pos(g->dx) || !finite_pos(g->dy) || !finite_pos(g->lx) || !finite_pos(g->ly) ||
        !finite_pos(g->dt) || !finite_pos(g->kB) || !finite_pos(g->mass) ||
        !finite_pos(g->mu_ref) || !finite_pos(g->T_ref) || !finite_pos(g->fnum_over_vol))
        return why = "non-positive physical parameter", 0;
    for (int w = 0; w < 4; ++w)
        if (!finite_pos(g->T_wall[w])) return why = "wall temperature", 0;
    if (!(g->eps_hat >= 0.0) || !(g->pivot_tol >= 0.0)) return why = "eps_hat/pivot_tol", 0;
    if (g->geometry == FP_CYLINDER2D) {
        if (!(g->circle[2] >= 0.0) || !finite_pos(g->T_body) || !finite_pos(g->n_inf) ||
            !finite_pos(g->T_inf) || !finite_pos(g->fnum) || !finite_pos(g->depth))
            return why = "cylinder parameters", 0;
        for (int k = 0; k < 3; ++k)
            if (!std::isfinite(g->u_inf[k]) || !std::isfinite(g->circle[k])) return why = "cylinder", 0;
    }
    return 1;
}

// ---- exact gas volume of the cells of the cylinder domain ------------------------------
// Coordinates relative to the circle centre.  The covered length of a vertical line at x
// is min(yb, h) - max(ya, -h), h = sqrt(R^2 - x^2); its integral over the cell is split
// where the chord ends cross the cell edges, and every piece uses
//   I(x) = int_{-R}^{x} h dX = R^2 (phi - sin(phi) cos(phi)) / 2,  phi = acos(-x / R),
// which, unlike the arcsine form, keeps its accuracy next to x = +-R.
static double chord_int(double x, double R) {
    const double t = std::max(-1.0, std::min(1.0, -x / R));
    const double phi = std::acos(t);
    return 0.5 * R * R * (phi - std::sin(phi) * std::cos(phi));
}

static double covered_area(double xa, double xb, double ya, double yb, double R) {
    const double lo = std::max(xa, -R), hi = std::min(xb, R);
    if (!(lo < hi)) return 0.0;
    double br[6];
    int nb = 0;
    br[nb++] = lo;
    br[nb++] = hi;
    for (double y : {ya, yb})
        if (std::fabs(y) < R) {
            const double a = std::sqrt(R * R - y * y);
            if (-a > lo && -a < hi) br[nb++] = -a;
            if (a > lo && a < hi) br[nb++] = a;
        }
    std::sort(br, br + nb);
    double tot = 0.0;
    for (int k = 0; k + 1 < nb; ++k) {
        const double p = br[k], q = br[k + 1];
        if (!(q > p)) continue;
        const double m = 0.5 * (p + q);
        const double h = std::sqrt(std::max(R * R - m * m, 0.0));
        if (std::min(yb, h) <= std::max(ya, -h)) continue;
        const double dI = chord_int(q, R) - chord_int(p, R);
        const double up = h < yb ? dI : yb * (q - p);      // integral of min(yb, h)
        const double dn = -h > ya ? -dI : ya * (q - p);    // integral of max(ya, -h)
        tot += up - dn;
    }
    return tot;
}

static void gas_volumes(const fp_config& g, std::vector<double>& vol) {
    const double cx = g.circle[0], cy = g.circle[1], R = g.circle[2];
    const double full = g.dx * g.dy;
    vol.assign((size_t)g.nx * g.ny, full);
    if (g.geometry != FP_CYLINDER2D) return;
    for (int32_t ky = 0; ky < g.ny; ++ky)
        for (int32_t kx = 0; kx < g.nx; ++kx) {
            const double xa = g.x0 + kx * g.dx, xb = xa + g.dx;
            const double ya = g.y0 + ky * g.dy, yb = ya + g.dy;
            double v = full - (R > 0.0 ? covered_area(xa - cx, xb - cx, ya - cy, yb - cy, R) : 0.0);
            if (v < 1e-12 * full) v = 0.0;
            vol[(size_t)ky * g.nx + kx] = v * g.depth;
        }
}

template <typename T>
static bool dalloc(T** p, size_t count) {
    return hipMalloc((void**)p, sizeof(T) * (count ? count : 1)) == hipSuccess;
}

extern "C" int fp_init(const fp_config* cfg, fp_ctx** out) {
    if (!cfg || !out) return FP_EINVAL;
    *out = nullptr;
    std::string why;
    if (!validate(cfg, why)) {
        fprintf(stderr, "fp_init: invalid configuration (%s)\n", why.c_str());
        return FP_EINVAL;
    }
    fp_ctx* c = new (std::nothrow) fp_ctx();
    if (!c) return FP_ENOMEM;
    c->cfg = *cfg;
    c->ncell = cfg->nx * cfg->ny;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return FP_EDEVICE;
    }
    const size_t nc = (size_t)c->ncell + 1;
    const size_t cap = (size_t)cfg->capacity;
    bool ok = dalloc(&c->cnt, nc) && dalloc(&c->ccnt, nc) && dalloc(&c->coff, nc + 1) &&
              dalloc(&c->ccur, nc) && dalloc(&c->cpair, 2 * nc) && dalloc(&c->cwave, cap) &&
              dalloc(&c->cmask, cap) &&
              dalloc(&c->gidx, cap) && dalloc(&c->blocksum, 2 * 8192) &&
              dalloc(&c->errcount, 2) && dalloc(&c->ncnt, 9 * (nc - 1) + 1) && dalloc(&c->farn, 1) &&
              dalloc(&c->bidx, cap) && dalloc(&c->pend, nc) && dalloc(&c->stepc, 1);
    // the sort counters start at zero; every fp_bin / fp_rebin leaves them zero again
    if (ok) ok = hipMemset(c->errcount, 0, 2 * sizeof(unsigned long long)) == hipSuccess &&
                 hipMemset(c->cnt, 0, sizeof(int32_t) * nc) == hipSuccess &&
                 hipMemset(c->ccnt, 0, sizeof(int32_t) * nc) == hipSuccess &&
                 hipMemset(c->ccur, 0, sizeof(int32_t) * nc) == hipSuccess &&
                 hipMemset(c->cpair, 0, sizeof(int32_t) * 2 * nc) == hipSuccess &&
                 hipMemset(c->farn, 0, sizeof(int32_t)) == hipSuccess &&
                 hipMemset(c->stepc, 0, sizeof(uint32_t)) == hipSuccess;
    if (ok && cfg->geometry == FP_CYLINDER2D) {
        std::vector<double> vol, nvol;
        gas_volumes(*cfg, vol);
        const double full = cfg->dx * cfg->dy * cfg->depth;
        nvol.resize(vol.size());
        for (size_t i = 0; i < vol.size(); ++i) nvol[i] = cfg->fnum / (vol[i] > 0.0 ? vol[i] : full);
        ok = dalloc(&c->vol, vol.size()) && dalloc(&c->nvol, vol.size()) && dalloc(&c->inj, 16);
        if (ok) ok = hipMemcpy(c->vol, vol.data(), sizeof(double) * vol.size(), hipMemcpyHostToDevice) == hipSuccess;
        if (ok) ok = hipMemcpy(c->nvol, nvol.data(), sizeof(double) * vol.size(), hipMemcpyHostToDevice) == hipSuccess;
        // inflow rectangles: a frame of width (|u_inf| + 4 sqrt(2 R T_inf)) dt around the box
        const double RT = cfg->kB / cfg->mass * cfg->T_inf;
        const double um = std::sqrt(cfg->u_inf[0] * cfg->u_inf[0] + cfg->u_inf[1] * cfg->u_inf[1] +
                                    cfg->u_inf[2] * cfg->u_inf[2]);
        const double w = (um + 4.0 * std::sqrt(2.0 * RT)) * cfg->dt;
        const double x0 = cfg->x0, y0 = cfg->y0, x1 = cfg->x0 + cfg->lx, y1 = cfg->y0 + cfg->ly;
        const double rect[4][4] = {{x0 - w, x0, y0 - w, y1 + w}, {x1, x1 + w, y0 - w, y1 + w},
                                   {x0, x1, y0 - w, y0}, {x0, x1, y1, y1 + w}};
        c->inj_slot0[0] = 0;
        for (int r = 0; r < 4; ++r) {
            for (int k = 0; k < 4; ++k) c->inj_rect[r][k] = rect[r][k];
            c->inj_lambda[r] = cfg->n_inf * ((rect[r][1] - rect[r][0]) * (rect[r][3] - rect[r][2])) *
                               cfg->depth / cfg->fnum;
            const double slots = std::floor(c->inj_lambda[r]) + 1.0;
            if (!(slots < 1e8)) ok = false;
            c->inj_slot0[r + 1] = c->inj_slot0[r] + (ok ? (int32_t)slots : 0);
        }
    } else if (ok) {
        std::vector<double> vol;
        gas_volumes(*cfg, vol);
        ok = dalloc(&c->vol, vol.size()) &&
             hipMemcpy(c->vol, vol.data(), sizeof(double) * vol.size(), hipMemcpyHostToDevice) == hipSuccess;
    }
    if (ok) ok = hipDeviceSynchronize() == hipSuccess;
    if (!ok) {
        fp_destroy(c);
        return FP_ENOMEM;
    }
    *out = c;
    return FP_OK;
}

extern "C" void fp_destroy(fp_ctx* c) {
    if (!c) return;
    (void)hipDeviceSynchronize();
    (void)hipFree(c->cnt);
    (void)hipFree(c->ccnt);
    (void)hipFree(c->coff);
    (void)hipFree(c->ccur);
    (void)hipFree(c->cpair);
    (void)hipFree(c->cwave);
    (void)hipFree(c->cmask);
    (void)hipFree(c->gidx);
    (void)hipFree(c->blocksum);
    (void)hipFree(c->errcount);
    (void)hipFree(c->ncnt);
    (void)hipFree(c->farn);
    (void)hipFree(c->pend);
    (void)hipFree(c->stepc);
    (void)hipFree(c->bidx);
    (void)hipFree(c->vol);
    (void)hipFree(c->nvol);
    for (void* q : {(void*)c->amr_state, (void*)c->amr_flag, (void*)c->amr_age, (void*)c->amr_sum,
                    (void*)c->leafmap, (void*)c->leafmap_old, (void*)c->leaf_node, (void*)c->leaf_node_old,
                    (void*)c->amr_first, (void*)c->amr_part, (void*)c->fine_vol, (void*)c->vol_old,
                    (void*)c->samp_old, (void*)c->wall_edge})
        (void)hipFree(q);
    (void)hipFree(c->inj);
    delete c;
}

extern "C" const char* fp_last_error(const fp_ctx* c) { return c ? c->err.c_str() : ""; }

extern "C" int64_t fp_error_count(fp_ctx* c, hipStream_t s) {
    if (!c) return FP_EINVAL;
    unsigned long long v = 0;
    if (hipMemcpyAsync(&v, c->errcount, sizeof(v), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return set_err(c, FP_EDEVICE, "fp_error_count: copy failed");
    return (int64_t)v;
}

static bool particles_ok(const fp_ctx* c, const fp_particles* p, bool need_pos) {
    if (!p || p->n < 0 || p->n > c->cfg.capacity) return false;
    if (p->n_dev && (p->capacity < p->n || p->capacity > c->cfg.capacity)) return false;
    if (slots_of(p) == 0) return true;
    if (!p->vx || !p->vy || !p->vz || !p->pid || !p->key) return false;
    if (need_pos && (!p->x || (c->cfg.geometry != FP_COUETTE1D && !p->y))) return false;
    return true;
}

extern "C" int fp_bin(fp_ctx* c, const fp_particles* src, fp_particles* dst, int32_t* offsets,
                      int32_t* perm, hipStream_t s) {
    if (!c || !offsets || !particles_ok(c, src, true) || !dst)
        return set_err(c, FP_EINVAL, "fp_bin: bad argument");
    if (slots_of(src) > 0 && (!dst->vx || !dst->vy || !dst->vz || !dst->pid || !dst->key || !dst->x ||
                              (c->cfg.geometry != FP_COUETTE1D && !dst->y)))
        return set_err(c, FP_EINVAL, "fp_bin: bad destination");
    if (dst->n_dev && dst->n_dev == src->n_dev)
        return set_err(c, FP_EINVAL, "fp_bin: src and dst share their device count");
    if (src->vx == dst->vx || src->x == dst->x || src->pid == dst->pid)
        return set_err(c, FP_EINVAL, "fp_bin: src and dst alias");
    const int rc = launch_bin(c, src, dst, offsets, perm, s);
    if (rc == FP_OK) c->sort_epoch = c->amr_epoch;
    return rc;
}

extern "C" int fp_rebin(fp_ctx* c, const fp_particles* src, const int32_t* src_offsets,
                        fp_particles* dst, int32_t* offsets, int32_t* perm, double* mom,
                        double* samp, hipStream_t s) {
    if (!c || !offsets || !src_offsets || !particles_ok(c, src, true) || !dst || (samp && !mom))
        return set_err(c, FP_EINVAL, "fp_rebin: bad argument");
    if (samp && samp == mom) return set_err(c, FP_EINVAL, "fp_rebin: samp and mom alias");
    if (c->amr_L >= 0 && c->sort_epoch != c->amr_epoch)
        return set_err(c, FP_EINVAL, "fp_rebin: the leaves changed since the last sort (fp_bin first)");
    if (slots_of(src) > 0 && (!dst->vx || !dst->vy || !dst->vz || !dst->pid || !dst->key || !dst->x ||
                              (c->cfg.geometry != FP_COUETTE1D && !dst->y)))
        return set_err(c, FP_EINVAL, "fp_rebin: bad destination");
    if (dst->n_dev && dst->n_dev == src->n_dev)
        return set_err(c, FP_EINVAL, "fp_rebin: src and dst share their device count");
    if (src->vx == dst->vx || src->x == dst->x || src->pid == dst->pid)
        return set_err(c, FP_EINVAL, "fp_rebin: src and dst alias");
    if (src_offsets == offsets) return set_err(c, FP_EINVAL, "fp_rebin: src_offsets and offsets alias");
    return launch_rebin(c, src, src_offsets, dst, offsets, perm, mom, samp, s);
}

extern "C" int fp_moments(fp_ctx* c, const fp_particles* p, const int32_t* offsets, double* mom,
                          hipStream_t s) {
    if (!c || !offsets || !mom || !particles_ok(c, p, false))
        return set_err(c, FP_EINVAL, "fp_moments: bad argument");
    return launch_moments(c, p, offsets, mom, nullptr, nullptr, s);
}

extern "C" int fp_moments_sample(fp_ctx* c, const fp_particles* p, const int32_t* offsets, double* mom,
                                 double* samp0, double* samp1, hipStream_t s) {
    if (!c || !offsets || !mom || !samp0 || samp1 == samp0 || !particles_ok(c, p, false))
        return set_err(c, FP_EINVAL, "fp_moments_sample: bad argument");
    return launch_moments(c, p, offsets, mom, samp0, samp1, s);
}

extern "C" int fp_closure_solve(fp_ctx* c, const double* mom, double* rec, int32_t* status,
                                hipStream_t s) {
    if (!c || !mom || !rec || !status) return set_err(c, FP_EINVAL, "fp_closure_solve: bad argument");
    if (c->cfg.moment_order == 3)
        return set_err(c, FP_EINVAL, "fp_closure_solve: the context gathers moments through third order only");
    return launch_closure(c, mom, rec, status, s);
}

extern "C" int fp_step(fp_ctx* c, fp_particles* p, const int32_t* offsets, const double* mom,
                       const double* rec, uint64_t step, uint32_t flags, hipStream_t s) {
    if (!c || (flags & ~7u) || !flags) return set_err(c, FP_EINVAL, "fp_step: bad flags");
    if (!particles_ok(c, p, (flags & (FP_STEP_MOVE | FP_STEP_KEYS)) != 0))
        return set_err(c, FP_EINVAL, "fp_step: bad particles");
    if ((flags & FP_STEP_COLLIDE) && (!offsets || !mom || !rec))
        return set_err(c, FP_EINVAL, "fp_step: COLLIDE needs offsets, mom and rec");
    if ((flags & FP_STEP_KEYS) && (flags & FP_STEP_MOVE))
        return set_err(c, FP_EINVAL, "fp_step: MOVE already writes keys");
    if (step > 0xFFFFFFFFull) return set_err(c, FP_EINVAL, "fp_step: step beyond 2^32");
    return launch_step(c, p, offsets, mom, rec, step, flags, nullptr, s);
}

extern "C" int fp_step_dev(fp_ctx* c, fp_particles* p, const int32_t* offsets, const double* mom,
                           const double* rec, const uint32_t* step_dev, uint32_t flags,
                           hipStream_t s) {
    if (!c || !step_dev || (flags & ~15u) || !(flags & 7u))
        return set_err(c, FP_EINVAL, "fp_step_dev: bad argument");
    if (!particles_ok(c, p, (flags & (FP_STEP_MOVE | FP_STEP_KEYS)) != 0))
        return set_err(c, FP_EINVAL, "fp_step_dev: bad particles");
    if ((flags & FP_STEP_COLLIDE) && (!offsets || !mom || !rec))
        return set_err(c, FP_EINVAL, "fp_step_dev: COLLIDE needs offsets, mom and rec");
    if ((flags & FP_STEP_KEYS) && (flags & FP_STEP_MOVE))
        return set_err(c, FP_EINVAL, "fp_step_dev: MOVE already writes keys");
    return launch_step(c, p, offsets, mom, rec, 0, flags, step_dev, s);
}

extern "C" int fp_counter_add(fp_ctx* c, uint32_t* ctr, uint32_t inc, hipStream_t s) {
    if (!c || !ctr) return set_err(c, FP_EINVAL, "fp_counter_add: bad argument");
    return launch_counter_add(c, ctr, inc, s);
}

extern "C" int fp_diagnostics(fp_ctx* c, const double* samp, double theta_inf, double n_inf,
                              double dg_inf, double* diag, hipStream_t s) {
    if (!c || !samp || !diag || !(theta_inf > 0.0) || !(n_inf > 0.0) || !std::isfinite(dg_inf))
        return set_err(c, FP_EINVAL, "fp_diagnostics: bad argument");
    return launch_diagnostics(c, samp, theta_inf, n_inf, dg_inf, diag, s);
}

extern "C" int fp_wall_sampling(fp_ctx* c, double* sums, int32_t nbins) {
    if (!c) return FP_EINVAL;
    if (c->cfg.geometry != FP_CYLINDER2D)
        return set_err(c, FP_EINVAL, "fp_wall_sampling: the cylinder domain only");
    if (sums && (nbins < 1 || nbins > 65536)) return set_err(c, FP_EINVAL, "fp_wall_sampling: nbins");
    c->wall = nullptr;
    c->wall_nbins = 0;
    if (!sums) return FP_OK;
    // bin edges by the cosine of the surface angle (host cosines, copied once)
    std::vector<double> edge((size_t)nbins + 1);
    for (int32_t k = 0; k <= nbins; ++k) edge[k] = std::cos((double)k * 3.14159265358979323846 / (double)nbins);
    (void)hipFree(c->wall_edge);
    c->wall_edge = nullptr;
    if (hipMalloc((void**)&c->wall_edge, sizeof(double) * edge.size()) != hipSuccess ||
        hipMemcpy(c->wall_edge, edge.data(), sizeof(double) * edge.size(), hipMemcpyHostToDevice) != hipSuccess)
        return set_err(c, FP_ENOMEM, "fp_wall_sampling: allocation failed");
    c->wall = sums;
    c->wall_nbins = nbins;
    return FP_OK;
}

extern "C" int fp_surface_coefficients(fp_ctx* c, const double* sums, int32_t nbins, double t_total,
                                       double* out, hipStream_t s) {
    if (!c || !sums || !out || nbins < 1 || nbins > 65536 || !(t_total > 0.0))
        return set_err(c, FP_EINVAL, "fp_surface_coefficients: bad argument");
    if (c->cfg.geometry != FP_CYLINDER2D || !(c->cfg.n_inf > 0.0))
        return set_err(c, FP_EINVAL, "fp_surface_coefficients: needs the cylinder's free stream");
    const double U2 = c->cfg.u_inf[0] * c->cfg.u_inf[0] + c->cfg.u_inf[1] * c->cfg.u_inf[1] +
                      c->cfg.u_inf[2] * c->cfg.u_inf[2];
    if (!(U2 > 0.0)) return set_err(c, FP_EINVAL, "fp_surface_coefficients: free stream at rest");
    return launch_surface(c, sums, nbins, t_total, out, s);
}

extern "C" int fp_sample_high(fp_ctx* c, const double* mom, double* hsamp, hipStream_t s) {
    if (!c || !mom || !hsamp || (const double*)hsamp == mom)
        return set_err(c, FP_EINVAL, "fp_sample_high: bad argument");
    if (c->cfg.moment_order == 3)
        return set_err(c, FP_EINVAL, "fp_sample_high: the records hold moments through third order");
    return launch_sample_high(c, mom, hsamp, s);
}

extern "C" int fp_high_order(fp_ctx* c, const double* hsamp, double* out, hipStream_t s) {
    if (!c || !hsamp || !out) return set_err(c, FP_EINVAL, "fp_high_order: bad argument");
    return launch_high_order(c, hsamp, out, s);
}

extern "C" int fp_sample(fp_ctx* c, const double* mom, double* samp, hipStream_t s) {
    if (!c || !mom || !samp) return set_err(c, FP_EINVAL, "fp_sample: bad argument");
    return launch_sample(c, mom, samp, s);
}

extern "C" int64_t fp_inject_slots(const fp_ctx* c) {
    if (!c || c->cfg.geometry != FP_CYLINDER2D) return 0;
    return c->inj_slot0[4];
}

extern "C" int fp_inject(fp_ctx* c, fp_particles* p, int64_t at, uint32_t* pid_next,
                         uint64_t step, hipStream_t s) {
    if (!c || !p || !pid_next || c->cfg.geometry != FP_CYLINDER2D)
        return set_err(c, FP_EINVAL, "fp_inject: bad argument or geometry");
    if (at < 0 || at + c->inj_slot0[4] > c->cfg.capacity)
        return set_err(c, FP_ECAPACITY, "fp_inject: capacity exceeded");
    if (!p->x || !p->y || !p->vx || !p->vy || !p->vz || !p->pid || !p->key)
        return set_err(c, FP_EINVAL, "fp_inject: bad particles");
    if (step > 0xFFFFFFFFull) return set_err(c, FP_EINVAL, "fp_inject: step beyond 2^32");
    return launch_inject(c, p, at, pid_next, (uint32_t)step, nullptr, nullptr, s);
}

extern "C" int fp_inject_dev(fp_ctx* c, fp_particles* p, uint32_t* pid_next, uint32_t* step_dev,
                             uint32_t flags, hipStream_t s) {
    if (!c || !p || !pid_next || !step_dev || c->cfg.geometry != FP_CYLINDER2D || (flags & ~FP_STEP_ADVANCE))
        return set_err(c, FP_EINVAL, "fp_inject_dev: bad argument or geometry");
    if (!p->n_dev || p->capacity < 1 || p->capacity > c->cfg.capacity)
        return set_err(c, FP_EINVAL, "fp_inject_dev: needs a device count and a capacity");
    if (!p->x || !p->y || !p->vx || !p->vy || !p->vz || !p->pid || !p->key)
        return set_err(c, FP_EINVAL, "fp_inject_dev: bad particles");
    return launch_inject(c, p, -1, pid_next, 0u, step_dev, (flags & FP_STEP_ADVANCE) ? step_dev : nullptr, s);
}

extern "C" int64_t fp_capacity_overflows(fp_ctx* c, hipStream_t s) {
    if (!c) return FP_EINVAL;
    unsigned long long v = 0;
    if (hipMemcpyAsync(&v, c->errcount + 1, sizeof(v), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return set_err(c, FP_EDEVICE, "fp_capacity_overflows: copy failed");
    return (int64_t)v;
}

extern "C" int fp_cell_volumes(fp_ctx* c, double* vol, hipStream_t s) {
    if (!c || !vol) return set_err(c, FP_EINVAL, "fp_cell_volumes: bad argument");
    if (hipMemcpyAsync(vol, c->vol, sizeof(double) * (size_t)c->ncell, hipMemcpyDeviceToDevice, s) !=
        hipSuccess)
        return set_err(c, FP_EDEVICE, "fp_cell_volumes: copy failed");
    return FP_OK;
}
