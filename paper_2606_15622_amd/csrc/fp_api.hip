// fp_api.hip -- context management and argument checking of the C ABI (include/fp.h).
#include <cmath>
#include <cstdio>
#include <new>

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
    if (g->geometry != FP_COUETTE1D && g->geometry != FP_CAVITY2D) return why = "geometry", 0;
    if (g->precision != FP_F32 && g->precision != FP_F64) return why = "precision", 0;
    if (g->conserve != FP_EXACT && g->conserve != FP_PAPER) return why = "conserve", 0;
    if (g->nx < 1 || g->ny < 1 || (int64_t)g->nx * g->ny > (1 << 28)) return why = "grid", 0;
    if (g->geometry == FP_COUETTE1D && g->ny != 1) return why = "1-D grid needs ny = 1", 0;
    if (g->capacity < 0 || g->capacity > ((int64_t)1 << 31) - 64) return why = "capacity", 0;
    if (g->max_bounces < 0 || g->max_bounces > 1000) return why = "max_bounces", 0;
    if (!finite_pos(g->dx) || !finite_pos(g->dy) || !finite_pos(g->lx) || !finite_pos(g->ly) ||
        !finite_pos(g->dt) || !finite_pos(g->kB) || !finite_pos(g->mass) ||
        !finite_pos(g->mu_ref) || !finite_pos(g->T_ref) || !finite_pos(g->fnum_over_vol))
        return why = "non-positive physical parameter", 0;
    for (int w = 0; w < 4; ++w)
        if (!finite_pos(g->T_wall[w])) return why = "wall temperature", 0;
    if (!(g->eps_hat >= 0.0) || !(g->pivot_tol >= 0.0)) return why = "eps_hat/pivot_tol", 0;
    return 1;
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
              dalloc(&c->ccur, nc) && dalloc(&c->cwave, cap) && dalloc(&c->cmask, cap) &&
              dalloc(&c->gidx, cap) && dalloc(&c->blocksum, 2 * 8192) &&
              dalloc(&c->errcount, 1);
    if (ok) ok = hipMemset(c->errcount, 0, sizeof(unsigned long long)) == hipSuccess;
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
    (void)hipFree(c->cwave);
    (void)hipFree(c->cmask);
    (void)hipFree(c->gidx);
    (void)hipFree(c->blocksum);
    (void)hipFree(c->errcount);
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
    if (p->n == 0) return true;
    if (!p->vx || !p->vy || !p->vz || !p->pid || !p->key) return false;
    if (need_pos && (!p->x || (c->cfg.geometry == FP_CAVITY2D && !p->y))) return false;
    return true;
}

extern "C" int fp_bin(fp_ctx* c, const fp_particles* src, fp_particles* dst, int32_t* offsets,
                      int32_t* perm, hipStream_t s) {
    if (!c || !offsets || !particles_ok(c, src, true) || !dst)
        return set_err(c, FP_EINVAL, "fp_bin: bad argument");
    if (src->n > 0 && (!dst->vx || !dst->vy || !dst->vz || !dst->pid || !dst->key || !dst->x ||
                       (c->cfg.geometry == FP_CAVITY2D && !dst->y)))
        return set_err(c, FP_EINVAL, "fp_bin: bad destination");
    if (src->vx == dst->vx || src->x == dst->x || src->pid == dst->pid)
        return set_err(c, FP_EINVAL, "fp_bin: src and dst alias");
    return launch_bin(c, src, dst, offsets, perm, s);
}

extern "C" int fp_moments(fp_ctx* c, const fp_particles* p, const int32_t* offsets, double* mom,
                          hipStream_t s) {
    if (!c || !offsets || !mom || !particles_ok(c, p, false))
        return set_err(c, FP_EINVAL, "fp_moments: bad argument");
    return launch_moments(c, p, offsets, mom, s);
}

extern "C" int fp_closure_solve(fp_ctx* c, const double* mom, double* rec, int32_t* status,
                                hipStream_t s) {
    if (!c || !mom || !rec || !status) return set_err(c, FP_EINVAL, "fp_closure_solve: bad argument");
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
    return launch_step(c, p, offsets, mom, rec, step, flags, s);
}

extern "C" int fp_sample(fp_ctx* c, const double* mom, double* samp, hipStream_t s) {
    if (!c || !mom || !samp) return set_err(c, FP_EINVAL, "fp_sample: bad argument");
    return launch_sample(c, mom, samp, s);
}
