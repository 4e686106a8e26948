"""ctypes binding of ``libfpgpu.so`` (include/fp.h).

Argument marshalling only: torch tensors provide device memory and the stream, and
every step of the path runs in the library's HIP kernels.  ``load()`` raises if the
library has not been built; there is no fallback.
"""
import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfpgpu.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "fp.h")

FP_OK, FP_EINVAL, FP_ENOMEM, FP_EDEVICE, FP_ECAPACITY = 0, -1, -2, -3, -4
FP_COUETTE1D, FP_CAVITY2D, FP_CYLINDER2D = 0, 1, 2
FP_F32, FP_F64 = 0, 1
FP_EXACT, FP_PAPER = 0, 1
(CELL_OK, CELL_EMPTY, CELL_FEW, CELL_SINGULAR, CELL_NONFINITE, CELL_NN,
 CELL_NN_FALLBACK) = range(7)
STEP_COLLIDE, STEP_MOVE, STEP_KEYS, STEP_ADVANCE = 1, 2, 4, 8
MOM_STRIDE, REC_STRIDE, SAMP_STRIDE, DIAG_STRIDE = 32, 16, 16, 24
NN_PARAMS, NN_TRAIN, NN_FEATURES, NN_OUTPUTS = 39408, 39312, 32, 16
LITE_PARAMS, LITE_TRAIN, LITE_FEATURES = 205904, 205840, 16
LOSS_MSE, LOSS_RESIDUAL = 0, 1


class FPConfig(C.Structure):
    _fields_ = [
        ("geometry", C.c_int32), ("precision", C.c_int32), ("conserve", C.c_int32),
        ("nx", C.c_int32), ("ny", C.c_int32), ("n_min", C.c_int32), ("max_bounces", C.c_int32),
        ("lanes", C.c_int32), ("moment_order", C.c_int32), ("reserved0", C.c_int32),
        ("capacity", C.c_int64),
        ("x0", C.c_double), ("y0", C.c_double), ("lx", C.c_double), ("ly", C.c_double),
        ("dx", C.c_double), ("dy", C.c_double), ("dt", C.c_double),
        ("kB", C.c_double), ("mass", C.c_double),
        ("mu_ref", C.c_double), ("T_ref", C.c_double), ("omega", C.c_double),
        ("fnum_over_vol", C.c_double), ("eps_hat", C.c_double), ("pivot_tol", C.c_double),
        ("T_wall", C.c_double * 4), ("u_wall", (C.c_double * 3) * 4),
        ("seed", C.c_uint64),
        ("circle", C.c_double * 3), ("T_body", C.c_double), ("n_inf", C.c_double),
        ("u_inf", C.c_double * 3), ("T_inf", C.c_double), ("fnum", C.c_double),
        ("depth", C.c_double),
    ]


class FPAMRParams(C.Structure):
    _fields_ = [("tau_grad", C.c_double), ("tau_coarse", C.c_double), ("shock_factor", C.c_double),
                ("p_inf", C.c_double), ("n_max", C.c_double), ("n_grad", C.c_double),
                ("eps", C.c_double), ("age_min", C.c_int32), ("reserved", C.c_int32)]


class FPParticles(C.Structure):
    _fields_ = [("x", C.c_void_p), ("y", C.c_void_p), ("vx", C.c_void_p), ("vy", C.c_void_p),
                ("vz", C.c_void_p), ("pid", C.c_void_p), ("key", C.c_void_p), ("n", C.c_int64),
                ("n_dev", C.c_void_p), ("capacity", C.c_int64)]


_lib = None


def load():
    """Load libfpgpu.so (built by ``paper_2606_15622_amd.build``); raises if missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2606_15622_amd/build.py")
        L = C.CDLL(LIB_PATH)
        P, vp, i32, i64, u32, u64 = C.POINTER, C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64
        L.fp_init.argtypes = [P(FPConfig), P(vp)]
        L.fp_init.restype = C.c_int
        L.fp_destroy.argtypes = [vp]
        L.fp_last_error.argtypes = [vp]
        L.fp_last_error.restype = C.c_char_p
        L.fp_error_count.argtypes = [vp, vp]
        L.fp_error_count.restype = i64
        L.fp_bin.argtypes = [vp, P(FPParticles), P(FPParticles), vp, vp, vp]
        L.fp_rebin.argtypes = [vp, P(FPParticles), vp, P(FPParticles), vp, vp, vp, vp, vp]
        L.fp_moments.argtypes = [vp, P(FPParticles), vp, vp, vp]
        L.fp_moments_sample.argtypes = [vp, P(FPParticles), vp, vp, vp, vp, vp]
        L.fp_closure_solve.argtypes = [vp, vp, vp, vp, vp]
        L.fp_step.argtypes = [vp, P(FPParticles), vp, vp, vp, u64, u32, vp]
        L.fp_sample.argtypes = [vp, vp, vp, vp]
        L.fp_step_dev.argtypes = [vp, P(FPParticles), vp, vp, vp, vp, u32, vp]
        L.fp_counter_add.argtypes = [vp, vp, u32, vp]
        L.fp_diagnostics.argtypes = [vp, vp, C.c_double, C.c_double, C.c_double, vp, vp]
        L.fp_inject.argtypes = [vp, P(FPParticles), i64, vp, u64, vp]
        L.fp_inject_dev.argtypes = [vp, P(FPParticles), vp, vp, u32, vp]
        L.fp_capacity_overflows.argtypes = [vp, vp]
        L.fp_capacity_overflows.restype = i64
        L.fp_inject_slots.argtypes = [vp]
        L.fp_inject_slots.restype = i64
        L.fp_cell_volumes.argtypes = [vp, vp, vp]
        L.fp_nn_create.argtypes = [vp, i64, P(vp)]
        L.fp_nn_destroy.argtypes = [vp]
        L.fp_nn_load.argtypes = [vp, vp, vp, vp]
        L.fp_closure_nn.argtypes = [vp, vp, vp, vp, vp, C.c_double, C.c_double, C.c_double, vp]
        L.fp_closure_nn_noalloc.argtypes = [vp, vp, vp, vp, vp, C.c_double, C.c_double, C.c_double,
                                            vp]
        L.fp_nn_outputs.argtypes = [vp, vp, vp, vp]
        L.fp_nn_infer.argtypes = [vp, vp, vp, vp, vp]
        L.fp_nn_sensitivity.argtypes = [vp, vp, vp, i32, C.c_double, u64, vp, vp]
        L.fp_sample_high.argtypes = [vp, vp, vp, vp]
        L.fp_high_order.argtypes = [vp, vp, vp, vp]
        L.fp_wall_sampling.argtypes = [vp, vp, i32]
        L.fp_surface_coefficients.argtypes = [vp, vp, i32, C.c_double, vp, vp]
        L.fp_amr_init.argtypes = [vp, i32]
        L.fp_amr_adapt.argtypes = [vp, P(FPAMRParams), vp, vp, P(FPParticles), i32, vp]
        L.fp_amr_tree.argtypes = [vp, vp, vp, vp, vp, vp]
        L.fp_ncell.argtypes = [vp]
        L.fp_ncell.restype = i32
        L.fp_amr_nodes.argtypes = [vp]
        L.fp_amr_nodes.restype = i64
        L.fp_nn_features.argtypes = [vp, vp, i64, vp, vp]
        L.fp_closure_build.argtypes = [vp, vp, i64, vp, vp]
        L.fp_nn_grad.argtypes = [vp, vp, vp, vp, vp, vp, i64, i32, vp, vp, vp]
        L.fp_nn_adam.argtypes = [vp, vp, vp, vp, vp, i64, C.c_float, vp]
        L.fp_nn_train_step.argtypes = [vp, vp, vp, vp, vp, i64, C.c_float, vp, vp, vp, i64, i32,
                                       vp, vp]
        L.fp_nn_targets.argtypes = [vp, vp, i64, vp, vp]
        L.fp_column_stats.argtypes = [vp, vp, i64, i32, vp, vp, vp]
        L.fp_lite_create.argtypes = [vp, i64, P(vp)]
        L.fp_lite_destroy.argtypes = [vp]
        L.fp_lite_load.argtypes = [vp, vp, vp, vp]
        L.fp_lite_infer.argtypes = [vp, vp, vp, vp, vp]
        L.fp_closure_lite.argtypes = [vp, vp, vp, vp, vp, C.c_double, C.c_double, C.c_double, vp]
        L.fp_lite_features.argtypes = [vp, vp, vp, i64, vp, vp]
        L.fp_lite_targets.argtypes = [vp, vp, i64, vp, vp]
        L.fp_lite_grad.argtypes = [vp, vp, vp, vp, vp, i64, vp, vp, vp]
        L.fp_lite_adam.argtypes = [vp, vp, vp, vp, vp, i64, C.c_float, vp]
        L.fp_lite_train_step.argtypes = [vp, vp, vp, vp, vp, i64, C.c_float, vp, vp, i64, vp, vp]
        L.fp_closure_solve_backward.argtypes = [vp, vp, vp, vp, vp, vp]
        L.fp_moments_backward.argtypes = [vp, P(FPParticles), vp, vp, vp, vp, vp, vp, vp]
        for f in ("fp_bin", "fp_rebin", "fp_moments", "fp_moments_sample", "fp_closure_solve", "fp_step", "fp_sample", "fp_nn_create",
                  "fp_nn_load", "fp_closure_nn", "fp_closure_nn_noalloc", "fp_nn_outputs", "fp_nn_infer", "fp_nn_sensitivity", "fp_nn_features",
                  "fp_closure_build", "fp_nn_grad", "fp_nn_adam", "fp_nn_train_step",
                  "fp_nn_targets", "fp_closure_solve_backward", "fp_moments_backward",
                  "fp_inject", "fp_inject_dev", "fp_cell_volumes", "fp_step_dev", "fp_counter_add", "fp_diagnostics",
                  "fp_amr_init", "fp_amr_adapt", "fp_amr_tree", "fp_wall_sampling",
                  "fp_surface_coefficients", "fp_sample_high", "fp_high_order", "fp_lite_create",
                  "fp_lite_load", "fp_lite_infer", "fp_closure_lite", "fp_lite_features",
                  "fp_lite_targets", "fp_lite_grad", "fp_lite_adam", "fp_lite_train_step",
                  "fp_column_stats"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def header_functions():
    """Names of the functions declared in include/fp.h."""
    import re
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|int32_t|int64_t|const char\*)\s+(fp_\w+)\s*\(", txt, re.M)))


def make_config(w: dict, capacity: int) -> FPConfig:
    c = FPConfig()
    c.geometry = {"couette1d": FP_COUETTE1D, "cavity2d": FP_CAVITY2D,
                  "cylinder2d": FP_CYLINDER2D}[w["geometry"]]
    c.precision = {"f32": FP_F32, "f64": FP_F64}[w["precision"]]
    c.conserve = {"exact": FP_EXACT, "paper": FP_PAPER}[w.get("conserve", "exact")]
    c.nx, c.ny = int(w["nx"]), int(w["ny"])
    c.n_min = int(w.get("n_min", 4))
    c.max_bounces = int(w.get("max_bounces", 8))
    c.lanes = int(w.get("lanes", 0))
    c.moment_order = int(w.get("moment_order", 5))
    c.capacity = int(capacity)
    c.x0, c.y0, c.lx, c.ly = float(w["x0"]), float(w["y0"]), float(w["lx"]), float(w["ly"])
    c.dx, c.dy, c.dt = float(w["dx"]), float(w["dy"]), float(w["dt"])
    c.kB, c.mass = float(w["kB"]), float(w["mass"])
    c.mu_ref, c.T_ref, c.omega = float(w["mu_ref"]), float(w["T_ref"]), float(w["omega"])
    c.fnum_over_vol, c.eps_hat = float(w["fnum_over_vol"]), float(w["eps_hat"])
    c.pivot_tol = float(w.get("pivot_tol", 1e-12))
    for k in range(4):
        c.T_wall[k] = float(w["T_wall"][k])
        for j in range(3):
            c.u_wall[k][j] = float(w["u_wall"][k][j])
    c.seed = int(w["seed"])
    for k in range(3):
        c.circle[k] = float(w.get("circle", (0.0, 0.0, 0.0))[k])
        c.u_inf[k] = float(w.get("u_inf", (0.0, 0.0, 0.0))[k])
    c.T_body = float(w.get("T_body", 0.0))
    c.n_inf = float(w.get("n_inf", 0.0))
    c.T_inf = float(w.get("T_inf", 0.0))
    c.fnum = float(w.get("fnum", 0.0))
    c.depth = float(w.get("depth", 1.0))
    return c


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Particles:
    """Device particle arrays (structure of arrays) of one storage precision."""

    def __init__(self, n, dtype, two_d, device="cuda", capacity=None, device_count=False):
        """device_count: the count lives in a device word (n_dev), which the sort writes
        and the injection advances; n is then only a launch-shape hint."""
        cap = int(capacity if capacity is not None else n)
        self.capacity = cap
        self.n = int(n)
        self.n_dev = (torch.tensor([int(n)], dtype=torch.int64, device=device)
                      if device_count else None)
        self.dtype = dtype
        self.two_d = two_d
        mk = lambda dt: torch.zeros(max(cap, 1), dtype=dt, device=device)
        self.x = mk(dtype)
        self.y = mk(dtype) if two_d else None
        self.vx, self.vy, self.vz = mk(dtype), mk(dtype), mk(dtype)
        self.pid = mk(torch.int32)
        self.key = mk(torch.int32)

    @classmethod
    def from_numpy(cls, w, state, capacity=None, device="cuda", device_count=False):
        dt = torch.float32 if w["precision"] == "f32" else torch.float64
        two_d = w["geometry"] != "couette1d"
        n = state["x"].shape[0]
        p = cls(n, dt, two_d, device, capacity, device_count)
        npdt = np.float32 if dt == torch.float32 else np.float64
        for k in ("x", "vx", "vy", "vz"):
            getattr(p, k)[:n].copy_(torch.from_numpy(np.ascontiguousarray(state[k], dtype=npdt)))
        if two_d:
            p.y[:n].copy_(torch.from_numpy(np.ascontiguousarray(state["y"], dtype=npdt)))
        p.pid[:n].copy_(torch.from_numpy(np.ascontiguousarray(state["pid"], dtype=np.uint32).view(np.int32)))
        if "key" in state:
            p.key[:n].copy_(torch.from_numpy(np.ascontiguousarray(state["key"], dtype=np.int32)))
        return p

    def struct(self):
        s = FPParticles()
        s.x, s.vx, s.vy, s.vz = (t.data_ptr() for t in (self.x, self.vx, self.vy, self.vz))
        s.y = self.y.data_ptr() if self.y is not None else None
        s.pid, s.key = self.pid.data_ptr(), self.key.data_ptr()
        s.n = self.n
        s.n_dev = self.n_dev.data_ptr() if self.n_dev is not None else None
        s.capacity = self.capacity
        return s

    def count(self):
        """The particle count (a host read of the device word when there is one)."""
        return int(self.n_dev.cpu()[0]) if self.n_dev is not None else self.n

    def numpy(self):
        n = self.count()
        out = {k: getattr(self, k)[:n].double().cpu().numpy() for k in ("x", "vx", "vy", "vz")}
        out["y"] = self.y[:n].double().cpu().numpy() if self.y is not None else np.zeros(n)
        out["pid"] = self.pid[:n].cpu().numpy().view(np.uint32).copy()
        out["key"] = self.key[:n].cpu().numpy().copy()
        return out


class Context:
    """An fp_ctx plus the entry points of include/fp.h."""

    def __init__(self, w: dict, capacity: int):
        self.lib = load()
        self.w = w
        self.cfg = make_config(w, capacity)
        self.ncell = int(w["nx"]) * int(w["ny"])
        h = C.c_void_p()
        rc = self.lib.fp_init(C.byref(self.cfg), C.byref(h))
        if rc != FP_OK:
            raise RuntimeError(f"fp_init failed ({rc})")
        self.h = h

    def close(self):
        if self.h:
            self.lib.fp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc != FP_OK:
            raise RuntimeError(f"{what} failed ({rc}): {self.lib.fp_last_error(self.h).decode()}")

    def error_count(self, stream=None):
        return self.lib.fp_error_count(self.h, _stream(stream))

    def bin(self, src, dst, offsets, perm=None, stream=None):
        a, b = src.struct(), dst.struct()
        self._check(self.lib.fp_bin(self.h, C.byref(a), C.byref(b), _ptr(offsets), _ptr(perm),
                                    _stream(stream)), "fp_bin")

    def rebin(self, src, src_offsets, dst, offsets, perm=None, mom=None, samp=None, stream=None):
        a, b = src.struct(), dst.struct()
        self._check(self.lib.fp_rebin(self.h, C.byref(a), _ptr(src_offsets), C.byref(b),
                                      _ptr(offsets), _ptr(perm), _ptr(mom), _ptr(samp),
                                      _stream(stream)), "fp_rebin")

    def moments(self, p, offsets, mom, stream=None):
        a = p.struct()
        self._check(self.lib.fp_moments(self.h, C.byref(a), _ptr(offsets), _ptr(mom),
                                        _stream(stream)), "fp_moments")

    def moments_sample(self, p, offsets, mom, samp0, samp1=None, stream=None):
        a = p.struct()
        self._check(self.lib.fp_moments_sample(self.h, C.byref(a), _ptr(offsets), _ptr(mom), _ptr(samp0),
                                               _ptr(samp1),
                                               _stream(stream)), "fp_moments_sample")

    def closure_solve(self, mom, rec, status, stream=None):
        self._check(self.lib.fp_closure_solve(self.h, _ptr(mom), _ptr(rec), _ptr(status),
                                              _stream(stream)), "fp_closure_solve")

    def step(self, p, offsets, mom, rec, step, flags, stream=None):
        a = p.struct()
        self._check(self.lib.fp_step(self.h, C.byref(a), _ptr(offsets), _ptr(mom), _ptr(rec),
                                     int(step), int(flags), _stream(stream)), "fp_step")

    def sample(self, mom, samp, stream=None):
        self._check(self.lib.fp_sample(self.h, _ptr(mom), _ptr(samp), _stream(stream)), "fp_sample")

    def step_dev(self, p, offsets, mom, rec, step_dev, flags, stream=None):
        a = p.struct()
        self._check(self.lib.fp_step_dev(self.h, C.byref(a), _ptr(offsets), _ptr(mom), _ptr(rec),
                                         _ptr(step_dev), int(flags), _stream(stream)), "fp_step_dev")

    def diagnostics(self, samp, theta_inf, n_inf, dg_inf, diag, stream=None):
        self._check(self.lib.fp_diagnostics(self.h, _ptr(samp), float(theta_inf), float(n_inf),
                                            float(dg_inf), _ptr(diag), _stream(stream)),
                    "fp_diagnostics")

    def counter_add(self, ctr, inc, stream=None):
        self._check(self.lib.fp_counter_add(self.h, _ptr(ctr), int(inc), _stream(stream)),
                    "fp_counter_add")

    def inject(self, p, at, pid_next, step, stream=None):
        a = p.struct()
        self._check(self.lib.fp_inject(self.h, C.byref(a), int(at), _ptr(pid_next), int(step),
                                       _stream(stream)), "fp_inject")

    def inject_dev(self, p, pid_next, step_dev, flags=0, stream=None):
        self._check(self.lib.fp_inject_dev(self.h, C.byref(p.struct()), _ptr(pid_next), _ptr(step_dev),
                                           int(flags), _stream(stream)), "fp_inject_dev")

    def capacity_overflows(self, stream=None):
        return int(self.lib.fp_capacity_overflows(self.h, _stream(stream)))

    def inject_slots(self):
        return int(self.lib.fp_inject_slots(self.h))

    def cell_volumes(self, vol, stream=None):
        self._check(self.lib.fp_cell_volumes(self.h, _ptr(vol), _stream(stream)), "fp_cell_volumes")

    # ---- high-order fields -------------------------------------------------------------
    def sample_high(self, mom, hsamp, stream=None):
        self._check(self.lib.fp_sample_high(self.h, _ptr(mom), _ptr(hsamp), _stream(stream)),
                    "fp_sample_high")

    def high_order(self, hsamp, out, stream=None):
        self._check(self.lib.fp_high_order(self.h, _ptr(hsamp), _ptr(out), _stream(stream)),
                    "fp_high_order")

    # ---- surface sampling of the cylinder ---------------------------------------------
    def wall_sampling(self, sums):
        """sums: float64 tensor [nbins][4] on the device (None stops)."""
        nb = int(sums.shape[0]) if sums is not None else 0
        self._check(self.lib.fp_wall_sampling(self.h, _ptr(sums), nb), "fp_wall_sampling")

    def surface_coefficients(self, sums, t_total, out, stream=None):
        self._check(self.lib.fp_surface_coefficients(self.h, _ptr(sums), int(sums.shape[0]),
                                                     float(t_total), _ptr(out), _stream(stream)),
                    "fp_surface_coefficients")

    # ---- adaptive quadtree ------------------------------------------------------------
    def amr_init(self, max_level):
        self._check(self.lib.fp_amr_init(self.h, int(max_level)), "fp_amr_init")
        self.ncell = int(self.lib.fp_ncell(self.h))

    def amr_adapt(self, prm, acc, samp, p, steps, stream=None):
        """prm: dict of fp_amr_params fields.  Synchronous; updates self.ncell."""
        q = FPAMRParams()
        for k in ("tau_grad", "tau_coarse", "shock_factor", "p_inf", "n_max", "n_grad", "eps"):
            setattr(q, k, float(prm[k]))
        q.age_min = int(prm["age_min"])
        a = p.struct() if p is not None else None
        self._check(self.lib.fp_amr_adapt(self.h, C.byref(q), _ptr(acc), _ptr(samp),
                                          C.byref(a) if a is not None else None, int(steps),
                                          _stream(stream)), "fp_amr_adapt")
        self.ncell = int(self.lib.fp_ncell(self.h))

    def amr_nodes(self):
        return int(self.lib.fp_amr_nodes(self.h))

    def amr_tree(self, state=None, age=None, leafmap=None, leaf_node=None, stream=None):
        self._check(self.lib.fp_amr_tree(self.h, _ptr(state), _ptr(age), _ptr(leafmap), _ptr(leaf_node),
                                         _stream(stream)), "fp_amr_tree")

    # ---- learned closure -------------------------------------------------------------
    def closure_build(self, mom, n, sys, stream=None):
        self._check(self.lib.fp_closure_build(self.h, _ptr(mom), int(n), _ptr(sys), _stream(stream)),
                    "fp_closure_build")

    def nn_features(self, mom, n, feats, stream=None):
        self._check(self.lib.fp_nn_features(self.h, _ptr(mom), int(n), _ptr(feats), _stream(stream)),
                    "fp_nn_features")

    def nn_targets(self, rec, n, targets, stream=None):
        self._check(self.lib.fp_nn_targets(self.h, _ptr(rec), int(n), _ptr(targets), _stream(stream)),
                    "fp_nn_targets")

    def closure_solve_backward(self, mom, rec, ybar, mombar, stream=None):
        self._check(self.lib.fp_closure_solve_backward(self.h, _ptr(mom), _ptr(rec), _ptr(ybar),
                                                       _ptr(mombar), _stream(stream)),
                    "fp_closure_solve_backward")

    def moments_backward(self, p, offsets, mom, mombar, gx, gy, gz, stream=None):
        a = p.struct()
        self._check(self.lib.fp_moments_backward(self.h, C.byref(a), _ptr(offsets), _ptr(mom),
                                                 _ptr(mombar), _ptr(gx), _ptr(gy), _ptr(gz),
                                                 _stream(stream)), "fp_moments_backward")

    def column_stats(self, x, mean, std, stream=None):
        n, k = x.shape
        self._check(self.lib.fp_column_stats(self.h, _ptr(x), int(n), int(k), _ptr(mean), _ptr(std),
                                             _stream(stream)), "fp_column_stats")

    def lite_features(self, mom, n, feats, nvol=None, stream=None):
        self._check(self.lib.fp_lite_features(self.h, _ptr(mom), _ptr(nvol), int(n), _ptr(feats),
                                              _stream(stream)), "fp_lite_features")

    def lite_targets(self, rec, n, targets, stream=None):
        self._check(self.lib.fp_lite_targets(self.h, _ptr(rec), int(n), _ptr(targets), _stream(stream)),
                    "fp_lite_targets")

    def lite_adam(self, params, grad, m, v, t, lr, stream=None):
        self._check(self.lib.fp_lite_adam(self.h, _ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(t),
                                          float(lr), _stream(stream)), "fp_lite_adam")

    def nn_adam(self, params, grad, m, v, t, lr, stream=None):
        self._check(self.lib.fp_nn_adam(self.h, _ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(t),
                                        float(lr), _stream(stream)), "fp_nn_adam")


class AMRSimulation:
    """Loop of the open cylinder domain on an adaptive quadtree (the grid of w is the
    finest level, max_level levels below the base grid): every adapt_every steps
    fp_amr_adapt on the sampling sums of the leaves since the last adaptation, then
    sort -> moments -> sums (and sample) -> closure -> collide + move -> inflow injection.
    The sort is a full fp_bin every step: fp_rebin also sorts on a tree (between
    adaptations), but there it treats the leaves as one row, and on the cylinder about a
    third of the particles that change leaf land in a leaf that is not next to their old
    one in depth-first order; that general path makes the re-sort slower than fp_bin
    (2.6 against 1.4 ms per step at 7.6e5 leaves).  The particle count and the step number
    live on the device (as in OpenSimulation); the adaptation every adapt_every steps is
    synchronous (it reads the new leaf count back)."""

    def __init__(self, w, state, max_level, prm, adapt_every, capacity=None, device="cuda"):
        self.w, self.prm, self.adapt_every = w, dict(prm), int(adapt_every)
        n0 = state["x"].shape[0]
        cap = int(capacity if capacity is not None else 2 * n0 + 1_000_000)
        self.ctx = Context(w, cap)
        self.ctx.amr_init(max_level)
        self.slots = self.ctx.inject_slots()
        self.a = Particles.from_numpy(w, state, capacity=cap, device=device, device_count=True)
        self.b = Particles(0, self.a.dtype, True, device, capacity=cap, device_count=True)
        self.a.n = self.b.n = min(n0 + self.slots, cap)   # launch-shape hint
        nf = int(w["nx"]) * int(w["ny"])   # at most this many leaves
        self.offs = [torch.zeros(nf + 1, dtype=torch.int32, device=device) for _ in range(2)]
        self.mom = torch.zeros((nf, MOM_STRIDE), dtype=torch.float64, device=device)
        self.rec = torch.zeros((nf, REC_STRIDE), dtype=torch.float64, device=device)
        self.status = torch.zeros(nf, dtype=torch.int32, device=device)
        self.samp = torch.zeros((nf, SAMP_STRIDE), dtype=torch.float64, device=device)
        self.acc = torch.zeros((nf, SAMP_STRIDE), dtype=torch.float64, device=device)
        self.pid_next = torch.tensor([int(state.get("pid_next", n0))], dtype=torch.int64,
                                     device=device).to(torch.int32)
        self.step_ctr = torch.zeros(1, dtype=torch.int32, device=device)
        self.since = None
        self.ctx.step(self.a, None, None, None, 0, STEP_KEYS)   # leaf keys from positions

    @property
    def ncell(self):
        return self.ctx.ncell

    @property
    def offsets(self):
        return self.offs[0][:self.ncell + 1]

    def adapt(self, steps):
        self.ctx.amr_adapt(self.prm, self.acc, self.samp, self.a, steps)

    def _adapt_due(self, s):
        """The adaptation that falls on step s (every adapt_every steps from the first)."""
        if self.since is None:
            self.since = s
        elif self.adapt_every > 0 and s - self.since >= self.adapt_every:
            self.adapt(s - self.since)
            self.since = s

    def _body(self, sample, closure):
        """One step at the device step number, which it advances (no adaptation)."""
        self.ctx.bin(self.a, self.b, self.offs[1])
        self.offs.reverse()
        self.a, self.b = self.b, self.a
        # moments, the adaptation sums and (when sampling) the output sums in one pass
        self.ctx.moments_sample(self.a, self.offs[0], self.mom, self.acc, self.samp if sample else None)
        if closure is None:
            self.ctx.closure_solve(self.mom, self.rec, self.status)
        else:
            closure(self.mom, self.rec, self.status)
        self.ctx.step_dev(self.a, self.offs[0], self.mom, self.rec, self.step_ctr,
                          STEP_COLLIDE | STEP_MOVE)
        self.ctx.inject_dev(self.a, self.pid_next, self.step_ctr, STEP_ADVANCE)

    def step(self, s, sample=False, closure=None):
        self._adapt_due(s)
        self.step_ctr.fill_(s)
        self._body(sample, closure)

    def run(self, step0, nsteps, n_skip=None):
        n_skip = self.w.get("n_skip", 0) if n_skip is None else n_skip
        for s in range(step0, step0 + nsteps):
            self.step(s, sample=s >= n_skip)

    def tree(self):
        """Host copies: (state[nodes], age[nodes], leafmap[nx ny], leaf_node[ncell])."""
        dev = self.mom.device
        nodes, nf = self.ctx.amr_nodes(), self.offs[0].shape[0] - 1
        st = torch.zeros(nodes, dtype=torch.int8, device=dev)
        age = torch.zeros(nodes, dtype=torch.int32, device=dev)
        lm = torch.zeros(nf, dtype=torch.int32, device=dev)
        ln = torch.zeros(max(self.ncell, 1), dtype=torch.int32, device=dev)
        self.ctx.amr_tree(st, age, lm, ln)
        torch.cuda.synchronize()
        return st.cpu().numpy(), age.cpu().numpy(), lm.cpu().numpy(), ln[:self.ncell].cpu().numpy()

    def kept(self):
        """Particles kept by the last sort (host read)."""
        return int(self.offs[0][self.ncell])

    def live(self):
        """Particles after the last move and injection, deleted and unused slots removed
        (host copy, for checks)."""
        out = self.a.numpy()
        keep = out["key"] < self.ncell
        return {k: v[keep] for k, v in out.items()}


class GraphAMRSimulation(AMRSimulation):
    """AMRSimulation whose steps between adaptations are HIP-graph replays (for callers that
    capture their loop): two steps per graph (the particle buffers, their count words and the
    offsets return to their places), the step number and the particle count advanced on the
    device.  An adaptation changes the leaf count and with it the launch shapes, so it drops
    the graphs; the next replay captures them again (once per adaptation interval).  Not
    faster than eager steps here: 1.67 against 1.65 ms per step at 7.6e5 leaves."""

    def __init__(self, *args, **kw):
        super().__init__(*args, **kw)
        self.graphs = {}

    def adapt(self, steps):
        super().adapt(steps)
        self.graphs = {}

    def _graph(self, sample):
        if sample not in self.graphs:
            g = torch.cuda.CUDAGraph()
            torch.cuda.synchronize()
            live = (self.step_ctr, self.samp, self.acc, self.pid_next, self.a.n_dev, self.b.n_dev)
            saved = tuple(t.clone() for t in live)
            with torch.cuda.graph(g):
                for _ in range(2):
                    self._body(sample, None)
            torch.cuda.synchronize()
            # capture executes nothing; restore anyway
            for t, v in zip(live, saved):
                t.copy_(v)
            self.graphs[sample] = g
        return self.graphs[sample]

    def run_pairs(self, npairs, sample=False):
        """Advance 2 * npairs steps by graph replays (from the device step number); no
        adaptation falls inside them."""
        g = self._graph(sample)
        for _ in range(npairs):
            g.replay()

    def run(self, step0, nsteps, n_skip=None):
        """The steps of AMRSimulation.run, the same adaptations at the same steps, by graph
        replays between them (an odd step before an adaptation, or before sampling starts,
        runs eagerly)."""
        n_skip = self.w.get("n_skip", 0) if n_skip is None else n_skip
        s, end = step0, step0 + nsteps
        while s < end:
            self._adapt_due(s)
            nxt = end if self.adapt_every <= 0 else min(self.since + self.adapt_every, end)
            if s < n_skip:
                nxt = min(nxt, n_skip)
            sample = s >= n_skip
            npairs = (nxt - s) // 2
            if npairs:
                self.step_ctr.fill_(s)
                self.run_pairs(npairs, sample)
                s += 2 * npairs
            if s < nxt:
                self.step(s, sample=sample)
                s += 1


class Network:
    """An fp_nn handle: BF16 image for inference plus training scratch."""

    def __init__(self, ctx: Context, max_batch: int = 0):
        self.ctx = ctx
        h = C.c_void_p()
        rc = ctx.lib.fp_nn_create(ctx.h, int(max_batch), C.byref(h))
        if rc != FP_OK:
            raise RuntimeError(f"fp_nn_create failed ({rc})")
        self.h = h
        self.max_batch = int(max_batch)

    def close(self):
        if self.h:
            self.ctx.lib.fp_nn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load(self, params, stream=None):
        c = self.ctx
        c._check(c.lib.fp_nn_load(c.h, self.h, _ptr(params), _stream(stream)), "fp_nn_load")

    def closure(self, mom, rec, status, tol_abs, tol_rel, relax=1.0, stream=None):
        c = self.ctx
        c._check(c.lib.fp_closure_nn(c.h, self.h, _ptr(mom), _ptr(rec), _ptr(status), float(tol_abs),
                                     float(tol_rel), float(relax), _stream(stream)), "fp_closure_nn")

    def closure_noalloc(self, mom, rec, status, tol_abs, tol_rel, relax=1.0, stream=None):
        c = self.ctx
        c._check(c.lib.fp_closure_nn_noalloc(c.h, self.h, _ptr(mom), _ptr(rec), _ptr(status),
                                             float(tol_abs), float(tol_rel), float(relax),
                                             _stream(stream)), "fp_closure_nn_noalloc")

    def sensitivity(self, mom, npass, p, seed, sens, stream=None):
        c = self.ctx
        c._check(c.lib.fp_nn_sensitivity(c.h, self.h, _ptr(mom), int(npass), float(p), int(seed),
                                         _ptr(sens), _stream(stream)), "fp_nn_sensitivity")

    def outputs(self, y, stream=None):
        c = self.ctx
        c._check(c.lib.fp_nn_outputs(c.h, self.h, _ptr(y), _stream(stream)), "fp_nn_outputs")

    def infer(self, mom, y, stream=None):
        c = self.ctx
        c._check(c.lib.fp_nn_infer(c.h, self.h, _ptr(mom), _ptr(y), _stream(stream)), "fp_nn_infer")

    def grad(self, params, feats, targets, sys, B, loss_kind, grad, loss, stream=None):
        c = self.ctx
        c._check(c.lib.fp_nn_grad(c.h, self.h, _ptr(params), _ptr(feats), _ptr(targets), _ptr(sys),
                                  int(B), int(loss_kind), _ptr(grad), _ptr(loss), _stream(stream)),
                 "fp_nn_grad")

    def train_step(self, params, m, v, t, lr, feats, targets, sys, B, loss_kind, loss, stream=None):
        c = self.ctx
        c._check(c.lib.fp_nn_train_step(c.h, self.h, _ptr(params), _ptr(m), _ptr(v), int(t),
                                        float(lr), _ptr(feats), _ptr(targets), _ptr(sys), int(B),
                                        int(loss_kind), _ptr(loss), _stream(stream)), "fp_nn_train_step")


class LiteNetwork:
    """An fp_lite handle: the paper's 16-256x4-9 ReLU surrogate (BF16 image for inference
    plus training scratch)."""

    def __init__(self, ctx: Context, max_batch: int = 0):
        self.ctx = ctx
        h = C.c_void_p()
        rc = ctx.lib.fp_lite_create(ctx.h, int(max_batch), C.byref(h))
        if rc != FP_OK:
            raise RuntimeError(f"fp_lite_create failed ({rc})")
        self.h = h
        self.max_batch = int(max_batch)

    def close(self):
        if self.h:
            self.ctx.lib.fp_lite_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load(self, params, stream=None):
        c = self.ctx
        c._check(c.lib.fp_lite_load(c.h, self.h, _ptr(params), _stream(stream)), "fp_lite_load")

    def infer(self, mom, y, stream=None):
        c = self.ctx
        c._check(c.lib.fp_lite_infer(c.h, self.h, _ptr(mom), _ptr(y), _stream(stream)), "fp_lite_infer")

    def closure(self, mom, rec, status, tol_abs, tol_rel, relax=1.0, stream=None):
        c = self.ctx
        c._check(c.lib.fp_closure_lite(c.h, self.h, _ptr(mom), _ptr(rec), _ptr(status), float(tol_abs),
                                       float(tol_rel), float(relax), _stream(stream)), "fp_closure_lite")

    def grad(self, params, feats, targets, B, grad, loss, stream=None):
        c = self.ctx
        c._check(c.lib.fp_lite_grad(c.h, self.h, _ptr(params), _ptr(feats), _ptr(targets), int(B),
                                    _ptr(grad), _ptr(loss), _stream(stream)), "fp_lite_grad")

    def train_step(self, params, m, v, t, lr, feats, targets, B, loss, stream=None):
        c = self.ctx
        c._check(c.lib.fp_lite_train_step(c.h, self.h, _ptr(params), _ptr(m), _ptr(v), int(t), float(lr),
                                          _ptr(feats), _ptr(targets), int(B), _ptr(loss), _stream(stream)),
                 "fp_lite_train_step")


class Simulation:
    """Host loop of the exact-closure step on one GPU (Algorithm "Baseline Physics
    Simulation Loop"): bin -> moments -> [sample] -> closure -> collide + move.
    All buffers stay on the device; nothing crosses to the host inside the loop."""

    def __init__(self, w, state, device="cuda"):
        self.w = w
        n = state["x"].shape[0]
        self.ctx = Context(w, n)
        self.a = Particles.from_numpy(w, state, device=device)
        self.b = Particles(n, self.a.dtype, self.a.two_d, device)
        nc = self.ctx.ncell
        # two offsets arrays: the re-sort reads the previous grouping and writes the next
        self.offs = [torch.zeros(nc + 1, dtype=torch.int32, device=device) for _ in range(2)]
        self.sorted = False        # a holds particles grouped by offs[0] with new keys
        self.mom = torch.zeros((nc, MOM_STRIDE), dtype=torch.float64, device=device)
        self.rec = torch.zeros((nc, REC_STRIDE), dtype=torch.float64, device=device)
        self.status = torch.zeros(nc, dtype=torch.int32, device=device)
        self.samp = torch.zeros((nc, SAMP_STRIDE), dtype=torch.float64, device=device)
        # the closure of the step: None = the exact closure, or a callable(mom, rec, status)
        self.closure_fn = None
        if "key" not in state:
            self.ctx.step(self.a, None, None, None, 0, STEP_KEYS)

    @property
    def offsets(self):
        """Cell start indices of the particles in a (after the last sort)."""
        return self.offs[0]

    def closure(self):
        if self.closure_fn is None:
            self.ctx.closure_solve(self.mom, self.rec, self.status)
        else:
            self.closure_fn(self.mom, self.rec, self.status)

    def sort(self, perm=None, mom=None, samp=None):
        """a -> b sorted by key (fp_rebin from the previous grouping after the first
        step, fp_bin before), then swap a and b; offsets describe the new a.  With mom,
        the moments of the sorted cells are written too, and with samp their time-average
        sums are added (by the re-sort itself, or by fp_moments_sample after the first
        sort)."""
        if self.sorted:
            self.ctx.rebin(self.a, self.offs[0], self.b, self.offs[1], perm, mom, samp)
        else:
            self.ctx.bin(self.a, self.b, self.offs[1], perm)
        self.offs.reverse()
        self.a, self.b = self.b, self.a
        if mom is not None and not self.sorted:
            if samp is not None:
                self.ctx.moments_sample(self.a, self.offsets, mom, samp)
            else:
                self.ctx.moments(self.a, self.offsets, mom)
        self.sorted = True

    def step(self, s, sample=False):
        self.sort(mom=self.mom, samp=self.samp if sample else None)
        self.closure()
        self.ctx.step(self.a, self.offsets, self.mom, self.rec, s, STEP_COLLIDE | STEP_MOVE)

    def run(self, step0, nsteps, n_skip=None):
        n_skip = self.w.get("n_skip", 0) if n_skip is None else n_skip
        for s in range(step0, step0 + nsteps):
            self.step(s, sample=s >= n_skip)


class GraphSimulation(Simulation):
    """Simulation whose step is captured once in a HIP graph (torch.cuda.CUDAGraph) and
    replayed; the Philox step number lives in device memory and the captured step
    advances it.  Two steps are captured back to back so that the particle ping-pong
    buffers return to their places; graphs with and without sampling are kept."""

    def __init__(self, w, state, step0=0, device="cuda"):
        super().__init__(w, state, device)
        self.step_ctr = torch.tensor([step0], dtype=torch.int32, device=device)
        self.graphs = {}

    def _body(self, sample):
        for _ in range(2):
            self.sort(mom=self.mom, samp=self.samp if sample else None)
            self.closure()
            self.ctx.step_dev(self.a, self.offsets, self.mom, self.rec, self.step_ctr,
                              STEP_COLLIDE | STEP_MOVE | STEP_ADVANCE)

    def _graph(self, sample):
        if sample not in self.graphs:
            g = torch.cuda.CUDAGraph()
            torch.cuda.synchronize()
            saved = self.step_ctr.clone()
            samp = self.samp.clone()
            was_sorted = self.sorted
            with torch.cuda.graph(g):
                self._body(sample)
            torch.cuda.synchronize()
            self.step_ctr.copy_(saved)   # capture does not execute; keep the counter anyway
            self.samp.copy_(samp)
            self.sorted = was_sorted
            self.graphs[sample] = g
        return self.graphs[sample]

    def run_pairs(self, npairs, sample=False):
        """Advance 2 * npairs steps by graph replays."""
        g = self._graph(sample)
        for _ in range(npairs):
            g.replay()


class OpenSimulation:
    """Loop of the open cylinder domain: sort -> moments -> [sample] -> closure -> collide +
    move (deleting particles that leave the box) -> inflow injection.  The particle count
    lives on the device (each particle buffer has its own count word: the sort writes the
    number it keeps, the injection appends behind it and advances it) and so does the step
    number, so a step needs no host read; GraphOpenSimulation captures it."""

    def __init__(self, w, state, capacity=None, device="cuda"):
        self.w = w
        n0 = state["x"].shape[0]
        cap = int(capacity if capacity is not None else 2 * n0 + 1_000_000)
        self.ctx = Context(w, cap)
        self.slots = self.ctx.inject_slots()
        self.a = Particles.from_numpy(w, state, capacity=cap, device=device, device_count=True)
        self.b = Particles(0, self.a.dtype, True, device, capacity=cap, device_count=True)
        # launch-shape hint of both buffers (the count itself is on the device)
        self.a.n = self.b.n = min(n0 + self.slots, cap)
        nc = self.ctx.ncell
        self.offs = [torch.zeros(nc + 1, dtype=torch.int32, device=device) for _ in range(2)]
        self.sorted = False
        self.mom = torch.zeros((nc, MOM_STRIDE), dtype=torch.float64, device=device)
        self.rec = torch.zeros((nc, REC_STRIDE), dtype=torch.float64, device=device)
        self.status = torch.zeros(nc, dtype=torch.int32, device=device)
        self.samp = torch.zeros((nc, SAMP_STRIDE), dtype=torch.float64, device=device)
        self.pid_next = torch.tensor([int(state.get("pid_next", n0))], dtype=torch.int64,
                                     device=device).to(torch.int32)
        self.step_ctr = torch.zeros(1, dtype=torch.int32, device=device)
        if "key" not in state:
            self.ctx.step(self.a, None, None, None, 0, STEP_KEYS)

    @property
    def offsets(self):
        return self.offs[0]

    def _body(self, sample, closure):
        """One step at the device step number; advances it."""
        # after the first step the live particles are grouped by their previous cells and
        # the injected ones follow them: the re-sort applies
        fused = self.sorted
        if self.sorted:
            self.ctx.rebin(self.a, self.offs[0], self.b, self.offs[1], None, self.mom,
                           self.samp if sample else None)
        else:
            self.ctx.bin(self.a, self.b, self.offs[1])
        self.offs.reverse()
        self.sorted = True
        self.a, self.b = self.b, self.a
        if not fused:
            if sample:
                self.ctx.moments_sample(self.a, self.offsets, self.mom, self.samp)
            else:
                self.ctx.moments(self.a, self.offsets, self.mom)
        if closure is None:
            self.ctx.closure_solve(self.mom, self.rec, self.status)
        else:
            closure(self.mom, self.rec, self.status)
        self.ctx.step_dev(self.a, self.offsets, self.mom, self.rec, self.step_ctr,
                          STEP_COLLIDE | STEP_MOVE)
        self.ctx.inject_dev(self.a, self.pid_next, self.step_ctr, STEP_ADVANCE)

    def step(self, s, sample=False, closure=None):
        self.step_ctr.fill_(s)
        self._body(sample, closure)

    def run(self, step0, nsteps, n_skip=None):
        n_skip = self.w.get("n_skip", 0) if n_skip is None else n_skip
        for s in range(step0, step0 + nsteps):
            self.step(s, sample=s >= n_skip)

    def kept(self):
        """Particles kept by the last sort (host read)."""
        return int(self.offsets[-1])

    def live(self):
        """Particles after the last move and injection, deleted and unused slots removed
        (host copy, for checks)."""
        out = self.a.numpy()
        keep = out["key"] < self.ctx.ncell
        return {k: v[keep] for k, v in out.items()}


class GraphOpenSimulation(OpenSimulation):
    """OpenSimulation whose step is captured once in a HIP graph and replayed: two steps
    back to back (the particle buffers and their count words return to their places), the
    step number and the particle count advanced on the device."""

    def __init__(self, w, state, capacity=None, device="cuda"):
        super().__init__(w, state, capacity, device)
        self.graphs = {}

    def _graph(self, sample):
        if sample not in self.graphs:
            if not self.sorted:
                raise RuntimeError("run one eager step before capturing (the first sort is general)")
            g = torch.cuda.CUDAGraph()
            torch.cuda.synchronize()
            saved = (self.step_ctr.clone(), self.samp.clone(), self.pid_next.clone(),
                     self.a.n_dev.clone(), self.b.n_dev.clone())
            with torch.cuda.graph(g):
                for _ in range(2):
                    self._body(sample, None)
            torch.cuda.synchronize()
            # capture executes nothing; restore anyway
            for t, v in zip((self.step_ctr, self.samp, self.pid_next, self.a.n_dev, self.b.n_dev), saved):
                t.copy_(v)
            self.graphs[sample] = g
        return self.graphs[sample]

    def run_pairs(self, npairs, sample=False):
        """Advance 2 * npairs steps by graph replays (from the device step number)."""
        g = self._graph(sample)
        for _ in range(npairs):
            g.replay()
