"""ctypes wrapper of the C oracle (``oracle/fp_oracle.c``).

TEST INFRASTRUCTURE ONLY.  The test suite, ``__graft_entry__.smoke()`` and the CPU
baseline of ``bench.py`` are the only callers.  It takes plain numpy arrays and a
workload dictionary (the same dictionary the GPU binding is configured from) and never
sees a GPU buffer.
"""
import ctypes as C
import os

import numpy as np

from . import build_oracle

_HERE = os.path.dirname(os.path.abspath(__file__))

OR_COUETTE1D, OR_CAVITY2D, OR_CYLINDER2D = 0, 1, 2
OR_F32, OR_F64 = 0, 1
OR_EXACT, OR_PAPER = 0, 1
OR_OK, OR_EMPTY, OR_FEW, OR_SINGULAR, OR_NONFINITE, OR_NN, OR_NN_FALLBACK = range(7)
PURPOSE_COLLISION, PURPOSE_WALL = 3, 4
MOM_STRIDE, REC_STRIDE, SAMP_STRIDE = 32, 16, 16


class OrConfig(C.Structure):
    _fields_ = [
        ("geometry", C.c_int32), ("precision", C.c_int32), ("conserve", C.c_int32),
        ("nx", C.c_int32), ("ny", C.c_int32), ("n_min", C.c_int32),
        ("max_bounces", C.c_int32),
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


_lib = None


def lib():
    """Load (building first if needed) the oracle shared library."""
    global _lib
    if _lib is None:
        path = build_oracle.LIB
        src = os.path.join(_HERE, "fp_oracle.c")
        if (not os.path.exists(path)) or os.path.getmtime(path) < os.path.getmtime(src):
            build_oracle.build()
        _lib = C.CDLL(path)
        _declare(_lib)
    return _lib


def _declare(L):
    P = C.POINTER
    d, i32, i64, u32, u64 = C.c_double, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64
    cfgp = P(OrConfig)
    L.or_philox4x32_10.argtypes = [P(u32), P(u32), P(u32)]
    L.or_uniforms.argtypes = [u64, u32, u32, u32, u32, P(d)]
    L.or_normals3.argtypes = [u64, u32, u32, u32, u32, P(d)]
    L.or_keys.argtypes = [cfgp, i64, P(d), P(d), P(i32)]
    L.or_bin.argtypes = [i32, i64, P(i32), P(i64), P(i32)]
    L.or_moments.argtypes = [i32, P(i32), P(d), P(d), P(d), P(d)]
    L.or_cell_params.argtypes = [cfgp, P(d), d, P(d), P(d)]
    L.or_cell_volumes.argtypes = [cfgp, P(d)]
    L.or_inject.argtypes = [cfgp, u32, P(u32), i64, P(d), P(d), P(d), P(d), P(d), P(u32), P(i32)]
    L.or_inject.restype = i64
    L.or_run_open.argtypes = [cfgp, i64, P(i64), P(d), P(d), P(d), P(d), P(d), P(u32), P(i32),
                              P(u32), u32, i32, u32, P(d), P(d), P(i32), P(d)]
    L.or_run_open.restype = C.c_int
    L.or_closure_system.argtypes = [P(d), d, P(d), P(d)]
    L.or_closure.argtypes = [cfgp, i32, P(d), P(d), P(d), P(i32)]
    L.or_update.argtypes = [cfgp, i32, P(i32), P(d), P(d), P(d), P(u32), P(d), P(d), u32]
    L.or_move.argtypes = [cfgp, i64, P(d), P(d), P(d), P(d), P(d), P(u32), P(i32), u32]
    L.or_move_wall.argtypes = [cfgp, i64, P(d), P(d), P(d), P(d), P(d), P(u32), P(i32), u32,
                               P(d), i32]
    L.or_sample.argtypes = [i32, P(i32), P(d), P(d), P(d), P(d)]
    L.or_set_threads.argtypes = [C.c_int]
    L.or_set_threads.restype = C.c_int
    L.or_run.argtypes = [cfgp, i64, P(d), P(d), P(d), P(d), P(d), P(u32), P(i32), u32, i32,
                         u32, P(d), P(d), P(i32), P(d)]
    L.or_run.restype = C.c_int


def _p(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


def set_threads(n=0):
    """Threads of the oracle's parallel loops (0: the OpenMP default); returns the count."""
    return int(lib().or_set_threads(int(n)))


def make_config(w: dict) -> OrConfig:
    """Oracle configuration from a workload dictionary (see the package's inputs module)."""
    c = OrConfig()
    c.geometry = {"couette1d": OR_COUETTE1D, "cavity2d": OR_CAVITY2D,
                  "cylinder2d": OR_CYLINDER2D}[w["geometry"]]
    c.precision = {"f32": OR_F32, "f64": OR_F64}[w["precision"]]
    c.conserve = {"exact": OR_EXACT, "paper": OR_PAPER}[w.get("conserve", "exact")]
    c.nx, c.ny = int(w["nx"]), int(w["ny"])
    c.n_min = int(w.get("n_min", 4))
    c.max_bounces = int(w.get("max_bounces", 8))
    c.x0, c.y0 = float(w["x0"]), float(w["y0"])
    c.lx, c.ly = float(w["lx"]), float(w["ly"])
    c.dx, c.dy = float(w["dx"]), float(w["dy"])
    c.dt = float(w["dt"])
    c.kB, c.mass = float(w["kB"]), float(w["mass"])
    c.mu_ref, c.T_ref, c.omega = float(w["mu_ref"]), float(w["T_ref"]), float(w["omega"])
    c.fnum_over_vol = float(w["fnum_over_vol"])
    c.eps_hat = float(w["eps_hat"])
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


# ---------------------------------------------------------------------------------------
def philox(ctr, key):
    L = lib()
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    L.or_philox4x32_10(c, k, o)
    return [o[i] for i in range(4)]


def uniforms(seed, pid, step, purpose, sub):
    L = lib()
    u = (C.c_double * 4)()
    L.or_uniforms(seed, pid, step, purpose, sub, u)
    return np.array(list(u))


def normals3(seed, pid, step, purpose, sub):
    L = lib()
    z = (C.c_double * 3)()
    L.or_normals3(seed, pid, step, purpose, sub, z)
    return np.array(list(z))


def keys(w, x, y=None):
    L = lib()
    cfg = make_config(w)
    x = _f64(x)
    y = _f64(y if y is not None else np.zeros_like(x))
    k = np.empty(x.shape[0], dtype=np.int32)
    L.or_keys(C.byref(cfg), x.shape[0], _p(x, C.c_double), _p(y, C.c_double), _p(k, C.c_int32))
    return k


def bin_particles(ncell, key):
    """Stable counting sort: returns (perm, offsets) with perm[j] = source index of slot j."""
    L = lib()
    key = np.ascontiguousarray(key, dtype=np.int32)
    n = key.shape[0]
    perm = np.empty(n, dtype=np.int64)
    off = np.empty(ncell + 1, dtype=np.int32)
    L.or_bin(int(ncell), n, _p(key, C.c_int32), _p(perm, C.c_int64), _p(off, C.c_int32))
    return perm, off


def moments(offsets, vx, vy, vz):
    L = lib()
    off = np.ascontiguousarray(offsets, dtype=np.int32)
    ncell = off.shape[0] - 1
    vx, vy, vz = _f64(vx), _f64(vy), _f64(vz)
    mom = np.empty((ncell, MOM_STRIDE), dtype=np.float64)
    L.or_moments(ncell, _p(off, C.c_int32), _p(vx, C.c_double), _p(vy, C.c_double),
                 _p(vz, C.c_double), _p(mom, C.c_double))
    return mom


def cell_params(w, mom_cell, nvol=None):
    L = lib()
    cfg = make_config(w)
    m = _f64(mom_cell)
    tau, eps2 = C.c_double(), C.c_double()
    nv = float(w["fnum_over_vol"] if nvol is None else nvol)
    L.or_cell_params(C.byref(cfg), _p(m, C.c_double), nv, C.byref(tau), C.byref(eps2))
    return tau.value, eps2.value


def cell_volumes(w):
    L = lib()
    cfg = make_config(w)
    vol = np.empty(int(w["nx"]) * int(w["ny"]), dtype=np.float64)
    L.or_cell_volumes(C.byref(cfg), _p(vol, C.c_double))
    return vol


def closure_system(mom_cell, eps_hat):
    L = lib()
    m = _f64(mom_cell)
    A = np.empty(81, dtype=np.float64)
    b = np.empty(9, dtype=np.float64)
    L.or_closure_system(_p(m, C.c_double), float(eps_hat), _p(A, C.c_double), _p(b, C.c_double))
    return A.reshape(9, 9), b


def closure(w, mom, nvol=None):
    L = lib()
    cfg = make_config(w)
    mom = _f64(mom)
    ncell = mom.shape[0]
    rec = np.empty((ncell, REC_STRIDE), dtype=np.float64)
    st = np.empty(ncell, dtype=np.int32)
    nv = _p(_f64(nvol), C.c_double) if nvol is not None else None
    L.or_closure(C.byref(cfg), ncell, _p(mom, C.c_double), nv, _p(rec, C.c_double),
                 _p(st, C.c_int32))
    return rec, st


def update(w, offsets, vx, vy, vz, pid, mom, rec, step):
    """Returns updated copies of (vx, vy, vz)."""
    L = lib()
    cfg = make_config(w)
    off = np.ascontiguousarray(offsets, dtype=np.int32)
    vx, vy, vz = _f64(vx).copy(), _f64(vy).copy(), _f64(vz).copy()
    pid = np.ascontiguousarray(pid, dtype=np.uint32)
    mom, rec = _f64(mom), _f64(rec)
    L.or_update(C.byref(cfg), off.shape[0] - 1, _p(off, C.c_int32), _p(vx, C.c_double),
                _p(vy, C.c_double), _p(vz, C.c_double), _p(pid, C.c_uint32),
                _p(mom, C.c_double), _p(rec, C.c_double), int(step))
    return vx, vy, vz


def move(w, x, y, vx, vy, vz, pid, step, wall=None):
    """Returns (x, y, vx, vy, vz, key) after free flight with walls.  wall: optional
    float64 array [nbins][4] to which the cylinder exchange sums are added in place."""
    L = lib()
    cfg = make_config(w)
    x = _f64(x).copy()
    y = _f64(y if y is not None else np.zeros_like(x)).copy()
    vx, vy, vz = _f64(vx).copy(), _f64(vy).copy(), _f64(vz).copy()
    pid = np.ascontiguousarray(pid, dtype=np.uint32)
    n = x.shape[0]
    key = np.empty(n, dtype=np.int32)
    if wall is None:
        L.or_move(C.byref(cfg), n, _p(x, C.c_double), _p(y, C.c_double), _p(vx, C.c_double),
                  _p(vy, C.c_double), _p(vz, C.c_double), _p(pid, C.c_uint32),
                  _p(key, C.c_int32), int(step))
    else:
        assert wall.dtype == np.float64 and wall.flags.c_contiguous and wall.shape[1] == 4
        L.or_move_wall(C.byref(cfg), n, _p(x, C.c_double), _p(y, C.c_double),
                       _p(vx, C.c_double), _p(vy, C.c_double), _p(vz, C.c_double),
                       _p(pid, C.c_uint32), _p(key, C.c_int32), int(step),
                       _p(wall, C.c_double), int(wall.shape[0]))
    return x, y, vx, vy, vz, key


def sample(offsets, vx, vy, vz, samp=None):
    L = lib()
    off = np.ascontiguousarray(offsets, dtype=np.int32)
    ncell = off.shape[0] - 1
    if samp is None:
        samp = np.zeros((ncell, SAMP_STRIDE), dtype=np.float64)
    vx, vy, vz = _f64(vx), _f64(vy), _f64(vz)
    L.or_sample(ncell, _p(off, C.c_int32), _p(vx, C.c_double), _p(vy, C.c_double),
                _p(vz, C.c_double), _p(samp, C.c_double))
    return samp


def run(w, state, step0, nsteps, n_skip=0, samp=None):
    """Full loop on a copy of ``state`` (dict of x, y, vx, vy, vz, pid, key).

    Returns (new_state, mom, rec, status, samp)."""
    L = lib()
    cfg = make_config(w)
    ncell = int(w["nx"]) * int(w["ny"])
    n = state["x"].shape[0]
    s = {k: _f64(state[k]).copy() for k in ("x", "vx", "vy", "vz")}
    s["y"] = _f64(state["y"] if state.get("y") is not None else np.zeros(n)).copy()
    s["pid"] = np.ascontiguousarray(state["pid"], dtype=np.uint32).copy()
    s["key"] = np.ascontiguousarray(state["key"], dtype=np.int32).copy()
    mom = np.zeros((ncell, MOM_STRIDE))
    rec = np.zeros((ncell, REC_STRIDE))
    st = np.zeros(ncell, dtype=np.int32)
    if samp is None:
        samp = np.zeros((ncell, SAMP_STRIDE))
    rc = L.or_run(C.byref(cfg), n, _p(s["x"], C.c_double), _p(s["y"], C.c_double),
                  _p(s["vx"], C.c_double), _p(s["vy"], C.c_double), _p(s["vz"], C.c_double),
                  _p(s["pid"], C.c_uint32), _p(s["key"], C.c_int32), int(step0), int(nsteps),
                  int(n_skip), _p(mom, C.c_double), _p(rec, C.c_double), _p(st, C.c_int32),
                  _p(samp, C.c_double))
    if rc != 0:
        raise MemoryError("oracle run failed to allocate")
    return s, mom, rec, st, samp


def inject(w, step, pid_next, room=10_000_000):
    """Returns (dict of appended arrays, new pid_next)."""
    L = lib()
    cfg = make_config(w)
    a = {k: np.empty(room) for k in ("x", "y", "vx", "vy", "vz")}
    pid = np.empty(room, dtype=np.uint32)
    key = np.empty(room, dtype=np.int32)
    pn = C.c_uint32(int(pid_next))
    k = L.or_inject(C.byref(cfg), int(step), C.byref(pn), room, *(_p(a[q], C.c_double) for q in
                    ("x", "y", "vx", "vy", "vz")), _p(pid, C.c_uint32), _p(key, C.c_int32))
    if k < 0:
        raise MemoryError("oracle injection room exceeded")
    out = {q: a[q][:k].copy() for q in a}
    out["pid"] = pid[:k].copy()
    out["key"] = key[:k].copy()
    return out, pn.value


def run_open(w, state, pid_next, step0, nsteps, capacity, n_skip=0, samp=None):
    """Open-domain loop (cylinder).  Returns (state, pid_next, mom, rec, status, samp)."""
    L = lib()
    cfg = make_config(w)
    ncell = int(w["nx"]) * int(w["ny"])
    n0 = state["x"].shape[0]
    s = {}
    for k in ("x", "y", "vx", "vy", "vz"):
        s[k] = np.zeros(capacity)
        s[k][:n0] = state[k]
    s["pid"] = np.zeros(capacity, dtype=np.uint32)
    s["pid"][:n0] = state["pid"]
    s["key"] = np.zeros(capacity, dtype=np.int32)
    s["key"][:n0] = state["key"]
    n = C.c_int64(n0)
    pn = C.c_uint32(int(pid_next))
    mom = np.zeros((ncell, MOM_STRIDE))
    rec = np.zeros((ncell, REC_STRIDE))
    st = np.zeros(ncell, dtype=np.int32)
    if samp is None:
        samp = np.zeros((ncell, SAMP_STRIDE))
    rc = L.or_run_open(C.byref(cfg), capacity, C.byref(n), *(_p(s[k], C.c_double) for k in
                       ("x", "y", "vx", "vy", "vz")), _p(s["pid"], C.c_uint32),
                       _p(s["key"], C.c_int32), C.byref(pn), int(step0), int(nsteps), int(n_skip),
                       _p(mom, C.c_double), _p(rec, C.c_double), _p(st, C.c_int32),
                       _p(samp, C.c_double))
    if rc != 0:
        raise RuntimeError(f"oracle open run failed ({rc})")
    out = {k: v[:n.value].copy() for k, v in s.items()}
    return out, pn.value, mom, rec, st, samp
