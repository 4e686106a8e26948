"""Benchmark of the cubic-FP particle step on one MI355X.

Workload (default): the 2-D lid-driven cavity, 100 x 100 cells, 100 particles per cell
(1e6 particles), FP32 particle storage, FP64 closure, exact closure, nominal Kn 1.0,
lid 50 m/s, diffuse walls at 273 K.  One step = bin -> moments -> sample -> closure ->
collide + move: the whole hot path.  Inputs are seeded synthetic states already resident
in HBM when the timed region starts.

Prints one JSON line: particle-steps/s (value), cell-closures/s, per-entry-point times
from HIP events on the launch stream, the roofline of the dominant single-kernel entry
point, the same measured on a scaled cavity (448 x 448 cells, 2e7 particles, beyond the
256 MB last-level cache), and the FP64 CPU oracle timed on a bounded sample.
"""
import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--kn", type=float, default=1.0)
    ap.add_argument("--no-scaled", action="store_true", help="skip the 2e7-particle cavity")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--scaled-steps", type=int, default=20)
    ap.add_argument("--no-other", action="store_true", help="skip the Couette and cylinder lines")
    ap.add_argument("--cylinder-steps", type=int, default=20)
    ap.add_argument("--amr-steps", type=int, default=100)
    ap.add_argument("--amr-only", action="store_true",
                    help="run only the quadtree cylinder line (for its kernel profile)")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-closure section (training, loop speeds, field errors)")
    ap.add_argument("--learned-only", action="store_true", help="run only the learned-closure section")
    return ap.parse_args()


# algorithmic bytes per launch of each entry point (FP32 2-D particles): what the
# operation must move at least, once each
#   step (collide+move): read x y vx vy vz pid, write x y vx vy vz key = 48 B/particle;
#                        per cell offsets 8 B, rec 128 B, U and T of mom 104 B
#   sort_moments:        the re-sort with the moment gather and the time-average sums in
#                        the same pass: read key x y vx vy vz pid 28 B, write the same
#                        28 B = 56 B/particle; per cell 8 B of old and 4 B of new offsets,
#                        the 256 B moment record, 14 sums read and written (224 B)
#   closure:             256 B in + 128 B + 4 B out per cell
def alg_bytes(kind, n, nc):
    return {"step": 48 * n + 240 * nc, "sort_moments": 56 * n + 492 * nc,
            "closure": 388 * nc}[kind]


def gpu_hold(torch, ms):
    """Keep the launch stream busy for about `ms` milliseconds (a bounded spin kernel), so
    that the host can enqueue far ahead and the queue never runs dry behind it."""
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    torch.cuda._sleep(1_000_000)
    e.record()
    torch.cuda.synchronize()
    per = max(s.elapsed_time(e), 1e-3) / 1_000_000       # ms per spin cycle
    torch.cuda._sleep(int(min(ms / per, 2e9)))


def entry_times(torch, F, sim, s, steps=20):
    """Per-entry-point durations inside the loop itself: `steps` eager steps (re-sort with
    moments and sums, closure, collide + move, in the loop's order) are enqueued behind a
    GPU hold, each entry point between two HIP events on the launch stream, so the events
    time back-to-back kernels with no host gaps.  Means in milliseconds."""
    ctx = sim.ctx
    names = ("sort_moments", "closure", "step")
    ev = {k: [] for k in names}
    torch.cuda.synchronize()
    gpu_hold(torch, 60.0)
    for i in range(steps):
        calls = (("sort_moments", lambda: sim.sort(mom=sim.mom, samp=sim.samp)),
                 ("closure", lambda: ctx.closure_solve(sim.mom, sim.rec, sim.status)),
                 ("step", lambda: ctx.step(sim.a, sim.offsets, sim.mom, sim.rec, s + i,
                                           F.STEP_COLLIDE | F.STEP_MOVE)))
        for k, fn in calls:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            ev[k].append((e0, e1))
    torch.cuda.synchronize()
    return {k: float(np.mean([a.elapsed_time(b) for a, b in v])) for k, v in ev.items()}


def run_workload(torch, F, I, w, steps, warmup, graph=True, kernel_times=True):
    """Warm up eagerly, then time `steps` steps: replays of the step captured in a HIP
    graph (graph=True) or eager launches.  Returns timings and per-kernel durations."""
    state = I.maxwellian_state(w)
    sim = F.GraphSimulation(w, state, step0=warmup) if graph else F.Simulation(w, state)
    sim.F = F
    n, nc = state["x"].shape[0], I.ncells(w)
    del state
    s = 0
    for _ in range(warmup):
        sim.step(s, sample=True)
        s += 1
    torch.cuda.synchronize()
    steps = steps + (steps % 2) if graph else steps
    if graph:
        sim.run_pairs(1, sample=True)        # capture outside the timed region
        s += 2
        torch.cuda.synchronize()
        sim.step_ctr.fill_(s)
    t0 = time.perf_counter()
    if graph:
        sim.run_pairs(steps // 2, sample=True)
    else:
        for _ in range(steps):
            sim.step(s, sample=True)
            s += 1
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    if graph:
        s = int(sim.step_ctr.cpu()[0])
    # per-entry-point durations (loop order, HIP events)
    ms = entry_times(torch, F, sim, s) if kernel_times else {}
    kern = {}
    for k, v in ms.items():
        gbs = alg_bytes(k, n, nc) / (v * 1e-3) / 1e9
        kern[k] = {"ms": round(v, 5), "alg_GBps": round(gbs, 1), "alg_bytes": alg_bytes(k, n, nc)}
    st = sim.status.cpu().numpy()
    return dict(n=n, nc=nc, t=t, steps=steps, kern=kern, ok_cells=int((st == F.CELL_OK).sum()))


def profile_value(name, key):
    """A per-launch figure from a committed counter summary under profiles/ (lines
    "key: value"), valid only while every source it lists ("source: <path> <sha256>") is
    unchanged; otherwise None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    val, ok = None, True
    for line in open(path):
        if line.startswith("source:"):
            _, rel, digest = line.split()
            f = os.path.join(ROOT, rel)
            ok = ok and os.path.exists(f) and hashlib.sha256(open(f, "rb").read()).hexdigest() == digest
        elif line.startswith(key + ":"):
            val = int(float(line.split()[1]))
    return val if ok else None


def counter_traffic(name):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy)."""
    return profile_value(name, "traffic_bytes_per_launch")


# VALU issue peak: 256 CUs x 4 SIMDs x 2.4 GHz SIMD-cycles per second; a wave64 VALU
# instruction keeps a SIMD busy 4 cycles at full rate (16 cycles for the quarter-rate
# transcendental, 64-bit integer multiply and similar instructions)
VALU_PEAK_CYCLES = 256 * 4 * 2.4e9


def roofline_alu(res, kind, profile):
    """The entry point against its VALU issue bound: its VALU-busy SIMD cycles per launch
    (SQ_ACTIVE_INST_VALU from the committed counter summary) over the live mean launch
    time, against the chip's SIMD-cycles per second."""
    cyc = profile_value(profile, "valu_busy_cycles_per_launch")
    if cyc is None:
        return None
    ms = res["kern"][kind]["ms"]
    ach = cyc / (ms * 1e-3)
    return {"bound": "alu", "achieved": round(ach / 1e12, 4), "peak": round(VALU_PEAK_CYCLES / 1e12, 4),
            "unit": "T VALU-busy SIMD-cycles/s", "frac": round(ach / VALU_PEAK_CYCLES, 4), "kernel": kind,
            "valu_busy_cycles_per_launch": cyc, "avg_ms": ms}


def roofline_of(res, kind="step", traffic_file=None):
    k = res["kern"][kind]
    ach = k["alg_GBps"]
    return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4),
            "traffic": counter_traffic(traffic_file) if traffic_file else None, "kernel": kind,
            "alg_bytes_per_launch": k["alg_bytes"], "avg_ms": k["ms"]}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline(I, w):
    """The FP64 oracle on the host: the headline cavity on all threads (its cell and
    particle loops run on OpenMP threads; the sort is serial) and on one thread, the
    closure stage alone, and the Couette channel's full 1000 steps on one thread."""
    from oracle import oracle as O
    state = I.maxwellian_state(w)
    state["key"] = O.keys(w, state["x"], state["y"])
    n = state["x"].shape[0]
    nproc = os.cpu_count() or 1
    out = {"kind": "oracle", "unit": "particle-steps/s", "cpu": cpu_model(), "nproc": nproc}
    threads = O.set_threads(0)
    nsteps = 40
    t0 = time.perf_counter()
    o, mom, _, _, _ = O.run(w, state, 0, nsteps, n_skip=0)
    t = time.perf_counter() - t0
    out.update(value=round(n * nsteps / t, 1), cores=threads,
               sample=f"{nsteps} full steps of the headline cavity ({n} particles) on {threads} "
                      f"threads of {nproc} ({out['cpu']}), {t:.1f} s")
    O.set_threads(1)
    t0 = time.perf_counter()
    O.run(w, state, 0, 10, n_skip=0)
    t1 = time.perf_counter() - t0
    out["single_thread"] = {"value": round(n * 10 / t1, 1), "cores": 1, "sample": f"10 steps, {t1:.1f} s"}
    ok = mom[:, 0] > 1
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        O.closure(w, mom)
    tc = (time.perf_counter() - t0) / reps
    out["closure_cell_closures_per_s"] = {"value": round(w["nx"] * w["ny"] / tc, 1), "cores": 1,
                                          "sample": f"the 9x9 closure of the {int(ok.sum())} solved "
                                                    f"cells of the cavity, {reps} times"}
    wc = I.couette(kn=0.1, ncell=100, ppc=100, precision="f64", seed=1)
    sc = I.maxwellian_state(wc)
    sc["key"] = O.keys(wc, sc["x"])
    t0 = time.perf_counter()
    O.run(wc, sc, 0, 1000, n_skip=500)
    t2 = time.perf_counter() - t0
    out["couette_1000_steps"] = {"value": round(1e4 * 1000 / t2, 1), "cores": 1, "seconds": round(t2, 2)}
    O.set_threads(0)
    return out


def couette_line(torch, F, I, steps=1000):
    """Configuration 1: the FP64 Couette channel, 100 cells x 100 particles, graph-replayed
    steps (launch-bound at this size)."""
    w = I.couette(kn=0.1, ncell=100, ppc=100, precision="f64")
    res = run_workload(torch, F, I, w, steps, 20, graph=True, kernel_times=False)
    return {"workload": "couette1d 100 cells x 100 particles, FP64, Kn 0.1",
            "value": round(res["n"] * res["steps"] / res["t"], 1), "unit": "particle-steps/s",
            "ms_per_step": round(res["t"] / res["steps"] * 1e3, 5),
            "cell_closures_per_s": round(res["nc"] * res["steps"] / res["t"], 1)}


def cylinder_line(torch, F, I, steps):
    """Configuration 5: Mach 10 argon past the cylinder, 400 x 300 cut cells, about 1.8e7
    particles, FP32, exact closure, open boundaries with inflow injection.  The particle
    count and the step number stay on the device; the timed steps are replays of two
    steps captured in a HIP graph (no host read inside).  particle-steps = the mean of the
    kept counts read before and after the timed window (the steady-state count drifts by
    well under 0.1 % over it) times the steps."""
    w = I.cylinder(precision="f32", seed=3)
    state = I.freestream_state(w)
    sim = F.GraphOpenSimulation(w, state)
    del state
    for s in range(10):
        sim.step(s, sample=True)
    sim.run_pairs(1, sample=True)          # capture outside the timed window
    torch.cuda.synchronize()
    k0 = sim.kept()
    steps = steps + (steps % 2)
    t0 = time.perf_counter()
    sim.run_pairs(steps // 2, sample=True)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    k1 = sim.kept()
    live = 0.5 * (k0 + k1) * steps
    return {"workload": "cylinder2d 400x300 cut cells, Mach 10 argon, about 1.8e7 particles, FP32",
            "value": round(live / t, 1), "unit": "particle-steps/s", "steps": steps,
            "ms_per_step": round(t / steps * 1e3, 4), "particles_kept": [k0, k1],
            "timed_loop": "HIP graph replay of two captured steps (device particle count)",
            "cell_closures_per_s": round(sim.ctx.ncell * steps / t, 1)}


def cylinder_amr_line(torch, F, I, steps, warm=300, every=100):
    """The cylinder on the adaptive quadtree: base grid 400 x 300 cells of 2 mm, two levels
    below it (finest 0.5 mm, 1600 x 1200 fine cells), the same free stream and about 1.8e7
    particles, FP32, exact closure; an adaptation every `every` steps on the sums since the
    last one (criteria thresholds of the paper, N_max = 4x the free-stream particles of a
    base cell).  Warm-up steps let the bow shock form and the tree follow it.  Eager steps
    with the particle count on the device; particle-steps from the mean of the kept counts
    before and after the timed window."""
    w = I.cylinder(cell=0.5e-3, nx=1600, ny=1200, precision="f32", seed=3)
    ppc_base = w["n_inf"] * (2e-3) ** 2 * w["depth"] / w["fnum"]
    prm = dict(tau_grad=0.10, tau_coarse=0.05, shock_factor=1.2,
               p_inf=w["n_inf"] * I.KB * w["T_inf"], n_max=4.0 * ppc_base, n_grad=200.0,
               eps=1e-300, age_min=2000)
    state = I.freestream_state(w)
    sim = F.AMRSimulation(w, state, 2, prm, every)
    del state
    for s in range(warm):
        sim.step(s)
    torch.cuda.synchronize()
    leaves0 = sim.ncell
    k0 = sim.kept()
    t0 = time.perf_counter()
    t_adapt = 0.0
    for s in range(warm, warm + steps):
        if s - sim.since >= every:
            torch.cuda.synchronize()
            ta = time.perf_counter()
            sim.adapt(s - sim.since)
            sim.since = s
            t_adapt += time.perf_counter() - ta
        sim.step(s, sample=True)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    live = 0.5 * (k0 + sim.kept()) * steps
    return {"workload": "cylinder2d on a quadtree: base 400x300 cells of 2 mm, 2 levels "
                        "(1600x1200 fine), Mach 10 argon, about 1.8e7 particles, FP32",
            "value": round(live / t, 1), "unit": "particle-steps/s", "steps": steps,
            "ms_per_step": round(t / steps * 1e3, 4), "adapt_every": every,
            "adapt_ms": round(t_adapt * 1e3 / max(1, steps // every), 3),
            "leaves_before": leaves0, "leaves_after": sim.ncell,
            "cell_closures_per_s": round(sim.ncell * steps / t, 1)}


def learned_section(torch):
    """The learned half of the metric (both networks trained in this run by the library's
    kernels; see paper_2606_15622_amd.learned.benchmark).  A failure is reported in the
    line instead of ending the benchmark."""
    from paper_2606_15622_amd import learned as LN
    try:
        return LN.benchmark(log=lambda msg: print(msg, file=sys.stderr, flush=True))
    except Exception as e:   # noqa: BLE001 - reported, not hidden
        return {"error": f"{type(e).__name__}: {e}"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the library has no multi-GPU path "
              f"(--gpus {args.gpus} requested)", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2606_15622_amd import fpgpu as F
    from paper_2606_15622_amd import inputs as I
    F.load()
    torch.cuda.set_device(0)

    if args.amr_only:
        print(json.dumps({"cylinder_amr": cylinder_amr_line(torch, F, I, args.amr_steps)}), flush=True)
        return
    if args.learned_only:
        print(json.dumps({"learned": learned_section(torch)}), flush=True)
        return
    w = I.cavity(kn=args.kn, ncell=100, ppc=100, precision="f32", seed=1)
    res = run_workload(torch, F, I, w, args.steps, args.warmup, graph=True)
    res_eager = run_workload(torch, F, I, w, min(args.steps, 50), 5, graph=False, kernel_times=False)
    n, nc = res["n"], res["nc"]
    ms_step = res["t"] / res["steps"] * 1e3
    pps = n * res["steps"] / res["t"]
    kern = res["kern"]
    dominant = max(kern, key=lambda k: kern[k]["ms"])
    out = {
        "metric": "particle-steps/s and cell-closures/s, exact vs learned closure, at <=1% field error",
        "value_is": "particle-steps/s of the whole loop with the exact closure; the learned "
                    "closure's loop speeds, closure rates and field errors are under learned",
        "value": round(pps, 1),
        "unit": "particle-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 particles, f64 moments/closure",
        "data": "synthetic (seeded Maxwellian initial state)",
        "config": {"workload": f"cavity2d 100x100 cells, 100 particles/cell, Kn {args.kn}, "
                               f"lid 50 m/s, exact closure", "particles": n, "cells": nc,
                   "parallelism": "single GPU"},
        "cell_closures_per_s": round(nc * res["steps"] / res["t"], 1),
        "closure_kernel_cell_closures_per_s": round(nc / (kern["closure"]["ms"] * 1e-3), 1),
        "kernels": kern,
        "roofline_1e6": roofline_of(res, dominant, f"{dominant}_cavity100x100x100_counters.txt"),
        "timed_loop": "HIP graph replay of two captured steps",
        "eager_particle_steps_per_s": round(res_eager["n"] * res_eager["steps"] / res_eager["t"], 1),
    }
    if not args.no_scaled:
        ws = I.cavity(kn=args.kn, ncell=448, ppc=100, precision="f32", seed=2)
        rs = run_workload(torch, F, I, ws, args.scaled_steps, 5, graph=True)
        out["scaled"] = {
            "workload": "cavity2d 448x448 cells, 100 particles/cell (2.0e7 particles)",
            "value": round(rs["n"] * rs["steps"] / rs["t"], 1), "unit": "particle-steps/s",
            "ms_per_step": round(rs["t"] / rs["steps"] * 1e3, 4), "kernels": rs["kern"],
            "roofline_step": roofline_of(rs, "step", "step_cavity448x448x100_counters.txt"),
            "roofline_sort_moments": roofline_of(rs, "sort_moments",
                                                 "sort_moments_cavity448x448x100_counters.txt"),
            "roofline_step_alu": roofline_alu(rs, "step", "step_cavity448x448x100_alu.txt"),
            "roofline_sort_moments_alu": roofline_alu(rs, "sort_moments",
                                                      "sort_moments_cavity448x448x100_alu.txt"),
        }
        # the roofline is taken where the state leaves the 256 MB last-level cache: the
        # dominant entry point of the 2e7-particle cavity (the 1e6 one fits in it)
        dom = max(rs["kern"], key=lambda k: rs["kern"][k]["ms"])
        out["roofline"] = dict(roofline_of(rs, dom, f"{dom}_cavity448x448x100_counters.txt"),
                               workload="cavity2d 448x448 cells, 2.0e7 particles")
    else:
        out["roofline"] = dict(out["roofline_1e6"], workload=out["config"]["workload"])
    if not args.no_other:
        out["couette"] = couette_line(torch, F, I)
        out["cylinder"] = cylinder_line(torch, F, I, args.cylinder_steps)
        out["cylinder_amr"] = cylinder_amr_line(torch, F, I, args.amr_steps)
    if not args.no_learned:
        out["learned"] = learned_section(torch)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(I, w)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
