"""fp_rebin (the re-sort of particles grouped by their previous cell) against the oracle's
stable counting sort, bit for bit: offsets, source permutation and every record.

The grouped input is built by the oracle (sort of a seeded state, then one oracle
flight that gives new keys); cases add far movers, deleted and invalid keys, an ungrouped
tail after the grouped range (as injection leaves it), empty and crowded cells, grids one
cell wide, the 1-D channel, and the full 2e7-particle cavity."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2606_15622_amd import inputs as I

pytestmark = pytest.mark.gpu


def fp():
    from paper_2606_15622_amd import fpgpu
    fpgpu.load()
    return fpgpu


def grouped_after_flight(w, state, step=3):
    """Oracle sort of state by its keys, then one oracle flight: particles grouped by old
    cell (offsets off0) carrying their new keys."""
    nc = I.ncells(w)
    key = O.keys(w, state["x"], state["y"])
    perm, off0 = O.bin_particles(nc, key)
    kept = int(off0[-1])
    s = {k: v[perm[:kept]] for k, v in state.items() if k != "key"}
    x, y, vx, vy, vz, key = O.move(w, s["x"], s["y"], s["vx"], s["vy"], s["vz"], s["pid"], step)
    s.update(x=x, y=y, vx=vx, vy=vy, vz=vz, key=key.astype(np.int32))
    return s, off0


def moment_scale(o):
    """Natural scale of every moment entry (theta^k for order 2k), as in the parity of
    fp_moments."""
    th = np.maximum(o[:, 4], 1e-300)
    scale = np.ones(o.shape)
    scale[:, 1:4] = np.sqrt(th)[:, None] + np.abs(o[:, 1:4])
    scale[:, 4:11] = th[:, None]
    scale[:, 11:21] = th[:, None] ** 1.5
    scale[:, 21:27] = th[:, None] ** 2
    scale[:, 27:30] = th[:, None] ** 2.5
    scale[:, 30] = th ** 3
    return scale


def run_rebin(F, w, s, off0, expect_errors=0):
    """fp_rebin twice without moments, then with the moment gather, then with moments and
    time-average sums: the sort must equal the oracle's bit for bit each time, the
    moments match the oracle's moments of the oracle-sorted cells (1e-10 of the natural
    scale, as for fp_moments), the sums the oracle's sums (as for fp_sample) and, bit for
    bit, what fp_sample adds from the gathered moments."""
    nc = I.ncells(w)
    n = s["x"].shape[0]
    ctx = F.Context(w, max(n, 1))
    a = F.Particles.from_numpy(w, s)
    b = F.Particles(n, a.dtype, w["geometry"] != "couette1d")
    src_off = torch.from_numpy(np.ascontiguousarray(off0, dtype=np.int32)).cuda()
    off = torch.full((nc + 1,), -7, dtype=torch.int32, device="cuda")
    perm = torch.full((max(n, 1),), -7, dtype=torch.int32, device="cuda")
    mom = torch.full((nc, 32), -7.0, dtype=torch.float64, device="cuda")
    operm, ooff = O.bin_particles(nc, s["key"])
    kept = int(ooff[-1])
    srt = {k: np.asarray(s[k])[operm[:kept]] for k in s}
    samp0 = np.random.default_rng(9).uniform(0.0, 1e3, (nc, 16))
    samp = torch.from_numpy(samp0).cuda()
    for rep in range(4):     # repeated: the counters must be left clean by every call
        with_mom = rep >= 2
        with_samp = rep == 3
        ctx.rebin(a, src_off, b, off, perm, mom if with_mom else None,
                  samp if with_samp else None)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(off.cpu().numpy(), ooff)
        np.testing.assert_array_equal(perm.cpu().numpy()[:kept], operm[:kept])
        b.n = kept
        out = b.numpy()
        for k in ("x", "y", "vx", "vy", "vz", "pid", "key"):
            if k == "y" and w["geometry"] == "couette1d":
                continue
            np.testing.assert_array_equal(out[k], srt[k], err_msg=k)
        b.n = n
        if with_mom and nc > 0:
            o = O.moments(ooff, srt["vx"], srt["vy"], srt["vz"])
            g = mom.cpu().numpy()
            np.testing.assert_array_equal(g[:, 0], o[:, 0])
            assert np.all(np.abs(g - o) <= 1e-10 * moment_scale(o))
        if with_samp and nc > 0:
            gs = samp.cpu().numpy()
            osamp = O.sample(ooff, srt["vx"], srt["vy"], srt["vz"], samp0.copy())
            scale = np.abs(osamp) + np.repeat(np.maximum(osamp[:, :1], 1), 16, 1) * 1e6
            assert np.all(np.abs(gs - osamp) <= 1e-10 * scale)
            ref = torch.from_numpy(samp0).cuda()
            ctx.sample(mom, ref)
            np.testing.assert_array_equal(gs, ref.cpu().numpy())
    assert ctx.error_count() == 4 * expect_errors
    return kept


def test_cavity_after_one_flight():
    F = fp()
    w = I.cavity(ncell=100, ppc=100, precision="f32", kn=1.0)
    s, off0 = grouped_after_flight(w, I.maxwellian_state(w, seed=3))
    moved = np.count_nonzero(s["key"] != np.repeat(np.arange(I.ncells(w)), np.diff(off0)))
    assert moved > 1000
    run_rebin(F, w, s, off0)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_far_movers_deleted_and_invalid(prec):
    F = fp()
    w = I.cavity(ncell=40, ppc=60, precision=prec)
    s, off0 = grouped_after_flight(w, I.maxwellian_state(w, seed=4))
    n = s["x"].shape[0]
    rng = np.random.default_rng(4)
    nc = I.ncells(w)
    far = rng.random(n) < 0.03
    s["key"][far] = rng.integers(0, nc, far.sum())
    gone = rng.random(n) < 0.01
    s["key"][gone] = nc
    bad = rng.choice(n, 5, replace=False)
    s["key"][bad] = [-1, nc + 1, 10**6, -5, nc + 7]
    run_rebin(F, w, s, off0, expect_errors=5)


def test_ungrouped_tail_after_grouped_range():
    F = fp()
    w = I.cavity(ncell=30, ppc=50, precision="f32")
    s, off0 = grouped_after_flight(w, I.maxwellian_state(w, seed=5))
    t = I.scattered_state(w, 20_000, seed=6)
    t["key"] = O.keys(w, t["x"], t["y"])
    t["key"][::17] = I.ncells(w)                     # some never entered
    t["pid"] = t["pid"] + 10**7
    s = {k: np.concatenate([np.asarray(s[k]), np.asarray(t[k]).astype(np.asarray(s[k]).dtype)]) for k in s}
    run_rebin(F, w, s, off0)


def test_everything_ungrouped():
    F = fp()
    w = I.cavity(ncell=25, precision="f64")
    s = I.scattered_state(w, 30_001, seed=7)
    s["key"] = O.keys(w, s["x"], s["y"])
    run_rebin(F, w, s, np.zeros(I.ncells(w) + 1, dtype=np.int32))


def test_crowded_and_empty_cells():
    F = fp()
    w = I.cavity(ncell=12, precision="f32")
    counts = np.zeros(144, dtype=np.int64)
    counts[[5, 6, 77]] = [3000, 1, 4500]
    counts[[20, 21, 22, 23]] = [256, 257, 200, 129]   # the re-sort's mask limits
    counts[100:110] = 7
    vx, vy, vz, off0 = I.mixture_cells(counts, seed=8, precision="f32")
    n = int(off0[-1])
    rng = np.random.default_rng(8)
    cell = np.repeat(np.arange(144), counts)
    key = cell.copy()
    step = rng.integers(-1, 2, (2, n))               # one neighbour step, clipped to the grid
    kx = np.clip(cell % 12 + step[0], 0, 11)
    ky = np.clip(cell // 12 + step[1], 0, 11)
    key = (ky * 12 + kx).astype(np.int32)
    x = (w["x0"] + (kx + 0.5) * w["dx"]).astype(np.float32).astype(np.float64)
    y = (w["y0"] + (ky + 0.5) * w["dy"]).astype(np.float32).astype(np.float64)
    s = dict(x=x, y=y, vx=vx, vy=vy, vz=vz, pid=rng.permutation(n).astype(np.uint32), key=key)
    run_rebin(F, w, s, off0.astype(np.int32))


@pytest.mark.parametrize("nx,ny", [(1, 9), (9, 1), (2, 2)])
def test_narrow_grids(nx, ny):
    F = fp()
    w = I.cavity(ncell=9, ppc=40, precision="f64")
    w = dict(w, nx=nx, ny=ny, lx=nx * w["dx"], ly=ny * w["dy"])
    s, off0 = grouped_after_flight(w, I.maxwellian_state(w, seed=9))
    run_rebin(F, w, s, off0)


def test_channel_1d_and_empty():
    F = fp()
    w = I.couette(ncell=100, ppc=100, precision="f64")
    s, off0 = grouped_after_flight(w, I.maxwellian_state(w, seed=10))
    run_rebin(F, w, s, off0)
    e = {k: v[:0] for k, v in s.items()}
    run_rebin(F, w, e, np.zeros(101, dtype=np.int32))


@pytest.mark.parametrize("lanes", [4, 8, 16, 32, 64])
def test_every_group_width(lanes):
    """Every lanes-per-cell width of the count and gather kernels (their group prefix
    sums and reductions), on a grid wider than the gather's column strips (70 = 32 + 32
    + a ragged 6), with 1 % far movers."""
    F = fp()
    w = dict(I.cavity(ncell=70, ppc=90, precision="f32", kn=1.0), lanes=lanes)
    s, off0 = grouped_after_flight(w, I.maxwellian_state(w, seed=11))
    rng = np.random.default_rng(11)
    far = rng.random(s["x"].shape[0]) < 0.01
    s["key"][far] = rng.integers(0, I.ncells(w), far.sum())
    run_rebin(F, w, s, off0)


def test_full_size_cavity():
    """2e7 particles on 448 x 448 cells, the launch shape of the scaled benchmark."""
    F = fp()
    w = I.cavity(ncell=448, ppc=100, precision="f32", seed=2)
    s, off0 = grouped_after_flight(w, I.maxwellian_state(w))
    assert s["x"].shape[0] > 1.9e7
    run_rebin(F, w, s, off0)
