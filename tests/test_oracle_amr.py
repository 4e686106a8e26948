"""Pins of the adaptive-quadtree oracle (Sec. "Extension to External Aerodynamics",
refinement and coarsening criteria): depth-first numbering and the fine-cell map against
an independent geometric construction, parent sums against the moments of the merged
particle population, each criterion on hand-made fields with the deviations worked out
by hand, and conservation of the sampling sums through splits and merges."""
import numpy as np
import pytest

from oracle import amr_oracle as A

FNUM, MASS = 2.0, 3.0
PRM = dict(tau_grad=0.10, tau_coarse=0.05, shock_factor=1.2, p_inf=1e30, n_max=1e9,
           n_grad=20, age_min=100, eps=1e-300)


def acc_row(nbar, ns, U, th):
    """Sampling sums of ns steps with nbar particles per step of mean velocity U and
    isotropic temperature th (per mass)."""
    S = nbar * ns
    r = np.zeros(A.SAMP)
    r[0] = S
    r[1:4] = S * np.asarray(U)
    vv = np.outer(U, U) + th * np.eye(3)
    r[4:10] = S * vv[[0, 0, 0, 1, 1, 2], [0, 1, 2, 1, 2, 2]]
    r[13] = ns
    return r


def refined_tree(nbx=2, nby=2, L=2, split=((0, 0, 0),)):
    t = A.Tree(nbx, nby, L)
    for (l, ix, iy) in split:
        t.state[l][iy, ix] = A.REFINED
        for c in range(4):
            t.state[l + 1][2 * iy + (c >> 1), 2 * ix + (c & 1)] = A.LEAF
    return t


def test_depth_first_numbering_and_fine_map():
    t = refined_tree(3, 2, 2, split=((0, 1, 0), (1, 3, 1), (0, 2, 1)))
    lv = t.leaves()
    # independent order: base cell row-major, then Morton index of the leaf's first fine cell
    def key(leaf):
        l, ix, iy = leaf
        s = t.L - l
        fx, fy = ix << s, iy << s
        b = (fy >> t.L) * t.nbx + (fx >> t.L)
        return b, A.morton(fx & 3, fy & 3, t.L)
    assert lv == sorted(lv, key=key)
    assert len(lv) == 6 - 2 + 8 - 1 + 4
    m = t.leaf_map()
    nxf = t.nbx << t.L
    for f in range(m.size):
        fx, fy = f % nxf, f // nxf
        hits = [i for i, (l, ix, iy) in enumerate(lv) if fx >> (t.L - l) == ix and fy >> (t.L - l) == iy]
        assert hits == [m[f]]
    for d in range(16):
        assert A.morton(*A.demorton(d, 2), 2) == d


def test_leaf_volumes():
    t = refined_tree(2, 2, 2)
    rng = np.random.default_rng(0)
    fine = rng.uniform(0, 1, (t.nby << 2) * (t.nbx << 2))
    fine[:5] = 0.0
    vol, nvol = A.leaf_volumes(t, fine, FNUM, 1.0)
    assert abs(vol.sum() - fine.sum()) < 1e-12
    m = t.leaf_map()
    for i in range(len(vol)):
        assert vol[i] == pytest.approx(fine[m == i].sum(), rel=1e-14)
        assert nvol[i] == FNUM / vol[i] if vol[i] > 0 else True
    t0 = A.Tree(2, 2, 0)
    f0 = rng.uniform(0, 1, 4)
    v0, _ = A.leaf_volumes(t0, f0, FNUM, 1.0)
    np.testing.assert_array_equal(v0, f0)


def test_parent_sums_are_the_merged_population():
    rng = np.random.default_rng(1)
    t = refined_tree(1, 1, 1)
    acc = np.zeros((4, A.SAMP))
    pops = []
    for i in range(4):
        v = rng.standard_normal((50 + 10 * i, 3)) * (1 + i) + i
        pops.append(v)
        acc[i, 0] = len(v)
        acc[i, 1:4] = v.sum(0)
        vv = np.einsum("pi,pj->ij", v, v)
        acc[i, 4:10] = vv[[0, 0, 0, 1, 1, 2], [0, 1, 2, 1, 2, 2]]
        acc[i, 13] = 1
    vol = np.array([1.0, 2.0, 3.0, 4.0])
    sums = A.node_sums(t, acc, vol)
    allv = np.concatenate(pops)
    rho, th, P = A.fields(sums[0][0, 0], FNUM, MASS)
    U = allv.mean(0)
    assert rho == pytest.approx(len(allv) * FNUM / 10.0, rel=1e-14)
    assert th == pytest.approx(((allv - U) ** 2).sum(1).mean() / 3, rel=1e-12)
    assert P == pytest.approx(rho * MASS * th, rel=1e-14)


def test_no_split_of_a_uniform_base_grid_and_count_limit():
    t = A.Tree(2, 2, 2)
    acc = np.array([acc_row(100, 10, (1, 0, 0), 2.0)] * 4)
    vol = np.ones(4)
    prm = dict(PRM)
    t2, ref, mer = A.adapt(t, acc, vol, prm, 10, FNUM, MASS)
    assert not ref and not mer and len(t2.leaves()) == 4
    assert np.all(t2.age[0] == 10)
    acc[2, 0] *= 1.5                    # 150 particles per step in leaf 2
    prm["n_max"] = 120
    t3, ref, _ = A.adapt(t, acc, vol, prm, 10, FNUM, MASS)
    assert ref == {(0, 0, 1)}           # leaf 2 = base cell (0, 1)
    assert len(t3.leaves()) == 7 and np.all(t3.state[1][2:4, 0:2] == A.LEAF)
    assert np.all(t3.age[1][2:4, 0:2] == 0)


def test_shock_criterion():
    t = A.Tree(2, 1, 1)
    acc = np.array([acc_row(100, 10, (0, 0, 0), 2.0), acc_row(100, 10, (0, 0, 0), 3.0)])
    vol = np.ones(2)
    prm = dict(PRM)
    p0 = 100 * FNUM * MASS * 2.0        # pressure of leaf 0
    prm["p_inf"] = p0 / 1.2 * 1.0001    # leaf 0 just below 1.2 p_inf, leaf 1 above
    _, ref, _ = A.adapt(t, acc, vol, prm, 1, FNUM, MASS)
    assert ref == {(0, 1, 0)}
    prm["n_grad"] = 10**6               # too few particles: no shock test
    _, ref, _ = A.adapt(t, acc, vol, prm, 1, FNUM, MASS)
    assert not ref


def test_gradient_criterion_worked_example():
    # children of one base cell: densities 1.2 : 1 : 1 : 1 at one temperature;
    # parent density 1.05, deviations 0.15/1.2 = 0.125 (> 0.10) and 0.05/1 = 0.05
    t = refined_tree(1, 1, 1)
    acc = np.array([acc_row(120, 4, (0, 0, 0), 1.0)] + [acc_row(100, 4, (0, 0, 0), 1.0)] * 3)
    vol = np.ones(4)
    sums = A.node_sums(t, acc, vol)
    assert A.fields(sums[0][0, 0], FNUM, MASS)[0] == pytest.approx(105 * FNUM)
    _, ref, mer = A.adapt(t, acc, vol, dict(PRM), 1, FNUM, MASS)
    assert ref == set() and not mer          # level 1 is the finest of this tree (L = 1)
    t2 = refined_tree(1, 1, 2)
    _, ref, mer = A.adapt(t2, acc, vol, dict(PRM), 1, FNUM, MASS)
    assert ref == {(1, 0, 0)} and not mer
    # temperature instead: 1.3 : 1 : 1 : 1 at one density -> parent theta 1.075,
    # deviation 0.225/1.3 = 0.173 for child 0; P follows theta
    acc = np.array([acc_row(100, 4, (0, 0, 0), 1.3)] + [acc_row(100, 4, (0, 0, 0), 1.0)] * 3)
    _, ref, _ = A.adapt(t2, acc, vol, dict(PRM), 1, FNUM, MASS)
    assert ref == {(1, 0, 0)}


def test_coarsening_rules():
    t = refined_tree(1, 1, 2)
    for c in range(4):
        t.age[1][c >> 1, c & 1] = 150
    base = [acc_row(100, 4, (0.5, 0, 0), 1.0)] * 4
    vol = np.ones(4)
    t2, ref, mer = A.adapt(t, np.array(base), vol, dict(PRM), 5, FNUM, MASS)
    assert mer == {(0, 0, 0)} and not ref
    assert t2.leaves() == [(0, 0, 0)] and t2.age[0][0, 0] == 0
    assert np.all(t2.state[1] == A.ABSENT)
    young = t.copy()
    young.age[1][1, 1] = 99
    _, _, mer = A.adapt(young, np.array(base), vol, dict(PRM), 5, FNUM, MASS)
    assert not mer
    prm = dict(PRM)
    prm["n_max"] = 350                  # merged mean count 400 > N_max
    _, _, mer = A.adapt(t, np.array(base), vol, prm, 5, FNUM, MASS)
    assert not mer
    # density 1.13 : 1 : 1 : 1 -> parent 1.0325, child-0 deviation 0.097/1.13 = 0.086
    # (> 0.05: no merge) while no child splits (all deviations < 0.10)
    acc = np.array([acc_row(113, 4, (0.5, 0, 0), 1.0)] + base[1:])
    _, ref, mer = A.adapt(t, acc, vol, dict(PRM), 5, FNUM, MASS)
    assert not ref and not mer
    # 1.04 : 1 : 1 : 1 -> deviations 0.03/1.04 and 0.01: merge
    acc = np.array([acc_row(104, 4, (0.5, 0, 0), 1.0)] + base[1:])
    _, _, mer = A.adapt(t, acc, vol, dict(PRM), 5, FNUM, MASS)
    assert mer == {(0, 0, 0)}


def test_empty_and_solid_leaves():
    t = refined_tree(1, 1, 2)
    for c in range(4):
        t.age[1][c >> 1, c & 1] = 500
    acc = np.array([acc_row(100, 4, (0, 0, 0), 1.0), np.zeros(A.SAMP), np.zeros(A.SAMP),
                    acc_row(100, 4, (0, 0, 0), 1.0)])
    acc[1, 13] = acc[2, 13] = 4
    vol = np.array([1.0, 0.0, 1.0, 1.0])
    t2, ref, mer = A.adapt(t, acc, vol, dict(PRM), 5, FNUM, MASS)
    # the empty children take no criterion; children 0 and 3 deviate from the parent
    # (density 200/3 per unit volume against 100): 0.33 > 0.10 -> split
    assert ref == {(1, 0, 0), (1, 1, 1)} and not mer
    prm = dict(PRM)
    prm["n_max"] = 10
    acc0 = np.zeros((4, A.SAMP))
    acc0[:, 13] = 4
    acc0[1, 0] = 4 * 50
    _, ref, _ = A.adapt(t, acc0, vol, prm, 5, FNUM, MASS)
    assert ref == set()                 # the only crowded leaf has no gas volume


def test_sampling_sums_survive_adaptation():
    t = refined_tree(2, 1, 2)
    rng = np.random.default_rng(3)
    fine = rng.uniform(0.5, 1.0, (1 << 2) * (2 << 2))
    vol, _ = A.leaf_volumes(t, fine, FNUM, 1.0)
    n = len(t.leaves())
    samp = np.array([acc_row(rng.uniform(50, 150), 7, rng.standard_normal(3), rng.uniform(1, 2))
                     for _ in range(n)])
    t2 = t.copy()
    # split base cell (1, 0) and merge the children of base cell (0, 0)
    t2.state[0][0, 1] = A.REFINED
    t2.state[1][0:2, 2:4] = A.LEAF
    t2.state[0][0, 0] = A.LEAF
    t2.state[1][0:2, 0:2] = A.ABSENT
    vol2, _ = A.leaf_volumes(t2, fine, FNUM, 1.0)
    s2 = A.remap_samp(t, t2, samp, vol, vol2)
    assert s2[:, 0].sum() == pytest.approx(samp[:, 0].sum(), rel=1e-14)
    assert s2[:, 1:13].sum(0) == pytest.approx(samp[:, 1:13].sum(0), rel=1e-12)
    # a split child keeps its parent's averaged velocity; the merged cell is the sum
    parent = samp[4]
    for i in range(1, 5):
        np.testing.assert_allclose(s2[i, 1:4] / s2[i, 0], parent[1:4] / parent[0], rtol=1e-14)
        assert s2[i, 13] == parent[13]
    np.testing.assert_allclose(s2[0, :13], samp[:4, :13].sum(0), rtol=1e-14)


def test_map_keys():
    t = refined_tree(2, 1, 1)
    m = t.leaf_map()
    k = A.map_keys(m, np.array([0, 3, 8, 7, 8]), 8, 5)
    assert list(k) == [m[0], m[3], 5, m[7], 5]


def test_level0_loop_is_the_uniform_oracle_loop():
    """The tree loop composed in Python, with no level below the base grid and no
    adaptation, against the oracle's own C loop of the open domain: the same numbers."""
    from oracle import oracle as O
    from paper_2606_15622_amd import inputs as I
    w = I.cylinder(cell=2e-2, nx=40, ny=30, fnum=1e15, precision="f64")
    s = I.freestream_state(w, seed=5)
    s["key"] = O.keys(w, s["x"], s["y"])
    n0 = s["x"].shape[0]
    fine = O.cell_volumes(w)
    a, apn, tree, amom, arec, ast, asamp, avol = A.run_open_amr(w, s, n0, 0, 3, 0, PRM, 0, fine)
    o, opn, omom, orec, ost, osamp = O.run_open(w, s, n0, 0, 3, capacity=4 * n0, n_skip=0)
    nc = w["nx"] * w["ny"]
    keep = o["key"] < nc
    o = {k: v[keep] for k, v in o.items()}
    live = a["key"] < nc
    assert apn == opn and len(tree.leaves()) == nc
    for k in ("x", "y", "vx", "vy", "vz", "pid", "key"):
        np.testing.assert_array_equal(a[k][live], o[k], err_msg=k)
    np.testing.assert_array_equal(ast, ost)
    np.testing.assert_array_equal(asamp, osamp)
    np.testing.assert_array_equal(avol, fine)
