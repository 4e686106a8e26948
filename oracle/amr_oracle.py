"""Plain FP64 oracle of the adaptive quadtree of the cylinder domain.  TEST INFRASTRUCTURE
ONLY (tests, smoke, CPU baseline).

Sec. "Extension to External Aerodynamics", Problem Description: hierarchical Cartesian
quadtree; a cell is split into four children when the largest normalised deviation
|phi_i - phi_parent| / (|phi_i| + eps) of density, temperature and pressure from its
parent exceeds tau_grad (0.10), when its particle count exceeds N_max, or when its
pressure exceeds a factor (1.2) of the free-stream pressure; four sibling leaves merge
into their parent when their deviations from it are all below tau_coarse (0.05), their
total particle count is low and every one of them has stayed unchanged for a number of
steps (2000).

Readings (the paper is silent on these):
  * the fields are averages over the steps since the last adaptation (sampling sums of
    the leaves: sum N, sum v, sum v v, number of samples in entry 13), rho = (sum N / samples) fnum /
    V (gas volume), U = sum v / sum N, theta = (sum |v|^2 / sum N - |U|^2) / 3 (the
    temperature up to the factor m/k_B, which cancels in the deviation), P = rho m theta;
  * a parent's sums are the sums of its four children (the merged population), its
    volume the sum of theirs; a level-0 cell has no parent and no gradient criterion;
  * eps only guards the division; a leaf whose sums hold fewer than n_grad particles
    takes neither the gradient nor the shock criterion (its fields are noise), and counts
    as zero deviation in the coarsening test; a leaf with no gas volume never splits;
  * "total particle count sufficiently low" is: mean count of the merged cell <= N_max
    (it would not split again at once), and the merged cell must not meet the shock
    criterion;
  * one level per adaptation: splits act on the leaves, merges on parents of four
    leaves, both decided on the tree as it was; ages count steps, new leaves start at 0;
  * leaves are numbered depth first (base cells row-major, children in the order
    (0,0) (1,0) (0,1) (1,1)); the context's grid is the finest level;
  * the sampling sums survive an adaptation: a new child takes its parent's sums scaled
    by its share of the parent's gas volume (its averaged fields are the parent's), a
    merged cell the sums of its children; the sample count is carried over.

Summation orders (children in the order above; fine cells of a leaf depth first) are
fixed so that the GPU reproduces every decision and volume bit for bit.
"""
import numpy as np

ABSENT, LEAF, REFINED = 0, 1, 2
SAMP = 16


def morton(lx, ly, L):
    d = 0
    for k in range(L):
        d |= ((lx >> k) & 1) << (2 * k)
        d |= ((ly >> k) & 1) << (2 * k + 1)
    return d


def demorton(d, L):
    lx = ly = 0
    for k in range(L):
        lx |= ((d >> (2 * k)) & 1) << k
        ly |= ((d >> (2 * k + 1)) & 1) << k
    return lx, ly


class Tree:
    """state[l] and age[l]: arrays [ny_l][nx_l] of the nodes of level l (nx_l = nbx 2^l)."""

    def __init__(self, nbx, nby, L):
        self.nbx, self.nby, self.L = nbx, nby, L
        self.state = [np.zeros((nby << l, nbx << l), dtype=np.int8) for l in range(L + 1)]
        self.age = [np.zeros((nby << l, nbx << l), dtype=np.int64) for l in range(L + 1)]
        self.state[0][:, :] = LEAF

    def copy(self):
        t = Tree(self.nbx, self.nby, self.L)
        t.state = [a.copy() for a in self.state]
        t.age = [a.copy() for a in self.age]
        return t

    def leaves(self):
        """(l, ix, iy) of every leaf, depth first."""
        out = []

        def walk(l, ix, iy):
            st = self.state[l][iy, ix]
            if st == LEAF:
                out.append((l, ix, iy))
            elif st == REFINED:
                for c in range(4):
                    walk(l + 1, 2 * ix + (c & 1), 2 * iy + (c >> 1))

        for by in range(self.nby):
            for bx in range(self.nbx):
                walk(0, bx, by)
        return out

    def fine_cells(self, l, ix, iy):
        """Row-major fine indices of node (l, ix, iy), depth first."""
        s = self.L - l
        nxf = self.nbx << self.L
        out = []
        for d in range(1 << (2 * s)):
            lx, ly = demorton(d, s)
            out.append(((iy << s) + ly) * nxf + (ix << s) + lx)
        return out

    def leaf_map(self):
        """leafmap[fine row-major] = id of the leaf that contains the fine cell."""
        m = np.full((self.nby << self.L) * (self.nbx << self.L), -1, dtype=np.int32)
        for i, (l, ix, iy) in enumerate(self.leaves()):
            m[self.fine_cells(l, ix, iy)] = i
        return m


def leaf_volumes(tree, fine_vol, fnum, full_fine):
    """Gas volume of every leaf (its fine cells summed depth first) and fnum / volume
    (the full cell volume where the gas volume is 0)."""
    vol, nvol = [], []
    for (l, ix, iy) in tree.leaves():
        v = 0.0
        for f in tree.fine_cells(l, ix, iy):
            v = v + float(fine_vol[f])
        full = full_fine * float(1 << (2 * (tree.L - l)))
        vol.append(v)
        nvol.append(fnum / (v if v > 0.0 else full))
    return np.array(vol), np.array(nvol)


def node_sums(tree, acc, vol):
    """sums[l][iy, ix] = (S0, S1x, S1y, S1z, S2, V, n_samples) of every leaf and refined
    node: S0 = sum N, S1 = sum v, S2 = sum |v|^2 from the leaf sampling sums acc; a
    refined node adds its children in the order (0,0) (1,0) (0,1) (1,1)."""
    L = tree.L
    sums = [np.zeros((tree.nby << l, tree.nbx << l, 7)) for l in range(L + 1)]
    for i, (l, ix, iy) in enumerate(tree.leaves()):
        a = acc[i]
        s2 = (a[4] + a[7]) + a[9]
        sums[l][iy, ix] = [a[0], a[1], a[2], a[3], s2, vol[i], a[13]]
    for l in range(L - 1, -1, -1):
        for iy in range(tree.nby << l):
            for ix in range(tree.nbx << l):
                if tree.state[l][iy, ix] != REFINED:
                    continue
                s = sums[l + 1][2 * iy, 2 * ix].copy()
                for c in (1, 2, 3):
                    ch = sums[l + 1][2 * iy + (c >> 1), 2 * ix + (c & 1)]
                    s[:6] = s[:6] + ch[:6]
                sums[l][iy, ix] = s
    return sums


def fields(s, fnum, mass):
    """(rho, theta, P) of node sums s (rho in m^-3, P in Pa)."""
    S0, V, ns = s[0], s[5], s[6]
    u0, u1, u2 = s[1] / S0, s[2] / S0, s[3] / S0
    th = (s[4] / S0 - ((u0 * u0 + u1 * u1) + u2 * u2)) / 3.0
    rho = ((S0 / ns) * fnum) / V
    return rho, th, (rho * mass) * th


def deviation(a, b, eps):
    return abs(a - b) / (abs(a) + eps)


def max_dev(fi, fp, eps):
    return max(deviation(fi[0], fp[0], eps), deviation(fi[1], fp[1], eps),
               deviation(fi[2], fp[2], eps))


def refine_flags(tree, sums, prm, fnum, mass):
    """Leaves (l, ix, iy) flagged for splitting."""
    out = set()
    for (l, ix, iy) in tree.leaves():
        if l >= tree.L:
            continue
        s = sums[l][iy, ix]
        S0, V, ns = s[0], s[5], s[6]
        if not V > 0.0:
            continue
        split = ns > 0 and S0 / ns > prm["n_max"]
        if S0 >= prm["n_grad"]:
            f = fields(s, fnum, mass)
            if f[2] > prm["shock_factor"] * prm["p_inf"]:
                split = True
            if l > 0:
                sp = sums[l - 1][iy >> 1, ix >> 1]
                if sp[0] >= prm["n_grad"] and max_dev(f, fields(sp, fnum, mass), prm["eps"]) > prm["tau_grad"]:
                    split = True
        if split:
            out.add((l, ix, iy))
    return out


def merge_flags(tree, sums, refine, prm, fnum, mass):
    """Refined nodes (l, ix, iy) whose four children (all leaves) merge."""
    out = set()
    for l in range(tree.L):
        for iy in range(tree.nby << l):
            for ix in range(tree.nbx << l):
                if tree.state[l][iy, ix] != REFINED:
                    continue
                kids = [(l + 1, 2 * ix + (c & 1), 2 * iy + (c >> 1)) for c in range(4)]
                if any(tree.state[k[0]][k[2], k[1]] != LEAF for k in kids):
                    continue
                s = sums[l][iy, ix]
                S0, ns = s[0], s[6]
                if ns > 0 and S0 / ns > prm["n_max"]:
                    continue
                fp = fields(s, fnum, mass) if S0 >= prm["n_grad"] else None
                if fp is not None and fp[2] > prm["shock_factor"] * prm["p_inf"]:
                    continue
                ok = True
                for k in kids:
                    if k in refine or tree.age[k[0]][k[2], k[1]] < prm["age_min"]:
                        ok = False
                        break
                    sk = sums[k[0]][k[2], k[1]]
                    # a child with n_grad particles makes the parent's count >= n_grad
                    if sk[0] >= prm["n_grad"] and \
                            not max_dev(fields(sk, fnum, mass), fp, prm["eps"]) < prm["tau_coarse"]:
                        ok = False
                        break
                if ok:
                    out.add((l, ix, iy))
    return out


def adapt(tree, acc, vol, prm, steps, fnum, mass):
    """One adaptation: returns (new tree, refine set, merge set)."""
    sums = node_sums(tree, acc, vol)
    ref = refine_flags(tree, sums, prm, fnum, mass)
    mer = merge_flags(tree, sums, ref, prm, fnum, mass)
    t = tree.copy()
    for l in range(tree.L + 1):
        for iy in range(tree.nby << l):
            for ix in range(tree.nbx << l):
                st = tree.state[l][iy, ix]
                par = (l - 1, ix >> 1, iy >> 1) if l > 0 else None
                if st == LEAF:
                    if (l, ix, iy) in ref:
                        t.state[l][iy, ix] = REFINED
                    elif par is not None and par in mer:
                        t.state[l][iy, ix] = ABSENT
                        t.age[l][iy, ix] = 0
                    else:
                        t.age[l][iy, ix] = min(tree.age[l][iy, ix] + steps, 2**31 - 1)
                elif st == REFINED:
                    if (l, ix, iy) in mer:
                        t.state[l][iy, ix] = LEAF
                        t.age[l][iy, ix] = 0
                elif par is not None and par in ref:
                    t.state[l][iy, ix] = LEAF
                    t.age[l][iy, ix] = 0
    return t, ref, mer


def remap_samp(old, new, samp_old, vol_old, vol_new):
    """Sampling sums of the new leaves from those of the old ones."""
    out = np.zeros((len(new.leaves()), SAMP))
    omap = old.leaf_map()
    olev = [l for (l, _, _) in old.leaves()]
    for i, (l, ix, iy) in enumerate(new.leaves()):
        f0 = new.fine_cells(l, ix, iy)[0]
        o = omap[f0]
        if olev[o] == l:
            out[i] = samp_old[o]
        elif olev[o] < l:
            r = vol_new[i] / vol_old[o]
            out[i, :13] = samp_old[o, :13] * r
            out[i, 13:] = samp_old[o, 13:]
        else:
            kids = [(l + 1, 2 * ix + (c & 1), 2 * iy + (c >> 1)) for c in range(4)]
            ids = [omap[new.fine_cells(*k)[0]] for k in kids]
            s = samp_old[ids[0]].copy()
            for k in ids[1:]:
                s[:13] = s[:13] + samp_old[k, :13]
            out[i] = s
    return out


def map_keys(leafmap, fine_key, nfine, nleaf):
    """Keys of the leaves from keys of the fine grid (nfine: deleted particle)."""
    k = np.asarray(fine_key)
    out = np.full(k.shape, nleaf, dtype=np.int32)
    live = (k >= 0) & (k < nfine)
    out[live] = leafmap[k[live]]
    return out


def run_open_amr(w, state, pid_next, step0, nsteps, max_level, prm, adapt_every, fine_vol,
                 n_skip=0, wall=None):
    """The open cylinder loop on the tree, composed from the oracle's steps: every
    adapt_every steps an adaptation on the sums since the last one (keys of the particles
    from their positions, sampling sums carried over), then sort, moments, sums, closure
    (density from the leaf gas volumes), velocity update, flight, injection.  fine_vol:
    gas volumes of the fine cells.  Returns (state, pid_next, tree, mom, rec, status,
    samp, vol) after the last step.  wall (optional, [nbins][4]): the exchange sums at the
    body are added to it."""
    from oracle import oracle as O
    nx, ny = int(w["nx"]), int(w["ny"])
    nfine = nx * ny
    L = int(max_level)
    fnum, mass = float(w["fnum"]), float(w["mass"])
    full_fine = (float(w["dx"]) * float(w["dy"])) * float(w["depth"])
    tree = Tree(nx >> L, ny >> L, L)
    vol, nvol = leaf_volumes(tree, fine_vol, fnum, full_fine)
    lm = tree.leaf_map()
    nleaf = len(vol)
    s = {k: np.asarray(state[k], dtype=np.float64).copy() for k in ("x", "y", "vx", "vy", "vz")}
    s["pid"] = np.asarray(state["pid"], dtype=np.uint32).copy()
    key = map_keys(lm, O.keys(w, s["x"], s["y"]), nfine, nleaf)
    acc = np.zeros((nleaf, SAMP))
    samp = np.zeros((nleaf, SAMP))
    since = step0
    mom = rec = st = None
    for step in range(step0, step0 + nsteps):
        if adapt_every > 0 and step - since >= adapt_every:
            new, _, _ = adapt(tree, acc, vol, prm, step - since, fnum, mass)
            vol2, nvol2 = leaf_volumes(new, fine_vol, fnum, full_fine)
            samp = remap_samp(tree, new, samp, vol, vol2)
            lm2 = new.leaf_map()
            nleaf2 = len(vol2)
            live = (key >= 0) & (key < nleaf)
            fk = O.keys(w, s["x"], s["y"])
            key = np.where(live, lm2[fk], nleaf2).astype(np.int32)
            tree, vol, nvol, lm, nleaf = new, vol2, nvol2, lm2, nleaf2
            acc = np.zeros((nleaf, SAMP))
            since = step
        perm, off = O.bin_particles(nleaf, key)
        perm = perm[:off[-1]]
        for k in s:
            s[k] = s[k][perm]
        mom = O.moments(off, s["vx"], s["vy"], s["vz"])
        acc = O.sample(off, s["vx"], s["vy"], s["vz"], acc)
        if step >= n_skip:
            samp = O.sample(off, s["vx"], s["vy"], s["vz"], samp)
        rec, st = O.closure(w, mom, nvol)
        s["vx"], s["vy"], s["vz"] = O.update(w, off, s["vx"], s["vy"], s["vz"], s["pid"], mom, rec, step)
        s["x"], s["y"], s["vx"], s["vy"], s["vz"], fk = O.move(w, s["x"], s["y"], s["vx"], s["vy"],
                                                               s["vz"], s["pid"], step, wall=wall)
        key = map_keys(lm, fk, nfine, nleaf)
        inj, pid_next = O.inject(w, step, pid_next)
        for k in ("x", "y", "vx", "vy", "vz", "pid"):
            s[k] = np.concatenate([s[k], inj[k].astype(s[k].dtype)])
        key = np.concatenate([key, map_keys(lm, inj["key"], nfine, nleaf)])
    s["key"] = key
    return s, pid_next, tree, mom, rec, st, samp, vol
