"""Pins of the oracle of the coefficient-sensitivity probe (Sec. "Heuristic
coefficient-sensitivity probe"): the vectorised Philox against the published known
answers and the big-integer reference, the mask's counter layout and drop rate, and a
network whose perturbed outputs take two values, where the standard deviations over the
passes have a closed form."""
import os

import numpy as np
import pytest

from oracle import mlp_oracle as M
from tests.ref_philox import philox4x32_10 as ref

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def test_vectorised_philox_known_answers_and_reference():
    rows = []
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        f = [int(t, 16) for t in line.replace("->", " ").split()]
        rows.append((f[0:4], f[4:6], f[6:10]))
    for ctr, key, out in rows:
        w = M.philox(*[np.array([v]) for v in ctr], *key)
        assert [int(x[0]) for x in w] == out
    rng = np.random.default_rng(5)
    c = rng.integers(0, 2**32, (4, 500), dtype=np.uint64)
    key = [int(v) for v in rng.integers(0, 2**32, 2, dtype=np.uint64)]
    w = np.stack(M.philox(c[0], c[1], c[2], c[3], *key), 1)
    for i in range(500):
        assert [int(v) for v in w[i]] == ref([int(v) for v in c[:, i]], key)


def test_mask_counter_layout_and_rate():
    seed, p = (9 << 32) | 4242, 0.2
    keep = M.dropout_keep(seed, 5, 7, p)
    assert keep.shape == (5, 7, 3, 128)
    thr = int(np.floor(p * 2**32))
    rng = np.random.default_rng(1)
    for _ in range(300):
        c, k, l, u = (int(rng.integers(5)), int(rng.integers(7)), int(rng.integers(3)),
                      int(rng.integers(128)))
        word = ref([c, k, 6, 32 * l + u // 4], [seed & 0xFFFFFFFF, seed >> 32])[u % 4]
        assert keep[c, k, l, u] == (word >= thr)
    big = M.dropout_keep(seed, 200, 20, p)
    assert abs(big.mean() - (1 - p)) < 0.005
    assert M.dropout_keep(seed, 3, 2, 0.0).all()


def two_valued_net(c3, col, rng):
    """W3 = 0 and b3 = c3: every layer-3 unit has the activation silu(c3) whatever the
    earlier masks; W4 has one non-zero column, so output j of a pass is b4_j or
    b4_j + W4[j, col] s silu(c3), as hidden unit col is kept or dropped."""
    d = {}
    for name, shp in M.SHAPES:
        d[name] = rng.standard_normal(shp) * 0.3
    d["x_std"] = rng.uniform(0.5, 1.5, M.NF)
    d["y_std"] = rng.uniform(0.05, 0.2, M.NO)
    d["W3"] = np.zeros((M.NH, M.NH))
    d["b3"] = np.full(M.NH, c3)
    w4 = np.zeros((M.NO, M.NH))
    w4[:, col] = rng.standard_normal(M.NO)
    d["W4"] = w4
    return d


def moments(n, rng):
    mom = np.zeros((n, 32))
    mom[:, 0] = rng.uniform(20, 200, n)
    mom[:, 4] = rng.uniform(0.5, 2.0, n)
    mom[:, 5:32] = rng.standard_normal((n, 27)) * 0.1
    for q, v in ((5, 1), (8, 1), (10, 1)):
        mom[:, q] += mom[:, 4] * v
    return mom


@pytest.mark.parametrize("p,npass", [(0.2, 50), (0.5, 9)])
def test_two_valued_outputs_closed_form(p, npass):
    rng = np.random.default_rng(3)
    c3, col, n, seed = 0.7, 45, 6, 12345
    d = two_valued_net(c3, col, rng)
    mom = moments(n, rng)
    sens = M.dropout_sensitivity(M.pack(d), mom, 0.01, npass, p, seed, emulate_bf16=False)
    keep = M.dropout_keep(seed, n, npass, p)[:, :, 2, col]
    kept = keep.sum(1)
    a = c3 / (1 + np.exp(-c3))
    amp = np.abs(d["W4"][:9, col] * d["y_std"][:9]) * a / (1 - p)
    # a two-valued sample with k of N passes at the upper value: population std
    # |step| sqrt(k (N - k)) / N
    frac = np.sqrt(kept * (npass - kept)) / npass
    want_c = np.sqrt((amp[:6] ** 2).sum()) * frac
    want_g = np.sqrt((amp[6:9] ** 2).sum()) * frac
    np.testing.assert_allclose(sens[:, 0], want_c, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(sens[:, 1], want_g, rtol=1e-12, atol=1e-15)
    assert np.all(kept > 0) and np.all(kept < npass)


def test_degenerate_cases():
    rng = np.random.default_rng(4)
    d = {name: rng.standard_normal(shp) * 0.2 for name, shp in M.SHAPES}
    d["x_std"] = np.ones(M.NF)
    d["y_std"] = np.ones(M.NO)
    mom = moments(8, rng)
    mom[2] = 0.0
    mom[2, 0] = 1.0          # one particle: no features
    mom[5, 4] = 0.0          # zero temperature
    flat = M.pack(d)
    # identical passes: zero up to the rounding of the mean of equal values
    assert np.all(M.dropout_sensitivity(flat, mom, 0.01, 10, 0.0, 7) < 1e-12)
    assert np.all(M.dropout_sensitivity(flat, mom, 0.01, 1, 0.3, 7) == 0.0)
    s = M.dropout_sensitivity(flat, mom, 0.01, 10, 0.3, 7)
    assert np.all(s[[2, 5]] == 0.0)
    assert np.all(s[[0, 1, 3, 4, 6, 7]] > 0.0)
