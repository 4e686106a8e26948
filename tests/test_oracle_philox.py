"""Pins of the oracle's Philox4x32-10 and normal generator (CPU)."""
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from tests.ref_philox import philox4x32_10 as ref

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        f = [int(t, 16) for t in line.replace("->", " ").split()]
        rows.append((f[0:4], f[4:6], f[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,out", _kat())
def test_known_answers(ctr, key, out):
    assert O.philox(ctr, key) == out
    assert ref(ctr, key) == out


def test_matches_bigint_reference_on_random_counters():
    rng = np.random.default_rng(11)
    for _ in range(2000):
        ctr = [int(v) for v in rng.integers(0, 2**32, 4, dtype=np.uint64)]
        key = [int(v) for v in rng.integers(0, 2**32, 2, dtype=np.uint64)]
        assert O.philox(ctr, key) == ref(ctr, key)


def test_uniform_mapping_and_counter_layout():
    seed = (7 << 32) | 12345
    for pid, step, purpose, sub in [(0, 0, 3, 0), (5, 99, 4, 2), (2**32 - 1, 7, 3, 1)]:
        r = ref([pid, step, purpose, sub], [seed & 0xFFFFFFFF, seed >> 32])
        u = O.uniforms(seed, pid, step, purpose, sub)
        np.testing.assert_array_equal(u, (np.array(r, dtype=np.float64) + 0.5) * 2.0**-32)
        assert np.all((u > 0) & (u < 1))
        z = O.normals3(seed, pid, step, purpose, sub)
        r0 = math.sqrt(-2 * math.log(u[0]))
        assert z[0] == pytest.approx(r0 * math.cos(2 * math.pi * u[1]), rel=1e-14, abs=1e-15)
        assert z[1] == pytest.approx(r0 * math.sin(2 * math.pi * u[1]), rel=1e-14, abs=1e-15)
        r1 = math.sqrt(-2 * math.log(u[2]))
        assert z[2] == pytest.approx(r1 * math.cos(2 * math.pi * u[3]), rel=1e-14, abs=1e-15)


def test_normals_are_standard():
    z = np.array([O.normals3(1, p, 3, 3, 0) for p in range(20000)])
    assert abs(z.mean()) < 0.02
    assert abs(z.var() - 1.0) < 0.03
    # kurtosis of a normal is 3
    assert abs((z**4).mean() / z.var() ** 2 - 3.0) < 0.15
