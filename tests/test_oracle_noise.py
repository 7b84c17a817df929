"""Pins of the oracle's noise source (sampling step, Sec. III-B, Eq. (3)).

Philox4x32-10 is pinned by the published known-answer vectors; the uniform
map by exact arithmetic; Box-Muller by its distribution (moments, KS test,
channel independence) and by special words whose normals have closed forms.
"""
import math
import os

import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            v = [int(t, 16) for t in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat())
def test_philox_known_answers(ctr, key, expect):
    assert O.philox(ctr, key) == expect


def test_u01_exact_and_open_interval():
    assert O.u01(0) == 2.0 ** -24
    assert O.u01(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    assert O.u01(1 << 9) == 3.0 * 2.0 ** -24
    # the low 9 bits are discarded
    assert O.u01(0x12345678) == O.u01(0x12345678 | 0x1FF)
    rng = np.random.default_rng(0)
    for w in rng.integers(0, 2 ** 32, size=2000, dtype=np.uint64):
        u = O.u01(int(w))
        assert 0.0 < u < 1.0
        assert float(np.float32(u)) == u  # exact in binary32 as well


def test_normals_of_known_answer_block():
    # counter (m, k, s, ch) = (0, 0, 0, 0) under seed 0 is the first KAT block;
    # its normals must be Box-Muller of the published words, evaluated here
    # with Python's libm independently of the oracle's C code.
    ctr, key, words = _kat()[0]
    u = [O.u01(w) for w in words]
    r0 = math.sqrt(-2.0 * math.log(u[0]))
    r1 = math.sqrt(-2.0 * math.log(u[2]))
    expect = [r0 * math.cos(2 * math.pi * u[1]), r0 * math.sin(2 * math.pi * u[1]),
              r1 * math.cos(2 * math.pi * u[3]), r1 * math.sin(2 * math.pi * u[3])]
    z = O.normals(0, 0, 0, 0, 0)
    np.testing.assert_allclose(z, expect, rtol=1e-15, atol=1e-15)
    # the pair radius is the same for both members of a pair
    assert abs(z[0] ** 2 + z[1] ** 2 - r0 * r0) < 1e-12


def test_seed_maps_to_key_words():
    # seed = key1 << 32 | key0
    ctr, key, words = _kat()[2]
    seed = (key[1] << 32) | key[0]
    # orc_normals builds the counter (m, k, s, ch); reproduce the third KAT block
    z = O.normals(seed, ctr[0], ctr[1], ctr[2], ctr[3])
    u = [O.u01(w) for w in words]
    r0 = math.sqrt(-2.0 * math.log(u[0]))
    assert abs(z[0] - r0 * math.cos(2 * math.pi * u[1])) < 1e-14


def test_normals_distribution():
    # 4 * 64 * 1024 = 262144 normals over (m, k) counters of one solve
    zs = np.array([O.normals(7, m, k, 3, 0) for m in range(256) for k in range(256)])
    flat = zs.ravel()
    assert abs(flat.mean()) < 0.01
    assert abs(flat.var() - 1.0) < 0.01
    assert stats.kstest(flat, "norm").pvalue > 1e-3
    # channels are uncorrelated, including the two members of a pair
    c = np.corrcoef(zs.T)
    assert np.max(np.abs(c - np.eye(4))) < 0.01
    # the fourth moment of a standard normal is 3
    assert abs(np.mean(flat ** 4) - 3.0) < 0.05


def test_counter_words_select_independent_streams():
    a = O.normals(1, 5, 6, 7, 0)
    assert not np.allclose(a, O.normals(1, 5, 6, 7, 1))  # channel block
    assert not np.allclose(a, O.normals(1, 5, 6, 8, 0))  # solve counter
    assert not np.allclose(a, O.normals(1, 6, 5, 7, 0))  # m and k not symmetric
    assert not np.allclose(a, O.normals(2, 5, 6, 7, 0))  # seed
