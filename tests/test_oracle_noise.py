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


def _python_normals(seed, m, k, s, ch):
    """Box-Muller of the Philox words of counter (m, k, s, ch), evaluated
    with Python's libm (the words themselves are pinned by the KAT above)."""
    w = O.philox([m, k, s, ch], [seed & 0xFFFFFFFF, seed >> 32])
    u = [(2 * (x >> 9) + 1) / 16777216.0 for x in w]
    r0 = math.sqrt(-2.0 * math.log(u[0]))
    r1 = math.sqrt(-2.0 * math.log(u[2]))
    return [r0 * math.cos(2 * math.pi * u[1]), r0 * math.sin(2 * math.pi * u[1]),
            r1 * math.cos(2 * math.pi * u[3]), r1 * math.sin(2 * math.pi * u[3])]


@pytest.mark.parametrize("objective", ["gate", "contour"])
def test_sampler_channel_map_and_clip_after_perturbation(objective):
    """Eq. (3) with per-rotor sigma: U^m_k[i] = clip(U*_k[i] + sigma_i z_i) with
    z_i the i-th normal of block (m, k, s, 0), each channel its own sigma
    (distinct values, so a swapped channel shows), clipped after the noise is
    added (U* sits at and next to the bounds, so clipping first would leave
    values outside them); contouring's speed V^m_k = clip(V*_k + sigma_v z,
    0, v_max) with z the first normal of block (m, k, s, 1)."""
    from paper_2509_14726_amd import synth
    N, seed, s = 9, 0x1234_5678_9ABC, 5
    sig = (0.3, 1.1, 2.7, 0.05)
    prm = synth.params(1, N, objective, seed, sigma=sig, sigma_v=3.0, v_max=4.0)
    w = synth.single_solve_workload(K=1, N=N, objective=objective, seed=seed)
    pb = O.Problem(synth.QUAD, prm, gates=w["gates"], path=w.get("path"), path_len=w.get("path_len", 0.0))
    lo, hi = synth.QUAD["t_min"], synth.QUAD["t_max"]
    Ustar = np.array([[hi, 6.9, 0.05, lo], [lo, 0.2, 3.0, hi], [3.5, hi, lo, 6.95]] * 3)[:N]
    Vstar = np.array([0.0, 4.0, 2.0, 3.9, 0.1, 4.0, 0.0, 1.0, 2.5])[:N]
    n_clipped = n_inside = 0
    for m in (0, 1, 17, 1023, 65535):
        U, V = pb.sample(Ustar.ravel(), Vstar, m, s)
        for k in range(N):
            z = _python_normals(seed, m, k, s, 0)
            for i in range(4):
                raw = Ustar[k, i] + sig[i] * z[i]
                want = min(max(raw, lo), hi)
                assert abs(U[k, i] - want) <= 1e-14 * max(1.0, abs(want)), (m, k, i)
                if raw < lo or raw > hi:
                    n_clipped += 1
                else:
                    n_inside += 1
            if objective == "contour":
                zv = _python_normals(seed, m, k, s, 1)[0]
                assert abs(V[k] - min(max(Vstar[k] + 3.0 * zv, 0.0), 4.0)) <= 1e-14, (m, k)
    assert n_clipped > 20 and n_inside > 20
