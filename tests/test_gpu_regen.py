"""The weighted average that draws the samples again (MPPI_FLAG_REGEN_AVERAGE)
against the one that reads the sample tensor, and against the oracle.

The regenerating average repeats the rollout's draw with the same counters and
the same operations, so a context with the flag must hand on the same
solution, report and warm state bit for bit as one without it, solve after
solve; where the rollout does not draw the samples itself (one- and two-wave
layouts) the flag has no effect.  Every case prints its name and sizes before
it touches the GPU.
"""
import sys

import numpy as np
import pytest

from paper_2509_14726_amd import mppi as M
from paper_2509_14726_amd import synth
from tests.parity import build_pair, solve_and_compare

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def _pair(w, precision):
    plain = M.Solver(w["quad"], w["params"], gates=w["gates"], path=w.get("path"),
                     path_len=w.get("path_len", 0.0), xref=w.get("xref"), ref_dt=w.get("ref_dt", 0.0),
                     precision=precision)
    prm = dict(w["params"], flags=M.FLAG_REGEN_AVERAGE)
    regen = M.Solver(w["quad"], prm, gates=w["gates"], path=w.get("path"), path_len=w.get("path_len", 0.0),
                     xref=w.get("xref"), ref_dt=w.get("ref_dt", 0.0), precision=precision)
    return plain, regen


def _warm_arrays(s):
    wd = s.get_warm()
    return (np.array(wd.U), np.array(wd.V), wd.g0, wd.solve_index, list(wd.allow), np.array(wd.x_prev))


@pytest.mark.parametrize("waves", ["3", "4"])
@pytest.mark.parametrize("objective", ["gate", "contour", "track"])
@pytest.mark.parametrize("precision", [M.FP32, M.FP64])
def test_regenerated_average_repeats_the_stored_one(precision, objective, waves, monkeypatch):
    # K + 1 = 2001 gives a ragged last tile; N = 37 a ragged last chunk
    say("regen bits", precision, objective, "waves", waves, "K=2000 N=37")
    monkeypatch.setenv("MPPI_ROLLOUT_WAVES", waves)
    w = synth.single_solve_workload(K=2000, N=37, objective=objective, seed=21, track_seed=3,
                                    **{"lambda": 5.0})
    plain, regen = _pair(w, precision)
    x = np.array(w["x0"], dtype=np.float64)
    for step in range(4):
        t = step * w["params"]["dt"]
        u0a, Ua, ia = plain.solve(x, t)
        u0b, Ub, ib = regen.solve(x, t)
        assert ia["regen_average"] == 0 and ib["regen_average"] == 1
        assert ib["rollout_waves"] == int(waves)
        np.testing.assert_array_equal(u0a, u0b)
        np.testing.assert_array_equal(Ua, Ub)
        for f in ("J_min", "S", "ess", "J_nom", "theta0", "g0", "i0", "shift", "solve_index", "status"):
            assert ia[f] == ib[f], f
        Ja, _ = plain.read_samples()
        Jb, _ = regen.read_samples()
        np.testing.assert_array_equal(Ja, Jb)
        wa, wb = _warm_arrays(plain), _warm_arrays(regen)
        for a, b in zip(wa, wb):
            np.testing.assert_array_equal(a, b)
        x = M.plant_step(w["quad"], x, u0a, w["params"]["dt"], 2)
    plain.close()
    regen.close()


@pytest.mark.parametrize("objective", ["gate", "contour", "track"])
@pytest.mark.parametrize("precision", [M.FP64, M.FP32])
def test_regenerated_average_against_the_oracle(precision, objective):
    """Three warm solves of a context with the flag against the oracle, with
    the tolerances of the other parity tests (the automatic layout of
    K = 4096 is the four-wave pipeline)."""
    say("regen vs oracle", precision, objective, "K=4096 N=60")
    w = synth.single_solve_workload(K=4096, N=60, objective=objective, seed=22, track_seed=4,
                                    **{"lambda": 20.0})
    w["params"] = dict(w["params"], flags=M.FLAG_REGEN_AVERAGE)
    dev, orc = build_pair(w, precision)
    x = np.array(w["x0"], dtype=np.float64)
    for step in range(3):
        st = solve_and_compare(dev, orc, x, step * w["params"]["dt"], precision)
        say("  step", step, "err_J", st["err_J"], "err_U", st["err_U"], "ambiguous", st["n_amb"])
        st_, info = dev.read_info()
        assert info["regen_average"] == 1
        u0 = dev.get_warm().U[:4]
        x = M.plant_step(w["quad"], x, np.array(u0), w["params"]["dt"], 2)
    dev.close()


def test_regeneration_needs_a_drawing_rollout(monkeypatch):
    """In the one-wave layout the flag is not in effect: the sample tensor is
    written and can be read; with it in effect the samples cannot be read."""
    say("regen flag effect", "K=1000 N=20")
    w = synth.single_solve_workload(K=1000, N=20, objective="gate", seed=23, track_seed=1)
    monkeypatch.setenv("MPPI_ROLLOUT_WAVES", "1")
    plain, regen = _pair(w, M.FP32)
    u0a, _, ia = plain.solve(w["x0"], 0.0)
    u0b, _, ib = regen.solve(w["x0"], 0.0)
    assert ib["regen_average"] == 0 and ib["rollout_waves"] == 1
    np.testing.assert_array_equal(u0a, u0b)
    _, Ub = regen.read_samples(want_U=True)
    assert Ub.shape[0] == 20
    plain.close()
    regen.close()
    monkeypatch.setenv("MPPI_ROLLOUT_WAVES", "4")
    plain, regen = _pair(w, M.FP32)
    plain.close()
    regen.solve(w["x0"], 0.0)
    regen.read_samples()
    with pytest.raises(M.MppiError, match="REGEN"):
        regen.read_samples(want_U=True)
    regen.close()


def test_regenerated_average_at_the_benchmark_point():
    """The benchmark workload (K = 8192, N = 100, gate, binary32, automatic
    layout: four waves with 4-step chunks): three warm solves with and without
    the flag agree bit for bit."""
    say("regen bits at the benchmark point", "K=8192 N=100")
    w = synth.single_solve_workload(K=8192, N=100, seed=1)
    plain, regen = _pair(w, M.FP32)
    x = np.array(w["x0"], dtype=np.float64)
    for step in range(3):
        t = step * w["params"]["dt"]
        u0a, Ua, ia = plain.solve(x, t)
        u0b, Ub, ib = regen.solve(x, t)
        assert ib["regen_average"] == 1 and ib["rollout_waves"] == 4
        np.testing.assert_array_equal(u0a, u0b)
        np.testing.assert_array_equal(Ua, Ub)
        assert ia["S"] == ib["S"] and ia["J_min"] == ib["J_min"] and ia["ess"] == ib["ess"]
        x = M.plant_step(w["quad"], x, u0a, w["params"]["dt"], 2)
    plain.close()
    regen.close()


@pytest.mark.parametrize("K,N", [(1, 1), (63, 256), (64, 5), (1, 256)])
@pytest.mark.parametrize("precision", [M.FP32, M.FP64])
def test_regenerated_average_at_extreme_shapes(precision, K, N):
    """A single sample, a full last tile (K + 1 = 64), a nominal alone in a
    new tile (K + 1 = 65) and the longest horizon: the flag repeats the
    stored-tensor solve bit for bit over two warm solves."""
    say("regen extreme shape", precision, "K", K, "N", N)
    w = synth.single_solve_workload(K=K, N=N, objective="gate", seed=31, track_seed=2)
    plain, regen = _pair(w, precision)
    x = np.array(w["x0"], dtype=np.float64)
    for step in range(2):
        t = step * w["params"]["dt"]
        u0a, Ua, ia = plain.solve(x, t)
        u0b, Ub, ib = regen.solve(x, t)
        assert ib["regen_average"] == 1
        np.testing.assert_array_equal(u0a, u0b)
        np.testing.assert_array_equal(Ua, Ub)
        assert ia["S"] == ib["S"] and ia["J_min"] == ib["J_min"]
        x = M.plant_step(w["quad"], x, u0a, w["params"]["dt"], 2)
    plain.close()
    regen.close()


@pytest.mark.parametrize("objective", ["gate", "contour", "track"])
def test_regenerated_average_in_the_drawing_one_wave_layout(objective, monkeypatch):
    """The one-wave rollout that draws its own samples (binary32) writes no
    sample tensor under the flag; the average draws the samples again with
    the rollout's counters and arithmetic: the same bits, solve after solve
    (K + 1 = 3001: a ragged last tile)."""
    say("regen bits, drawing one-wave layout", objective, "K=3000 N=41")
    monkeypatch.setenv("MPPI_ROLLOUT_WAVES", "1")
    monkeypatch.setenv("MPPI_ROLLOUT_DRAW", "1")
    w = synth.single_solve_workload(K=3000, N=41, objective=objective, seed=24, track_seed=5,
                                    **{"lambda": 5.0})
    plain, regen = _pair(w, M.FP32)
    x = np.array(w["x0"], dtype=np.float64)
    for step in range(4):
        t = step * w["params"]["dt"]
        u0a, Ua, ia = plain.solve(x, t)
        u0b, Ub, ib = regen.solve(x, t)
        assert ia["regen_average"] == 0 and ib["regen_average"] == 1
        assert ib["rollout_waves"] == 1 and ib["rollout_draw"] == 1 and ia["rollout_draw"] == 1
        np.testing.assert_array_equal(u0a, u0b)
        np.testing.assert_array_equal(Ua, Ub)
        for f in ("J_min", "S", "ess", "J_nom", "theta0", "g0", "solve_index"):
            assert ia[f] == ib[f], f
        Ja, _ = plain.read_samples()
        Jb, _ = regen.read_samples()
        np.testing.assert_array_equal(Ja, Jb)
        for a, b in zip(_warm_arrays(plain), _warm_arrays(regen)):
            np.testing.assert_array_equal(a, b)
        x = M.plant_step(w["quad"], x, u0a, w["params"]["dt"], 2)
    with pytest.raises(M.MppiError, match="REGEN"):
        regen.read_samples(want_U=True)
    plain.close()
    regen.close()


def test_context_autotuner_chooses_restores_and_caches(tmp_path):
    """mppi_autotune at the benchmark point (four-wave layout): both averages
    timed, the faster kept, the warm state as before the timed solves, the
    choice written to the cache and taken from it the next time; the tuned
    context then solves as an untuned twin does, bit for bit."""
    import json

    import torch
    say("context autotuner", "K=8192 N=100")
    w = synth.single_solve_workload(K=8192, N=100, seed=1)
    a, b = _pair(w, M.FP32)
    b.close()
    twin = M.Solver(w["quad"], w["params"], gates=w["gates"], precision=M.FP32)
    x = np.array(w["x0"], dtype=np.float64)
    a.solve(x, 0.0)
    twin.solve(x, 0.0)
    before = _warm_arrays(a)
    req = torch.zeros(M.REQ_DOUBLES, dtype=torch.float64, device="cuda")
    req[:13] = torch.from_numpy(x)
    req[13] = 0.02
    cache = str(tmp_path / "tune.json")
    r = a.autotune(req.data_ptr(), reps=2, cache_path=cache)
    say("  ", r)
    assert r["from_cache"] == 0 and r["ms_stored"] > 0 and r["ms_regen"] > 0
    assert r["regen_average"] == (1 if r["ms_regen"] < r["ms_stored"] else 0)
    for p, q in zip(before, _warm_arrays(a)):
        np.testing.assert_array_equal(p, q)
    data = json.load(open(cache))
    (key, ent), = data.items()
    assert key.startswith("ctx|gfx") and "|gate|fp32|K13|N6|w4" in key and ent["regen_average"] == r["regen_average"]
    r2 = a.autotune(req.data_ptr(), reps=2, cache_path=cache)
    assert r2["from_cache"] == 1 and r2["regen_average"] == r["regen_average"]
    u0a, Ua, ia = a.solve(x, 0.02)
    u0t, Ut, it = twin.solve(x, 0.02)
    assert ia["regen_average"] == r["regen_average"]
    np.testing.assert_array_equal(u0a, u0t)
    np.testing.assert_array_equal(Ua, Ut)
    # where the rollout reads a sample tensor there is one choice, not timed
    ws = synth.single_solve_workload(K=1000, N=20, seed=2)
    import os
    os.environ["MPPI_ROLLOUT_WAVES"] = "2"
    try:
        c = M.Solver(ws["quad"], ws["params"], gates=ws["gates"], precision=M.FP32)
    finally:
        del os.environ["MPPI_ROLLOUT_WAVES"]
    rc = c.autotune(req.data_ptr(), reps=2, cache_path=cache)
    assert rc == {"regen_average": 0, "from_cache": 0, "ms_stored": 0.0, "ms_regen": 0.0}
    for s in (a, twin, c):
        s.close()
