"""The race harness around the device solver, against the FP64 oracle.

Every step of the flight the harness scores is an MPPI step that matches the
oracle from the same warm state (the device's, imported).  For the gate
objective the closed loop is also well conditioned (a 1e-13 offset of the
start state stays at 1e-13 over 40 steps of the oracle's own loop), so two
independent loops, the device's and the oracle's, fly the same path and the
race metrics agree.  The contouring and tracking loops amplify such offsets
by 1e4-1e5 over 40 steps (near-tied samples under the softmax), so there
only the step-by-step check applies."""
import sys

import numpy as np
import pytest

from paper_2509_14726_amd import mppi as M
from paper_2509_14726_amd import race
from paper_2509_14726_amd import synth
from tests.parity import build_pair, solve_and_compare

pytestmark = pytest.mark.gpu


def _workload(objective):
    return synth.single_solve_workload(K=512, N=30, objective=objective, seed=6, track_seed=1,
                                       sigma=(0.15,) * 4, **{"lambda": 10.0})


@pytest.mark.parametrize("precision", [M.FP64, M.FP32])
@pytest.mark.parametrize("objective", ["gate", "contour", "track"])
def test_flight_steps_match_the_oracle(objective, precision):
    print("[gpu-case] race flight step by step", objective, precision, "K=512 N=30 25 steps", flush=True)
    sys.stdout.flush()
    w = _workload(objective)
    dev, orc = build_pair(w, precision)

    def solve(x, t):
        st = solve_and_compare(dev, orc, x, t, precision, sigma=0.15)
        return st["U"][0], st["info"]

    fl = race.fly(solve, w["quad"], w["x0"], 25, w["params"]["dt"])
    assert fl["error"] is None
    sc = race.score(fl, w, objective)
    assert sc["flight_time_s"] == pytest.approx(25 * w["params"]["dt"])
    assert np.isfinite(sc["pass_error_m_mean"]) and sc["total_min_N"] >= 0.0
    dev.close()


def test_independent_gate_flights_agree():
    print("[gpu-case] race harness, independent loops, gate, fp64, 40 steps", flush=True)
    w = _workload("gate")
    dev, orc = build_pair(w, M.FP64)
    ow = orc.warm(0)

    def dev_solve(x, t):
        u0, _, info = dev.solve(x, t)
        return u0, info

    def orc_solve(x, t):
        r = orc.solve(ow, x, t)
        assert r["status"] == 0
        return r["U"][0], r

    dt = w["params"]["dt"]
    fd = race.fly(dev_solve, w["quad"], w["x0"], 40, dt)
    fo = race.fly(orc_solve, w["quad"], w["x0"], 40, dt)
    assert fd["error"] is None and fo["error"] is None
    err = float(np.abs(fd["X"] - fo["X"]).max())
    print("[gpu-case]   max state difference", err, flush=True)
    assert err <= 1e-9
    sd, so = race.score(fd, w, "gate"), race.score(fo, w, "gate")
    for k in sd:
        if sd[k] is None or isinstance(sd[k], int):
            assert sd[k] == so[k], k
        else:
            assert abs(sd[k] - so[k]) <= 1e-9 * max(1.0, abs(so[k])), (k, sd[k], so[k])
    dev.close()


@pytest.mark.parametrize("objective", ["gate", "contour", "track"])
def test_race_configuration_steps_match_the_oracle(objective):
    """The race the benchmark flies (thrust-rate input, 8192 samples, 20
    steps of 0.03 s, its per-objective noise and temperature, the circuit
    track), binary32, step by step against the oracle for 20 control steps."""
    import bench
    st = bench.RACE_SETTINGS[objective]
    print("[gpu-case] race configuration step by step", objective, st, "K=8192 N=20 20 steps", flush=True)
    hover = synth.QUAD["mass"] * synth.QUAD["gravity"] / 4.0
    w = synth.race_workload(K=8192, N=20, objective=objective, seed=1, track_seed=1, dt=0.03, steps=40,
                            sigma=(st["sigma"],) * 4, sigma_v=5.0, input_model=M.INPUT_RATE,
                            rate_lim=(-10.0, 10.0), dv_lim=(-20.0, 20.0), **{"lambda": st["lam"]})
    dev, orc = build_pair(w, M.FP32)

    def solve(x, t):
        r = solve_and_compare(dev, orc, x, t, M.FP32, sigma=st["sigma"])
        return r["U"][0], r["info"]

    x0 = np.concatenate([w["x0"], np.full(4, hover)])
    fl = race.fly(solve, w["quad"], x0, 20, 0.03)
    assert fl["error"] is None and fl["X"].shape == (21, 17)
    dev.close()
