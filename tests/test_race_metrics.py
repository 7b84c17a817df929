"""CPU pins of the race metrics (paper_2509_14726_amd.race) on paths whose
answers are known in closed form: straight flights past and through gates,
a constant tracking offset, a hand-made thrust log."""
import math

import numpy as np

from paper_2509_14726_amd import race


def _line(x0, x1, n, y=0.0, z=1.0):
    t = np.linspace(0.0, 1.0, n)
    P = np.stack([x0 + (x1 - x0) * t, np.full(n, y), np.full(n, z)], axis=1)
    return P, t


def test_pass_error_is_the_perpendicular_distance_of_a_straight_pass():
    # the path runs along x at y = 0.3, z = 1.4; gate centre (5, 0, 1): the
    # nearest point is (5, 0.3, 1.4), at distance 0.5 -- between samples
    P, _ = _line(0.1, 9.7, 7, y=0.3, z=1.4)
    gates = np.array([[5.0, 0.0, 1.0, 0.0], [20.0, 0.0, 1.0, 0.0]])
    pe = race.waypoint_pass_errors(P, gates)
    assert abs(pe[0] - 0.5) < 1e-12
    # beyond the end of the path: distance to the last point (9.7, 0.3, 1.4)
    assert abs(pe[1] - math.sqrt(10.3 ** 2 + 0.3 ** 2 + 0.4 ** 2)) < 1e-12


def test_crossing_time_is_interpolated_on_the_segment():
    # x(t) = 2 t + 0.25 passes x = 5 at t = 2.375
    t = np.arange(0.0, 4.01, 0.5)
    P = np.stack([2.0 * t + 0.25, np.zeros_like(t), np.ones_like(t)], axis=1)
    gates = np.array([[5.0, 0.0, 1.0, 0.0]])
    res = race.lap(P, t, gates, 1.5)
    assert res["gates_passed"] == 1 and abs(res["pass_times"][0] - 2.375) < 1e-12
    assert abs(res["lap_time"] - 2.375) < 1e-12


def test_passes_outside_the_square_or_backwards_do_not_count():
    t = np.linspace(0.0, 1.0, 11)
    gates = np.array([[5.0, 0.0, 1.0, 0.0]])
    # lateral offset 0.76 > 0.75: outside the 1.5 m square
    P = np.stack([10.0 * t, np.full_like(t, 0.76), np.ones_like(t)], axis=1)
    assert race.lap(P, t, gates, 1.5)["gates_passed"] == 0
    # on the edge (0.75): inside the closed square
    P[:, 1] = 0.75
    assert race.lap(P, t, gates, 1.5)["gates_passed"] == 1
    # flown against the gate normal (yaw 0 points along +x): no pass
    P = np.stack([10.0 - 10.0 * t, np.zeros_like(t), np.ones_like(t)], axis=1)
    assert race.lap(P, t, gates, 1.5)["gates_passed"] == 0
    # a gate turned by pi faces -x: the same backward flight passes it
    gates_back = np.array([[5.0, 0.0, 1.0, math.pi]])
    assert race.lap(P, t, gates_back, 1.5)["gates_passed"] == 1


def test_lap_counts_only_the_next_gate_in_order():
    # gates along x at 2, 4, 6 in the order 0: x=4, 1: x=2, 2: x=6; a flight
    # along +x passes x=2 (gate 1, not next), x=4 (gate 0), x=6 (gate 2, but
    # gate 1 is next): one pass only
    t = np.linspace(0.0, 8.0, 81)
    P = np.stack([t, np.zeros_like(t), np.ones_like(t)], axis=1)
    gates = np.array([[4.0, 0.0, 1.0, 0.0], [2.0, 0.0, 1.0, 0.0], [6.0, 0.0, 1.0, 0.0]])
    res = race.lap(P, t, gates, 1.5)
    assert res["gates_passed"] == 1 and abs(res["pass_times"][0] - 4.0) < 1e-12
    assert res["lap_time"] is None
    # in track order 2, 4, 6 the lap completes at the third pass, t = 6
    ordered = gates[[1, 0, 2]]
    res = race.lap(P, t, ordered, 1.5)
    assert res["gates_passed"] == 3 and abs(res["lap_time"] - 6.0) < 1e-12


def test_tracking_rmse_of_a_constant_offset():
    ref_dt = 0.02
    n = 50
    xref = np.zeros((n + 10, 13))
    xref[:, 0] = np.arange(n + 10) * 0.1
    t = np.arange(n) * ref_dt
    P = xref[:n, :3] + np.array([0.1, 0.2, 0.2])
    assert abs(race.tracking_rmse(P, t, xref, ref_dt) - 0.3) < 1e-12
    # past the end of the reference the last row is held
    t_late = np.full(3, 100.0)
    P_late = np.tile(xref[-1, :3], (3, 1)) + np.array([0.0, 0.0, 2.0])
    assert abs(race.tracking_rmse(P_late, t_late, xref, ref_dt) - 2.0) < 1e-12


def test_thrust_profile():
    U = np.array([[1.0, 2.0, 3.0, 4.0], [0.0, 2.0, 2.0, 2.0], [7.0, 1.0, 1.0, 1.0], [2.0, 2.0, 2.0, 2.0]])
    p = race.thrust_profile(U, 0.0, 7.0)
    assert p["total_mean_N"] == (10.0 + 6.0 + 10.0 + 8.0) / 4
    assert p["total_min_N"] == 6.0 and p["total_max_N"] == 10.0
    assert p["saturated_share"] == 0.5
    assert race.thrust_profile(np.zeros((0, 4)), 0.0, 7.0)["total_mean_N"] is None


def test_fly_closes_the_loop_with_the_host_plant():
    """A controller that always commands hover thrust keeps a level body at
    rest: the logged states stay at the start, the times advance by dt, and
    a controller error ends the flight with its message."""
    from paper_2509_14726_amd import mppi as M
    from paper_2509_14726_amd import synth
    q = synth.QUAD
    x0 = np.zeros(13)
    x0[2] = 3.0
    x0[6] = 1.0
    hover = np.full(4, synth.hover_thrust(q))
    fl = race.fly(lambda x, t: (hover, {"t": t}), q, x0, 10, 0.02)
    assert fl["error"] is None and fl["X"].shape == (11, 13) and fl["U"].shape == (10, 4)
    np.testing.assert_allclose(fl["t"], np.arange(11) * 0.02, rtol=0, atol=1e-15)
    np.testing.assert_allclose(fl["X"], np.tile(x0, (11, 1)), rtol=0, atol=1e-12)

    def failing(x, t):
        if t > 0.05:
            raise M.MppiError(M.E_NONFINITE, "all costs non-finite")
        return hover, {}

    fl = race.fly(failing, q, x0, 10, 0.02)
    assert fl["X"].shape == (4, 13) and "non-finite" in fl["error"]


def test_loop_track_gates_face_along_the_path():
    """The race circuit: flying the path table in the direction of increasing
    arc length crosses every gate front to back, inside its square, in track
    order (the race metrics count all of them on one lap of the table)."""
    from paper_2509_14726_amd import synth
    for seed in (1, 2, 3):
        gates = synth.loop_track(seed)
        path, L = synth.path_table(gates)
        # start just before gate 0's plane: rotate the table to begin there
        i0 = int(np.argmin(np.linalg.norm(path[:, :3] - gates[0, :3], axis=1)))
        P = np.roll(path[:, :3], 5 - i0, axis=0)
        lp = race.lap(P, np.arange(len(P)) * 0.01, gates, 1.5)
        assert lp["gates_passed"] == len(gates), seed
        assert np.all(race.waypoint_pass_errors(P, gates) < 0.05)
    w = synth.race_workload(objective="track", steps=100)
    assert w["xref"].shape == (100 + 20 + 1, 13) and w["params"]["N"] == 20 and w["params"]["dt"] == 0.03
    n = np.array([np.cos(gates[0, 3]), np.sin(gates[0, 3]), 0.0])
    x0 = synth.start_state(gates)
    assert abs(float((gates[0, :3] - x0[:3]) @ n) - 2.0) < 1e-12


def test_serving_drones_take_the_rate_input_only_for_contouring_when_asked():
    """The serving workload's drones: thrust input for every drone by
    default; with contour_input="rate" the contouring drones take the rate
    input model (17-state start, thrusts at hover) and the gate drones keep
    thrust."""
    from paper_2509_14726_amd import mppi as M
    from paper_2509_14726_amd import serving, synth
    ws = serving.drone_workloads(24)
    assert all(w["x0"].size == 13 and w["params"].get("input_model", M.INPUT_THRUST) == M.INPUT_THRUST
               for w in ws)
    wr = serving.drone_workloads(24, contour_input="rate")
    objs = {w["params"]["objective"] for w in wr}
    assert objs == {synth.OBJ_GATE, synth.OBJ_CONTOUR}
    for w0, w in zip(ws, wr):
        assert w["params"]["K"] == w0["params"]["K"] and w["params"]["N"] == w0["params"]["N"]
        if w["params"]["objective"] == synth.OBJ_CONTOUR:
            assert w["params"]["input_model"] == M.INPUT_RATE and w["x0"].size == 17
            assert np.allclose(w["x0"][13:], synth.hover_thrust(w["quad"]))
            assert np.array_equal(w["x0"][:13], w0["x0"])
        else:
            assert w["x0"].size == 13 and w["params"].get("input_model", M.INPUT_THRUST) == M.INPUT_THRUST
