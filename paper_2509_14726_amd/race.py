"""Closed-loop race evaluation around the solver.

A controller flies against the binary64 host plant (RK4 of Eq. (2) with the
first input of every solve held over the control step), and the flown path is
scored with the race metrics of the paper's evaluation (Sec. V-A):

* the pass error at each waypoint: the smallest distance of the flown path
  (piecewise linear between the logged states) to the gate centre;
* the gate passes in track order and the lap time: a pass is the geometric
  crossing of the gate square of Sec. IV-A (front to behind, inside the
  closed square), and only the next gate of the lap counts;
* the position error against a time-indexed reference (tracking);
* the total-thrust profile: mean, extremes, and the share of control steps
  with a rotor at a thrust bound (the saturation the paper's Fig. 4 shows).

Everything here runs on the host; the solver is the only device code.
"""
from __future__ import annotations

import math

import numpy as np

from . import mppi as M


def fly(solve, quad: dict, x0, steps: int, dt: float, substeps: int = 4) -> dict:
    """Close the loop for `steps` control steps of length dt.

    solve(x, t) returns (u0, info) for state x at time t; the plant then
    advances x by dt with u0 held (RK4, `substeps` substeps).  A 17-component
    state is the rate input model's (the four thrusts last, u0 their rates).
    Returns the times t[0..S], states X[0..S], inputs U[0..S-1] and the solve
    reports, S = the number of completed steps (fewer than `steps` when a
    solve raised; `error` then holds its message)."""
    x = np.asarray(x0, dtype=np.float64).copy()
    plant = M.plant_step_rate if x.size == 17 else M.plant_step
    ts, xs, us, infos = [0.0], [x.copy()], [], []
    error = None
    for i in range(steps):
        t = i * dt
        try:
            u0, info = solve(x, t)
        except M.MppiError as e:
            error = str(e)
            break
        u0 = np.asarray(u0, dtype=np.float64)
        x = plant(quad, x, u0, dt, substeps)
        ts.append(t + dt)
        xs.append(x.copy())
        us.append(u0.copy())
        infos.append(info)
    return {"t": np.array(ts), "X": np.array(xs), "U": np.array(us).reshape(-1, 4), "info": infos,
            "error": error}


def point_segment_distance(a, b, c) -> float:
    """Distance from point c to the segment a-b (3-vectors)."""
    ab = b - a
    l2 = float(ab @ ab)
    s = 0.0 if l2 == 0.0 else min(1.0, max(0.0, float((c - a) @ ab) / l2))
    return float(np.linalg.norm(a + s * ab - c))


def waypoint_pass_errors(P, gates) -> np.ndarray:
    """Per gate: the smallest distance of the path P (S x 3, piecewise
    linear) to the gate centre."""
    P = np.asarray(P, dtype=np.float64)
    out = np.empty(len(gates))
    for g, row in enumerate(np.asarray(gates, dtype=np.float64)):
        c = row[:3]
        if len(P) == 1:
            out[g] = float(np.linalg.norm(P[0] - c))
        else:
            out[g] = min(point_segment_distance(P[i], P[i + 1], c) for i in range(len(P) - 1))
    return out


def gate_frame(row):
    """Centre, normal n (direction of travel) and lateral axis h of a gate
    row (cx, cy, cz, yaw)."""
    c = np.asarray(row[:3], dtype=np.float64)
    yaw = float(row[3])
    n = np.array([math.cos(yaw), math.sin(yaw), 0.0])
    h = np.array([-math.sin(yaw), math.cos(yaw), 0.0])
    return c, n, h


def crossing_time(pa, pb, ta: float, tb: float, row, size: float):
    """Time at which the segment pa->pb (flown from ta to tb) passes the gate
    square, or None: the signed plane distance goes from < 0 to >= 0 and the
    plane intersection lies inside the closed size x size square."""
    c, n, h = gate_frame(row)
    sa = float((pa - c) @ n)
    sb = float((pb - c) @ n)
    if not (sa < 0.0 <= sb):
        return None
    f = sa / (sa - sb)
    y = pa + f * (pb - pa)
    half = 0.5 * size
    if abs(float((y - c) @ h)) <= half and abs(float(y[2] - c[2])) <= half:
        return ta + f * (tb - ta)
    return None


def lap(P, t, gates, size: float, start_gate: int = 0) -> dict:
    """Gate passes in track order from `start_gate` along the path P at times
    t: only a pass of the next gate of the lap counts.  Returns the number of
    gates passed, their pass times, and the lap time (the pass time of the
    gate that completes one lap of all G gates) or None."""
    P = np.asarray(P, dtype=np.float64)
    G = len(gates)
    g, times = start_gate % G, []
    for i in range(len(P) - 1):
        tc = crossing_time(P[i], P[i + 1], float(t[i]), float(t[i + 1]), gates[g], size)
        if tc is not None:
            times.append(tc)
            g = (g + 1) % G
    lap_time = times[G - 1] if len(times) >= G else None
    return {"gates_passed": len(times), "pass_times": times, "lap_time": lap_time}


def tracking_rmse(P, t, xref, ref_dt: float) -> float:
    """Root-mean-square position error of P at times t against the reference
    row nearest in time (the last row held past the end)."""
    P = np.asarray(P, dtype=np.float64)
    idx = np.clip(np.floor(np.asarray(t) / ref_dt + 0.5).astype(int), 0, len(xref) - 1)
    e = P - np.asarray(xref, dtype=np.float64)[idx, :3]
    return float(np.sqrt(np.mean(np.sum(e * e, axis=1))))


def thrust_profile(U, t_min: float, t_max: float) -> dict:
    """Total thrust per control step (mean, min, max) and the share of steps
    with at least one rotor at a thrust bound."""
    U = np.asarray(U, dtype=np.float64).reshape(-1, 4)
    if U.shape[0] == 0:
        return {"total_mean_N": None, "total_min_N": None, "total_max_N": None, "saturated_share": None}
    tot = U.sum(axis=1)
    sat = np.any((U <= t_min) | (U >= t_max), axis=1)
    return {"total_mean_N": float(tot.mean()), "total_min_N": float(tot.min()),
            "total_max_N": float(tot.max()), "saturated_share": float(sat.mean())}


def score(flight: dict, w: dict, objective: str) -> dict:
    """All race metrics of one flight of workload w."""
    P = flight["X"][:, :3]
    t = flight["t"]
    gates = w["gates"]
    size = w["params"].get("gate_size", 1.5)
    pe = waypoint_pass_errors(P, gates)
    lp = lap(P, t, gates, size)
    out = {"pass_error_m_mean": float(pe.mean()), "pass_error_m_max": float(pe.max()),
           "gates_passed_in_order": lp["gates_passed"], "lap_time_s": lp["lap_time"],
           "flight_time_s": float(t[-1])}
    # the thrusts: the inputs, or the states of the rate model after each step
    T = flight["X"][1:, 13:17] if flight["X"].shape[1] == 17 else flight["U"]
    out.update(thrust_profile(T, w["quad"]["t_min"], w["quad"]["t_max"]))
    if objective == "track":
        out["tracking_rmse_m"] = tracking_rmse(P, t, w["xref"], w["ref_dt"])
    return out
