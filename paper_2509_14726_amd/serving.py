"""Serving workload driver: many simulated drones issue MPPI solve requests
as Poisson arrivals; the continuous-batching server (mppi_server_*) admits and
batches them as launch slots and device memory free up.

Each drone has its own seeded track, K in {2048, 8192}, N in {50, 100} and a
gate-progress or contouring objective (50/50), fixed for the drone (its warm
start needs a stable shape).  Gate drones sample the rotor thrusts (0.15 N
of noise per rotor, lambda = 10).  Contouring drones do the same by default;
with contour_input="rate" they fly the paper's input model (Sec. III-A):
thrust rates with 10 N/s of noise, bounds +-10 N/s, the progress
acceleration with 5 m/s^2 of noise, lambda = 10, the thrusts as four more
states.  Over these 1-2 s horizons contouring drones with thrust as the input
fall away from the path and those with thrust rates follow it; rate drones
run one-wave rollouts, in launches of their own, which costs latency.  Between two of its requests a drone's FP64 host plant advances
with the last control it received (RK4, substeps of at most 5 ms).  A drone whose state leaves a sane envelope (non-finite, more than
1 km from the origin, or spinning faster than 1000 rad/s) is counted as a
crash and respawned at its start (its solver keeps the warm state and
re-converges from it).  Arrivals are paced
in wall clock; latency = time the result is retired - arrival time, where
the retire time is the clock read just before the server call that found the
solve finished.
"""
from __future__ import annotations

import time

import numpy as np

from . import mppi as M
from . import synth


def drone_workloads(n_drones: int, seed: int = 4, contour_input: str = "thrust"):
    out = []
    for d in range(n_drones):
        rng = np.random.default_rng(4000 + d)
        K = int(rng.choice([2048, 8192]))
        N = int(rng.choice([50, 100]))
        obj = "gate" if rng.uniform() < 0.5 else "contour"
        rate = obj == "contour" and contour_input == "rate"
        if not rate:
            # thrust noise of 0.15 N with lambda = 10: with 1 N per rotor and
            # step the samples spin this airframe and the drones tumble
            over = dict(sigma=(0.15,) * 4)
        else:
            over = dict(sigma=(10.0,) * 4, sigma_v=5.0, input_model=M.INPUT_RATE,
                        rate_lim=(-10.0, 10.0), dv_lim=(-20.0, 20.0))
        w = synth.single_solve_workload(K=K, N=N, objective=obj, seed=4000 + d, track_seed=4000 + d,
                                        **over, **{"lambda": 10.0})
        w["params"] = dict(w["params"], flags=M.FLAG_EXTERNAL_WORKSPACE)
        if rate:
            w["x0"] = np.concatenate([w["x0"], np.full(4, synth.hover_thrust(w["quad"]))])
        out.append(w)
    return out


def arrivals(n_drones: int, seconds: float, rate_hz: float, seed: int = 4):
    rng = np.random.default_rng(seed)
    times, ids = [], []
    for d in range(n_drones):
        n = int(seconds * rate_hz * 1.5) + 16
        t = np.cumsum(rng.exponential(1.0 / rate_hz, size=n))
        t = t[t < seconds]
        times.append(t)
        ids.append(np.full(t.size, d, dtype=np.int32))
    t = np.concatenate(times)
    i = np.concatenate(ids)
    o = np.argsort(t, kind="stable")
    return t[o], i[o]


def _plant(quad, x, u, elapsed):
    n = max(2, int(np.ceil(elapsed / 0.005)))
    step = M.plant_step_rate if x.size == 17 else M.plant_step
    return step(quad, x, u, elapsed, n)


def _rest_input(w):
    """The input a drone holds before its first result: hover thrust, or no
    thrust change for the rate model."""
    return np.zeros(4) if w["x0"].size == 17 else np.full(4, synth.hover_thrust(w["quad"]))


def _sane(x) -> bool:
    return bool(np.all(np.isfinite(x)) and np.linalg.norm(x[0:3]) < 1e3 and np.linalg.norm(x[10:13]) < 1e3)


def simulate(n_drones: int = 512, seconds: float = 60.0, rate_hz: float = 50.0,
             budget_bytes: float = 32 * 2 ** 30, n_slots: int = 4, max_batch: int = 0,
             precision: int = M.FP32, seed: int = 4, contour_input: str = "thrust", log=None):
    ws = drone_workloads(n_drones, seed, contour_input)
    solvers = [M.Solver(w["quad"], w["params"], gates=w["gates"], path=w.get("path"),
                        path_len=w.get("path_len", 0.0), precision=precision) for w in ws]
    server = M.Server(solvers, budget_bytes=budget_bytes, n_slots=n_slots, max_batch=max_batch)
    t_arr, d_arr = arrivals(n_drones, seconds, rate_hz, seed)
    x = [w["x0"].copy() for w in ws]
    u = [_rest_input(w) for w in ws]
    t_state = np.zeros(n_drones)
    crashes = 0
    lat = []
    steps = 0.0
    idx, n_total = 0, t_arr.size
    t0 = time.perf_counter()
    next_log = 5.0
    while True:
        now = time.perf_counter() - t0
        while idx < n_total and t_arr[idx] <= now:
            d = int(d_arr[idx])
            ta = float(t_arr[idx])
            if ta > t_state[d]:
                x[d] = _plant(ws[d]["quad"], x[d], u[d], ta - t_state[d])
                t_state[d] = ta
            if not _sane(x[d]):
                crashes += 1
                x[d] = ws[d]["x0"].copy()
                u[d] = _rest_input(ws[d])
            server.submit(d, x[d], ta, ta)
            idx += 1
        # the server stamps the solves it retires with this clock: read it
        # after the plant steps and submissions above, not before them
        now = time.perf_counter() - t0
        server.progress(now)
        for r in server.poll():
            lat.append(r["t_done"] - r["t_arrival"])
            if r["status"] == M.OK:
                u[r["drone"]] = np.array(r["u0"])
        if log and now >= next_log:
            st = server.stats()
            log(f"t={now:.1f}s submitted={st['submitted']} completed={st['completed']} "
                f"queued={st['queued']} in_flight={st['in_flight']} launches={st['launches']}")
            next_log += 5.0
        if idx >= n_total:
            st = server.stats()
            if st["queued"] == 0 and st["in_flight"] == 0:
                break
    wall = time.perf_counter() - t0
    st = server.stats()
    server.close()
    for s in solvers:
        s.close()
    lat = np.array(lat)
    return {
        "drones": n_drones, "seconds": seconds, "rate_hz": rate_hz, "requests": int(n_total),
        "completed": int(st["completed"]), "launches": int(st["launches"]),
        "wall_s": wall, "rollout_steps_per_s": st["rollout_steps"] / wall,
        "solves_per_s": st["completed"] / wall,
        "p50_ms": float(np.percentile(lat, 50) * 1e3) if lat.size else None,
        "p99_ms": float(np.percentile(lat, 99) * 1e3) if lat.size else None,
        "mean_batch": st["completed"] / max(st["launches"], 1),
        "peak_bytes_in_flight": st["peak_bytes_in_flight"], "budget_bytes": budget_bytes,
        "n_slots": n_slots, "max_batch": max_batch, "crashes": crashes, "contour_input": contour_input,
    }
