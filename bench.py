#!/usr/bin/env python3
"""Throughput of the MPPI sampling step on one MI355X.

One step = one MPPI solve (noise, clipped samples, RK4 rollouts with the
gate-progress cost, softmax weights, weighted update, warm-start hand-over)
at K = 8192 samples, N = 100 steps, dt = 0.02 s on a seeded 7-gate track,
driven from device memory (mppi_solve_device): the state and time of every
step are already resident in HBM when the timed region starts.

Prints one JSON line: rollout-steps/s (K*N per solve time), the roofline of
the dominant kernel (the rollout) from HIP events recorded on the solver's
stream, and the FP64 CPU oracle timed on the host cores on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work of one rollout step of the gate objective, counted by the
# oracle's op-counting build (the oracle's own source with binary64 counted):
# the mean over the first 256 samples of the cold benchmark solve of its
# additions, multiplications, divisions and square roots per sample and step,
# 24.0 for the sampling of Eq. (3) and 544.1 for RK4 of Eq. (2) with the gate
# cost of Eq. (6)-(7), the switch test and the rate penalty.  A CPU test
# recounts it.
FLOPS_PER_ROLLOUT_STEP = 568.1
# Peak vector throughput of MI355X (256 CUs, 2.4 GHz): FP32 with packed FMA,
# FP64
PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBPS = 8000.0

# HBM bytes per launch measured with rocprofv3 --pmc FETCH_SIZE and, in a run
# of its own, WRITE_SIZE (KiB per dispatch, mean of 12 dispatches of the
# benchmark workload), scaled by what the same counters read for a plain
# 256 MiB device copy (FETCH_SIZE 131085.2 KiB -> x 2.0, WRITE_SIZE
# 262144.0 KiB -> x 1.0); see profiles/k_rollout4_gate_k8192_n100_traffic.md.
# They hold only for the workload (K = 8192, N = 100, gate, binary32, the
# four-wave layout with 4-step chunks; the average reading the sample tensor
# or drawing the samples again) and the device sources they were taken on
# (sha256 of kernels.hip, device.hpp, rollout.hpp, noise.hpp in that order);
# otherwise the traffic is reported as null.
TRAFFIC_SOURCES = "fb4b8f90baacc8aedb9d869f966968959d580ebad4ea0565a29b5417ce29b7b9"
FETCH_SCALE, WRITE_SCALE = 262144.0 / 131085.2, 262144.0 / 262144.0
TRAFFIC_KIB = {("k_rollout4", 0): (185.7, 12836.4), ("k_final", 0): (6575.5, 6.6),
               ("k_rollout4", 1): (185.6, 38.0), ("k_final", 1): (211.5, 6.6)}
TRAFFIC_WORKLOADS = {(8192, 100, "fp32", 0), (8192, 100, "fp32", 1)}
ROLLOUT_KERNELS = {1: "k_rollout", 2: "k_rollout_split", 3: "k_rollout3", 4: "k_rollout4"}


def rollout_kernel(waves: int) -> str:
    """The rollout kernel of a layout (the solve report names the layout)."""
    return ROLLOUT_KERNELS[waves]


def device_sources_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "device.hpp", "rollout.hpp", "noise.hpp"):
        with open(os.path.join(ROOT, "paper_2509_14726_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_bytes(kernel: str, workload=(8192, 100, "fp32", 0)):
    """Measured HBM bytes per launch of a kernel (fetch + write), or None when
    the workload (K, N, precision, regenerating average) or the device
    sources differ from the ones the counters were taken on."""
    if (workload not in TRAFFIC_WORKLOADS or device_sources_hash() != TRAFFIC_SOURCES
            or (kernel, workload[3]) not in TRAFFIC_KIB):
        return None
    f, w = TRAFFIC_KIB[(kernel, workload[3])]
    return (f * FETCH_SCALE + w * WRITE_SCALE) * 1024.0


def _cpu_info():
    """Host CPU model, logical CPUs of the machine and of this process."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return model, os.cpu_count() or 1, usable


def _oracle_problem(w, cores, eps_dec=0.0):
    from oracle import oracle as O
    prm = dict(w["params"], eps_dec=eps_dec, n_threads=cores)
    return O.Problem(w["quad"], prm, gates=w["gates"], path=w.get("path"), path_len=w.get("path_len", 0.0),
                     xref=w.get("xref"), ref_dt=w.get("ref_dt", 0.0))


def _time_oracle(w, cores, seconds):
    from oracle import oracle as O
    pb = _oracle_problem(w, cores)
    warm = pb.warm()
    K, N = pb.cfg.K, pb.cfg.N
    n, t0 = 0, time.perf_counter()
    while True:
        r = pb.solve(warm, w["x0"], n * pb.cfg.dt)
        assert r["status"] == O.OK
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds or n >= 1000:
            break
    return n * K * N / el, n, el


def oracle_errors(w, rec, cores):
    """Error of one device solve against the FP64 oracle solving from the
    device's exported warm state: the largest relative cost error (samples
    whose decision lies within 1e-4 of a threshold excluded), the update
    stage (the oracle's Eq. (4)-(5) fed with the device's costs) and the
    controls end to end (the oracle's own costs; the device's only for those
    ambiguous samples), relative to max(|U|, sigma); plus J_min and ESS."""
    import numpy as np
    from oracle import oracle as O
    pb = _oracle_problem(w, cores, eps_dec=1e-4)

    def warm():
        wd = rec["warm"]
        o = pb.warm(wd.g0)
        o.warm = wd.warm
        o.s = wd.solve_index
        for j in range(O.MASK_WORDS):
            o.allow[j] = wd.allow[j]
        o.t_prev = wd.t_prev
        o.x_prev[:] = list(wd.x_prev)
        o.theta0 = wd.theta0
        o.U[:] = list(wd.U)
        o.V[:] = list(wd.V)
        return o

    t0 = time.perf_counter()
    r = pb.solve(warm(), rec["x0"], rec["t"])
    amb = r["margin"] < 1e-4
    Jd = rec["J"]
    fin = np.isfinite(r["J"]) & np.isfinite(Jd) & ~amb
    scale = np.maximum(np.abs(r["J"]), r["absJ"])
    err_J = float((np.abs(Jd - r["J"])[fin] / scale[fin]).max())
    e2e = r if not amb.any() else pb.solve(warm(), rec["x0"], rec["t"], J_rep=Jd, rep_mask=amb.astype(np.uint8))
    stage = pb.solve(warm(), rec["x0"], rec["t"], J_rep=Jd, rep_mask=np.ones(Jd.size, np.uint8))
    sig = max(w["params"]["sigma"])
    U = rec["U"]
    return {"K": pb.cfg.K, "N": pb.cfg.N, "err_J": err_J,
            "err_U": float((np.abs(U - stage["U"]) / np.maximum(np.abs(stage["U"]), sig)).max()),
            "err_U_e2e": float((np.abs(U - e2e["U"]) / np.maximum(np.abs(e2e["U"]), sig)).max()),
            "err_J_min": abs(rec["info"]["J_min"] - stage["J_min"]) / max(abs(stage["J_min"]), 1e-300),
            "err_ess": abs(rec["info"]["ess"] - stage["ess"]) / stage["ess"],
            "ambiguous_samples": int(amb.sum()), "oracle_s": time.perf_counter() - t0}


def cpu_baseline(w, seconds: float = 12.0, single_seconds: float = 6.0):
    """The FP64 oracle as it stands on the host cores, repeated full solves
    of the benchmark workload for about `seconds` seconds with OpenMP over
    the samples, and for about `single_seconds` on one thread.  The thread
    count is the CPUs this process may run on, at most 16: the GPU host
    allots 16 CPUs per GPU, whatever the machine has."""
    model, nproc, usable = _cpu_info()
    cores = min(usable, 16)
    v, n, el = _time_oracle(w, cores, seconds)
    v1, n1, el1 = _time_oracle(w, 1, single_seconds)
    K, N = w["params"]["K"], w["params"]["N"]
    return {"value": v, "unit": "rollout-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} full solves of the benchmark workload (K={K}, N={N}) in {el:.1f} s, FP64, "
                      f"{cores} threads; {n1} solves in {el1:.1f} s on one thread",
            "single_thread_value": v1, "cpu_model": model, "nproc": nproc, "cpus_usable": usable,
            "thread_cap": "16 threads: the CPU share of one GPU on the GPU host"}


def _timing_stream():
    """The stream the extras time on: the current one, or a new one when the
    current one is the null stream (a context given the null stream makes a
    stream of its own, and events on the null stream would then time
    nothing of it)."""
    import torch
    s = torch.cuda.current_stream()
    return s if s.cuda_stream != 0 else torch.cuda.Stream()


def batched_bench(steps: int = 20, n: int = 256):
    """256 uneven instances (K in {1024..16384}, N in [30, 150], 5-12 gates),
    one persistent launch sequence per step under a captured HIP graph, launch
    shape picked by the autotuner.  Returns rollout-steps/s over the batch."""
    import torch
    from paper_2509_14726_amd import mppi as M
    from paper_2509_14726_amd import synth
    specs = synth.batch_instances(n)
    ws = [synth.single_solve_workload(K=d["K"], N=d["N"], n_gates=d["n_gates"], track_seed=d["track_seed"],
                                      seed=d["seed"]) for d in specs]
    stream = _timing_stream()
    solvers = [M.Solver(w["quad"], w["params"], gates=w["gates"], precision=M.FP32) for w in ws]
    B = M.Batch(solvers, stream=stream.cuda_stream)
    reqs = torch.zeros((n, M.REQ_DOUBLES), dtype=torch.float64, device="cuda")
    for i, w in enumerate(ws):
        reqs[i, :13] = torch.from_numpy(w["x0"])
    u0s = torch.zeros((n, 4), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    best, tuned_ms, _ = B.autotune(reqs.data_ptr(), u0s.data_ptr(), reps=3)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        B.solve_device(reqs.data_ptr(), u0s.data_ptr())
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    work = sum(d["K"] * d["N"] for d in specs)
    assert torch.isfinite(u0s).all().item()
    B.close()
    for sv in solvers:
        sv.close()
    return {"instances": n, "rollout_steps_per_batch": work, "ms_per_batch": ms,
            "rollout_steps_per_s": work / (ms * 1e-3), "autotuned": best, "autotune_ms": tuned_ms,
            "graph": True, "precision": "fp32"}


# Per-objective noise (thrust rate, N/s) and temperature of the race; the
# paper prints lambda = 0.01 for its own, unprinted, cost weights, so lambda
# is chosen here for this project's weights.
RACE_SETTINGS = {"gate": dict(sigma=20.0, lam=0.1), "contour": dict(sigma=10.0, lam=10.0),
                 "track": dict(sigma=5.0, lam=1.0)}


def closed_loop_race(seconds: float = 20.0):
    """The closed-loop race: the paper's input model (thrust rates, bounds
    +-10 N/s; progress acceleration +-20 m/s^2) with the sampling parameters
    of its simulation table (8192 samples, 20 steps of 0.03 s) on a seeded
    7-gate circuit, `seconds` of flight for each objective (gate progress;
    contouring on the 2000-point arc-length path; tracking of the 5 m/s
    reference).  Between solves the FP64 host plant (RK4, 4 substeps) advances
    with the first input of each solve, so every solve goes through the host
    entry point (upload, solve, download).  Reports the host-observed solve
    latency and the race metrics of the flight (paper_2509_14726_amd.race:
    waypoint pass errors, gate passes in order and lap time, tracking error,
    total-thrust profile)."""
    import numpy as np
    from paper_2509_14726_amd import mppi as M
    from paper_2509_14726_amd import race
    from paper_2509_14726_amd import synth
    out = {}
    dt = 0.03
    steps = int(round(seconds / dt))
    hover = synth.QUAD["mass"] * synth.QUAD["gravity"] / 4.0
    for obj in ("gate", "contour", "track"):
        st = RACE_SETTINGS[obj]
        w = synth.race_workload(K=8192, N=20, objective=obj, seed=1, track_seed=1, dt=dt, steps=steps,
                                sigma=(st["sigma"],) * 4, sigma_v=5.0, input_model=M.INPUT_RATE,
                                rate_lim=(-10.0, 10.0), dv_lim=(-20.0, 20.0), **{"lambda": st["lam"]})
        sv = M.Solver(w["quad"], w["params"], gates=w["gates"], path=w.get("path"),
                      path_len=w.get("path_len", 0.0), xref=w.get("xref"), ref_dt=w.get("ref_dt", 0.0),
                      precision=M.FP32)
        lat = []

        def solve(x, t):
            t0 = time.perf_counter()
            u0, _, info = sv.solve(x, t, want_U=False)
            lat.append(time.perf_counter() - t0)
            return u0, info

        x0 = np.concatenate([w["x0"], np.full(4, hover)])
        fl = race.fly(solve, w["quad"], x0, steps, dt, substeps=4)
        sv.close()
        n_done = len(lat)
        # latency over the steps after the first: the first solve of a
        # process also loads the kernels' code objects
        lat = np.array(lat[1:] if len(lat) > 1 else lat)
        rec = {"steps": n_done,
               "status": "ok" if fl["error"] is None else f"stopped at step {n_done}: {fl['error']}",
               "input": "thrust rate", "sigma_N_per_s": st["sigma"], "lambda": st["lam"], "K": 8192, "N": 20,
               "dt": dt, "solve_ms_mean": float(lat.mean() * 1e3),
               "solve_ms_p99": float(np.percentile(lat, 99) * 1e3)}
        infos = fl["info"]
        if obj == "gate":
            # switches of the controller's current gate (measured passes)
            rec["gates_passed"] = int(sum(1 for a, b in zip(infos, infos[1:]) if b["g0"] != a["g0"]))
        if obj == "contour":
            adv = 0.0
            for a, b in zip(infos, infos[1:]):
                d = b["theta0"] - a["theta0"]
                # the shorter way round the closed path
                if d < -0.5 * w["path_len"]:
                    d += w["path_len"]
                elif d > 0.5 * w["path_len"]:
                    d -= w["path_len"]
                adv += d
            rec["arc_length_m"] = adv
        r = race.score(fl, w, obj)
        r.pop("pass_times", None)
        rec["race"] = r
        out[obj] = rec
    return out


def paper_table_config(steps: int = 200):
    """The sampling parameters of the paper's simulation table (Sec. V-A,
    Table I: 8192 samples, 20-step horizon, dt = 0.03 s, lambda = 0.01) with
    this project's quadrotor and gate objective, as context for the paper's
    own solve time (about 0.4 ms on its desktop GPU, Sec. V-B): mean solve
    time device-driven and through the synchronous host entry point, with
    thrust as the input and with the paper's thrust-rate input."""
    import numpy as np
    import torch
    from paper_2509_14726_amd import mppi as M
    from paper_2509_14726_amd import synth
    out = {"K": 8192, "N": 20, "dt": 0.03, "lambda": 0.01, "paper_desktop_ms": 0.4,
           "paper_hardware": "RTX 3090, JAX (context, other hardware)"}
    hover = synth.QUAD["mass"] * synth.QUAD["gravity"] / 4.0
    for name, over in (("thrust_input", {}),
                       ("rate_input", dict(input_model=M.INPUT_RATE, rate_lim=(-10.0, 10.0), sigma=(20.0,) * 4))):
        w = synth.single_solve_workload(K=8192, N=20, dt=0.03, seed=1, **{"lambda": 0.01}, **over)
        stream = _timing_stream()
        sv = M.Solver(w["quad"], w["params"], gates=w["gates"], precision=M.FP32, stream=stream.cuda_stream)
        x0 = w["x0"] if not over else np.concatenate([w["x0"], np.full(4, hover)])
        req = torch.zeros((steps, M.REQ_DOUBLES), dtype=torch.float64, device="cuda")
        req[:, :13] = torch.from_numpy(w["x0"]).cuda()
        req[:, M.REQ_THRUST:M.REQ_THRUST + 4] = hover
        req[:, 13] = torch.arange(steps, dtype=torch.float64, device="cuda") * 0.03
        u0 = torch.zeros((steps, 4), dtype=torch.float64, device="cuda")
        for i in range(10):
            sv.solve_device(req[i].data_ptr(), u0[i].data_ptr())
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for i in range(steps):
            sv.solve_device(req[i].data_ptr(), u0[i].data_ptr())
        e1.record(stream)
        torch.cuda.synchronize()
        dev_ms = e0.elapsed_time(e1) / steps
        lat = []
        for i in range(steps):
            t0 = time.perf_counter()
            sv.solve(x0, (steps + i) * 0.03, want_U=False)
            lat.append(time.perf_counter() - t0)
        sv.close()
        out[name] = {"solve_ms_device": dev_ms, "solve_ms_host_entry_mean": float(np.mean(lat) * 1e3),
                     "rollout_steps_per_s": 8192 * 20 / (dev_ms * 1e-3)}
    return out


def fp64_solve(steps: int = 100):
    """The benchmark workload with every step of the path in binary64 (the
    FP64 variant): mean solve time, device-driven."""
    import torch
    from paper_2509_14726_amd import mppi as M
    from paper_2509_14726_amd import synth
    w = synth.single_solve_workload(K=8192, N=100, seed=1)
    stream = _timing_stream()
    sv = M.Solver(w["quad"], w["params"], gates=w["gates"], precision=M.FP64, stream=stream.cuda_stream)
    req = torch.zeros((steps + 10, M.REQ_DOUBLES), dtype=torch.float64, device="cuda")
    req[:, :13] = torch.from_numpy(w["x0"]).cuda()
    req[:, 13] = torch.arange(steps + 10, dtype=torch.float64, device="cuda") * 0.02
    u0 = torch.zeros((steps + 10, 4), dtype=torch.float64, device="cuda")
    for i in range(10):
        sv.solve_device(req[i].data_ptr(), u0[i].data_ptr())
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(10, steps + 10):
        sv.solve_device(req[i].data_ptr(), u0[i].data_ptr())
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    sv.close()
    return {"K": 8192, "N": 100, "ms_per_solve": ms, "rollout_steps_per_s": 8192 * 100 / (ms * 1e-3)}


def large_bench(steps: int = 5):
    """K = 262144, N = 200, dt = 0.01 on a 12-gate track: the N x K x 4 sample
    tensor (839 MB) streams through HBM; the final average accumulates in
    binary64."""
    import torch
    from paper_2509_14726_amd import mppi as M
    from paper_2509_14726_amd import synth
    w = synth.single_solve_workload(K=262144, N=200, dt=0.01, n_gates=12, track_seed=5, seed=5)
    stream = _timing_stream()
    sv = M.Solver(w["quad"], w["params"], gates=w["gates"], precision=M.FP32, stream=stream.cuda_stream)
    req = torch.zeros((steps + 1, M.REQ_DOUBLES), dtype=torch.float64, device="cuda")
    req[:, :13] = torch.from_numpy(w["x0"]).cuda()
    req[:, 13] = torch.arange(steps + 1, dtype=torch.float64, device="cuda") * 0.01
    u0 = torch.zeros((steps + 1, 4), dtype=torch.float64, device="cuda")
    sv.solve_device(req[0].data_ptr(), u0[0].data_ptr())
    torch.cuda.synchronize()
    sv.set_profiling(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(1, steps + 1):
        sv.solve_device(req[i].data_ptr(), u0[i].data_ptr())
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    kern, _ = sv.read_profile()
    _, info = sv.read_info()
    rec = _accuracy_record(sv, w["x0"], (steps + 1) * 0.01)
    # the same solve with the stored and with the regenerating average (the
    # context autotuner times both and restores the warm state)
    tune = sv.autotune(req[0].data_ptr(), reps=3, force=True)
    sv.close()
    K, N = 262144, 200
    # algorithmic bytes of the average: the sample tensor, the costs and the
    # tile minima, each read once (the blocks of later steps find the costs
    # in L2)
    avg_bytes = K * N * 16 + K * 4 + ((K + 64) // 64) * 4
    # with the rollout drawing its samples the first slot times the head kernel
    return {"K": K, "N": N, "ms_per_solve": ms, "rollout_steps_per_s": K * N / (ms * 1e-3),
            "rollout_draws_samples": bool(info["rollout_draw"]),
            "kernels_ms": {"head" if info["rollout_draw"] else "sample": float(kern[0]),
                           "rollout": float(kern[1]), "average": float(kern[2])},
            "average_bytes_per_launch": avg_bytes,
            "average_GBps": avg_bytes / (float(kern[2]) * 1e-3) / 1e9,
            "solve_ms_stored_average": tune["ms_stored"], "solve_ms_regenerating_average": tune["ms_regen"],
            "autotuner_choice": "regenerating" if tune["regen_average"] else "stored"}, w, rec


def _accuracy_record(sv, x0, t):
    """One more solve through the host entry point, with the warm state it
    started from and its sample costs: what the oracle comparison needs."""
    import numpy as np
    wd = sv.get_warm()
    u0, U, info = sv.solve(x0, t)
    J, _ = sv.read_samples()
    return {"warm": wd, "x0": np.array(x0, dtype=np.float64), "t": t, "u0": u0, "U": U, "info": info, "J": J}


def copy_calibration(mib: int, reps: int = 3):
    """A plain device-to-device copy of a known size: the HBM byte counters
    (FETCH_SIZE, WRITE_SIZE) read for it, divided by the bytes it moves, give
    the scale applied to the same counters of the library's kernels."""
    import torch
    x = torch.ones(mib * 2 ** 20 // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    return {"MiB": mib, "copies": reps, "bytes_read_per_copy": mib * 2 ** 20, "bytes_written_per_copy": mib * 2 ** 20}


def layout_sweep(steps: int = 30):
    """Device-driven solve time of every rollout layout (forced with
    MPPI_ROLLOUT_WAVES) around the automatic rule's crossover: the four-wave
    workgroups run one per CU, so past two rounds (2 x 256 tiles of 64
    samples) one wave per 64 samples wins."""
    import torch
    from paper_2509_14726_amd import mppi as M
    from paper_2509_14726_amd import synth
    stream = _timing_stream()
    rows = []
    for N in (50, 100, 200):
        for K in (8192, 16383, 16384, 32767, 32768, 65000):
            row = {"K": K, "N": N, "tiles": (K + 64) // 64}
            for waves in ("1", "2", "3", "4", ""):
                os.environ["MPPI_ROLLOUT_WAVES"] = waves
                w = synth.single_solve_workload(K=K, N=N, seed=2)
                sv = M.Solver(w["quad"], w["params"], gates=w["gates"], precision=M.FP32,
                              stream=stream.cuda_stream)
                req = torch.zeros((steps + 5, M.REQ_DOUBLES), dtype=torch.float64, device="cuda")
                req[:, :13] = torch.from_numpy(w["x0"]).cuda()
                req[:, 13] = torch.arange(steps + 5, dtype=torch.float64, device="cuda") * w["params"]["dt"]
                u0 = torch.zeros((steps + 5, 4), dtype=torch.float64, device="cuda")
                for i in range(5):
                    sv.solve_device(req[i].data_ptr(), u0[i].data_ptr())
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for i in range(5, steps + 5):
                    sv.solve_device(req[i].data_ptr(), u0[i].data_ptr())
                e1.record(stream)
                torch.cuda.synchronize()
                st, info = sv.read_info()
                assert st == M.OK, info
                row["auto" if waves == "" else f"waves{waves}_us"] = (
                    info["rollout_waves"] if waves == "" else 1e3 * e0.elapsed_time(e1) / steps)
                sv.close()
            os.environ.pop("MPPI_ROLLOUT_WAVES", None)
            print(json.dumps(row), flush=True)
            rows.append(row)
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--K", type=int, default=8192)
    ap.add_argument("--N", type=int, default=100)
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched, large-solve and serving measurements")
    ap.add_argument("--serving-seconds", type=float, default=60.0)
    ap.add_argument("--layout-sweep", action="store_true",
                    help="time every rollout layout over K and N around the automatic choice and exit")
    ap.add_argument("--regen", action="store_true",
                    help="the weighted average draws the samples again instead of reading the sample tensor")
    ap.add_argument("--large-only", action="store_true",
                    help="run only the large solve (K = 262144, N = 200) and print its figures; "
                         "for profiling its kernels")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device to device three times and exit: the known "
                         "traffic that scales the HBM byte counters of a profile")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path (asked for {args.gpus})",
              file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration > 0:
        print(json.dumps({"copy_calibration": copy_calibration(args.copy_calibration)}), flush=True)
        return
    if args.layout_sweep:
        import torch
        torch.cuda.set_stream(torch.cuda.Stream(torch.device("cuda:0")))
        layout_sweep()
        return
    if args.large_only:
        import torch
        # the extras time on the current stream: make it one of our own
        torch.cuda.set_stream(torch.cuda.Stream(torch.device("cuda:0")))
        print(json.dumps({"large": large_bench(steps=2)[0]}), flush=True)
        return

    import torch
    from paper_2509_14726_amd import mppi as M
    from paper_2509_14726_amd import synth

    w = synth.single_solve_workload(K=args.K, N=args.N, seed=1)
    prm = w["params"]
    if args.regen:
        prm = dict(prm, flags=M.FLAG_REGEN_AVERAGE)
    prec = M.FP32 if args.precision == "fp32" else M.FP64
    dev = torch.device("cuda:0")
    # a stream of our own (default priority): the solver's kernels and the
    # timing events share it
    stream = torch.cuda.Stream(dev)
    torch.cuda.set_stream(stream)
    solver = M.Solver(w["quad"], prm, gates=w["gates"], precision=prec, stream=stream.cuda_stream,
                      allocator=M.TorchAllocator(0))
    prof_steps = min(args.steps, 100)
    total = args.warmup + args.steps + prof_steps
    # one request record per step (state, time), resident in HBM
    reqs = torch.zeros((total, M.REQ_DOUBLES), dtype=torch.float64, device=dev)
    reqs[:, :13] = torch.from_numpy(w["x0"]).to(dev)
    reqs[:, 13] = torch.arange(total, dtype=torch.float64, device=dev) * prm["dt"]
    u0 = torch.zeros((total, 4), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()

    for i in range(args.warmup):
        solver.solve_device(reqs[i].data_ptr(), u0[i].data_ptr())
    torch.cuda.synchronize()
    # timed region: K solves, nothing else on the stream
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record(stream)
    for i in range(args.warmup, args.warmup + args.steps):
        solver.solve_device(reqs[i].data_ptr(), u0[i].data_ptr())
    t_end.record(stream)
    torch.cuda.synchronize()
    ms_total = t_start.elapsed_time(t_end)
    # per-kernel durations: HIP events recorded by the library on the solver's
    # stream around each kernel, over a second pass of solves
    solver.set_profiling(True)
    for i in range(args.warmup + args.steps, total):
        solver.solve_device(reqs[i].data_ptr(), u0[i].data_ptr())
    kern_ms, n_prof = solver.read_profile()
    st, info = solver.read_info()
    assert st == M.OK, info
    rk = rollout_kernel(info["rollout_waves"])
    # the counters hold for one workload; a forced layout is another
    wl = None if os.environ.get("MPPI_ROLLOUT_WAVES") else (args.K, args.N, args.precision,
                                                               int(info["regen_average"]))
    assert torch.isfinite(u0).all().item()

    K, N = args.K, args.N
    ms_per_step = ms_total / args.steps
    value = K * N / (ms_per_step * 1e-3)
    roll_ms = float(kern_ms[1])
    avg_ms = float(kern_ms[2])
    # algorithmic bytes of the weighted average: the sample tensor, the costs
    # and the tile minima, each read once (every horizon step's block reads
    # all costs, but only the first reaches HBM: L2 serves the others)
    avg_bytes = K * N * 16 + K * 4 + ((K + 64) // 64) * 4
    if info["regen_average"]:  # the samples are drawn again, not read
        avg_bytes -= K * N * 16
    flops = FLOPS_PER_ROLLOUT_STEP * K * N
    achieved = flops / (roll_ms * 1e-3) / 1e12
    # the rollout computes in the precision of the solve
    peak = PEAK_FP32_TFLOPS if prec == M.FP32 else PEAK_FP64_TFLOPS
    out = {
        "metric": f"rollout-steps/sec (K*N/s) at K={K},N={N}",
        "value": value,
        "unit": "rollout-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == M.FP32 else "f64",
        "data": "synthetic",
        "config": {"workload": f"single MPPI solve, gate-progress objective, K={K}, N={N}, dt={prm['dt']}, "
                               f"lambda={prm['lambda']}, sigma=1 N, seeded 7-gate track",
                   "K": K, "N": N, "objective": "gate", "precision": args.precision,
                   "average": "regenerated" if info["regen_average"] else "stored samples"},
        "kernels_ms": {"sample": float(kern_ms[0]), "rollout": roll_ms, "average": float(kern_ms[2]),
                       "solves_timed": n_prof},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic_bytes(rk, wl),
                     "kernel": rk, "flops_per_launch": flops},
        # the weighted average streams the sample tensor once: HBM-bound
        "average_kernel": {"bound": "hbm", "kernel": "k_final", "bytes_per_launch": avg_bytes,
                           "achieved": avg_bytes / (avg_ms * 1e-3) / 1e9, "peak": PEAK_HBM_GBPS,
                           "unit": "GB/s", "frac": avg_bytes / (avg_ms * 1e-3) / 1e9 / PEAK_HBM_GBPS,
                           "traffic": traffic_bytes("k_final", wl)},
    }
    if info["regen_average"]:
        # drawing the samples again it is bound by the vector ALU of the N
        # CUs that run its blocks: reported as redraws per second
        out["average_kernel"] = {"bound": "alu", "kernel": "k_final", "redraws_per_launch": K * N,
                                 "redraws_per_s": K * N / (avg_ms * 1e-3), "cus_used": min(N, 256),
                                 "bytes_per_launch": avg_bytes, "traffic": traffic_bytes("k_final", wl)}
    acc_records = [(w, _accuracy_record(solver, w["x0"], total * prm["dt"]))]
    solver.close()
    if not args.no_extras:
        for name, fn in (("batched", batched_bench), ("large", large_bench), ("closed_loop", closed_loop_race),
                         ("paper_table_config", paper_table_config), ("fp64", fp64_solve)):
            try:
                res = fn()
                if name == "large":
                    res, w_large, rec_large = res
                    acc_records.append((w_large, rec_large))
                out[name] = res
            except Exception as e:  # reported, never silently dropped
                out[name] = {"error": repr(e)}
        try:
            from paper_2509_14726_amd import serving
            out["serving"] = serving.simulate(n_drones=512, seconds=args.serving_seconds, rate_hz=50.0,
                                              budget_bytes=32 * 2 ** 30, n_slots=4)
        except Exception as e:
            out["serving"] = {"error": repr(e)}
        try:
            # the same drones with the contouring half on the paper's rate input
            from paper_2509_14726_amd import serving
            out["serving_rate_contour"] = serving.simulate(n_drones=512, seconds=args.serving_seconds,
                                                           rate_hz=50.0, budget_bytes=32 * 2 ** 30, n_slots=4,
                                                           contour_input="rate")
        except Exception as e:
            out["serving_rate_contour"] = {"error": repr(e)}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
        # the FP64 oracle from each measured solve's exported warm state
        cores = out["cpu_baseline"]["cores"]
        out["accuracy"] = {}
        for wk, rec in acc_records:
            key = "metric" if wk is w else "large"
            try:
                out["accuracy"][key] = oracle_errors(wk, rec, cores)
            except Exception as e:
                out["accuracy"][key] = {"error": repr(e)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
