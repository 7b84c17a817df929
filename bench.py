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

# Algorithmic work of one rollout step of the gate objective, counted from the
# method's definition (see the design notes): RK4 of Eq. (2) 437 flops, gate
# cost (Eq. (6)-(7), switch test, rate penalty) 58 flops.
FLOPS_PER_ROLLOUT_STEP = 495
# Peak FP32 vector throughput of MI355X (256 CUs, 2.4 GHz, packed FMA)
PEAK_FP32_TFLOPS = 157.3


def cpu_baseline(w, seconds: float = 12.0):
    """The FP64 oracle as it stands, on all host cores (at most 16), repeated
    full solves of the benchmark workload for about `seconds` seconds."""
    from oracle import oracle as O
    cores = min(os.cpu_count() or 1, 16)
    prm = dict(w["params"], eps_dec=0.0, n_threads=cores)
    pb = O.Problem(w["quad"], prm, gates=w["gates"])
    warm = pb.warm()
    K, N = prm["K"], prm["N"]
    n, t0 = 0, time.perf_counter()
    while True:
        r = pb.solve(warm, w["x0"], n * prm["dt"])
        assert r["status"] == O.OK
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds or n >= 1000:
            break
    return {"value": n * K * N / el, "unit": "rollout-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} full solves of the benchmark workload (K={K}, N={N}) in {el:.1f} s, FP64"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--K", type=int, default=8192)
    ap.add_argument("--N", type=int, default=100)
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path (asked for {args.gpus})",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2509_14726_amd import mppi as M
    from paper_2509_14726_amd import synth

    w = synth.single_solve_workload(K=args.K, N=args.N, seed=1)
    prm = w["params"]
    prec = M.FP32 if args.precision == "fp32" else M.FP64
    dev = torch.device("cuda:0")
    # a stream of our own (default priority): the solver's kernels and the
    # timing events share it
    stream = torch.cuda.Stream(dev)
    torch.cuda.set_stream(stream)
    solver = M.Solver(w["quad"], prm, gates=w["gates"], precision=prec, stream=stream.cuda_stream,
                      allocator=M.TorchAllocator(0))
    total = args.warmup + args.steps
    # one request record per step (state, time), resident in HBM
    reqs = torch.zeros((total, M.REQ_DOUBLES), dtype=torch.float64, device=dev)
    reqs[:, :13] = torch.from_numpy(w["x0"]).to(dev)
    reqs[:, 13] = torch.arange(total, dtype=torch.float64, device=dev) * prm["dt"]
    u0 = torch.zeros((total, 4), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()

    for i in range(args.warmup):
        solver.solve_device(reqs[i].data_ptr(), u0[i].data_ptr())
    torch.cuda.synchronize()
    solver.set_profiling(True)
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record(stream)
    for i in range(args.warmup, total):
        solver.solve_device(reqs[i].data_ptr(), u0[i].data_ptr())
    t_end.record(stream)
    torch.cuda.synchronize()
    ms_total = t_start.elapsed_time(t_end)
    kern_ms, n_prof = solver.read_profile()
    st, info = solver.read_info()
    assert st == M.OK, info
    assert torch.isfinite(u0).all().item()

    K, N = args.K, args.N
    ms_per_step = ms_total / args.steps
    value = K * N / (ms_per_step * 1e-3)
    roll_ms = float(kern_ms[1])
    flops = FLOPS_PER_ROLLOUT_STEP * K * N
    achieved = flops / (roll_ms * 1e-3) / 1e12
    out = {
        "metric": "rollout-steps/sec (K*N/s) at K=8192,N=100",
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
                   "K": K, "N": N, "objective": "gate", "precision": args.precision},
        "kernels_ms": {"sample": float(kern_ms[0]), "rollout": roll_ms, "average": float(kern_ms[2]),
                       "solves_timed": n_prof},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None,
                     "kernel": "k_rollout", "flops_per_launch": flops},
    }
    solver.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
