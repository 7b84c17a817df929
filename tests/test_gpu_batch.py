"""Batched solves (one persistent launch sequence for many uneven contexts)
against the same contexts solved alone, through the C ABI."""
import sys

import numpy as np
import pytest

from paper_2509_14726_amd import mppi as M
from paper_2509_14726_amd import synth
from tests.parity import build_pair, solve_and_compare, warm_to_oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)


def make_instances(n, seed, objectives=("gate",), precision=M.FP32):
    rng = np.random.default_rng(seed)
    inst = []
    for i in range(n):
        K = int(rng.choice([64, 200, 1024, 2048]))
        N = int(rng.integers(5, 60))
        obj = objectives[i % len(objectives)]
        w = synth.single_solve_workload(K=K, N=N, objective=obj, seed=100 + i, track_seed=100 + i,
                                        n_gates=int(rng.integers(5, 13)), **{"lambda": 30.0})
        inst.append(w)
    return inst


def solver_for(w, precision):
    return M.Solver(w["quad"], w["params"], gates=w["gates"], path=w.get("path"),
                    path_len=w.get("path_len", 0.0), xref=w.get("xref"), ref_dt=w.get("ref_dt", 0.0),
                    precision=precision)


@pytest.mark.parametrize("precision", [M.FP32, M.FP64])
@pytest.mark.parametrize("use_graph,waves", [(True, 4), (True, 3), (False, 2), (True, 1)])
def test_batch_equals_solo(precision, use_graph, waves, monkeypatch):
    import torch
    say("batch vs solo", precision, "graph", use_graph, "waves", waves)
    monkeypatch.setenv("MPPI_ROLLOUT_WAVES", str(waves))
    inst = make_instances(12, seed=1, objectives=("gate", "contour", "track"), precision=precision)
    solo = [solver_for(w, precision) for w in inst]
    bat = [solver_for(w, precision) for w in inst]
    B = M.Batch(bat, rollout_waves=waves, use_graph=use_graph)
    n = len(inst)
    reqs = torch.zeros((n, M.REQ_DOUBLES), dtype=torch.float64, device="cuda")
    u0s = torch.zeros((n, 4), dtype=torch.float64, device="cuda")
    xs = [w["x0"].copy() for w in inst]
    for step in range(4):
        for i, w in enumerate(inst):
            reqs[i, :13] = torch.from_numpy(xs[i])
            reqs[i, 13] = step * w["params"]["dt"]
        torch.cuda.synchronize()
        B.solve_device(reqs.data_ptr(), u0s.data_ptr())
        torch.cuda.synchronize()
        got = u0s.cpu().numpy()
        for i, w in enumerate(inst):
            u0, U, info = solo[i].solve(xs[i], step * w["params"]["dt"])
            st, info_b = bat[i].read_info()
            assert st == M.OK
            assert np.array_equal(got[i], u0), (step, i, got[i], u0)
            assert info_b["J_min"] == info["J_min"] and info_b["g0"] == info["g0"]
            Jb, _ = bat[i].read_samples()
            Js, _ = solo[i].read_samples()
            assert np.array_equal(Jb, Js)
            xs[i] = M.plant_step(w["quad"], xs[i], u0, w["params"]["dt"], 2)
    B.close()


def test_batch_subsets_and_graph_replays():
    """Replays of one captured graph with changing subsets: each replay
    equals the eager (uncaptured) result for the same subset, and contexts
    outside a subset keep their warm state."""
    import torch
    say("subsets")
    inst = make_instances(10, seed=2)
    A = [solver_for(w, M.FP32) for w in inst]
    E = [solver_for(w, M.FP32) for w in inst]
    BA = M.Batch(A, rollout_waves=1, use_graph=True)
    BE = M.Batch(E, rollout_waves=1, use_graph=False)
    n = len(inst)
    reqs = torch.zeros((n, M.REQ_DOUBLES), dtype=torch.float64, device="cuda")
    for i, w in enumerate(inst):
        reqs[i, :13] = torch.from_numpy(w["x0"])
    ua = torch.zeros((n, 4), dtype=torch.float64, device="cuda")
    ue = torch.zeros((n, 4), dtype=torch.float64, device="cuda")
    subsets = [list(range(n)), [3, 1, 7], [0], [9, 8, 7, 6, 5, 4], [2, 5]]
    count = [0] * n
    for r, sub in enumerate(subsets):
        sub_reqs = reqs[sub].contiguous()
        sub_reqs[:, 13] = 0.02 * (r + 1)
        torch.cuda.synchronize()
        BA.solve_device(sub_reqs.data_ptr(), ua.data_ptr(), active=sub)
        BE.solve_device(sub_reqs.data_ptr(), ue.data_ptr(), active=sub)
        torch.cuda.synchronize()
        assert torch.equal(ua[:len(sub)], ue[:len(sub)]), r
        for i in sub:
            count[i] += 1
        for i in range(n):
            assert A[i].get_warm().solve_index == count[i] == E[i].get_warm().solve_index
    BA.close()
    BE.close()


def test_batch_rejects_bad_arguments():
    say("batch args")
    inst = make_instances(2, seed=3)
    S = [solver_for(w, M.FP32) for w in inst]
    with pytest.raises(M.MppiError):
        M.Batch([S[0], S[0]])
    B = M.Batch(S)
    with pytest.raises(M.MppiError):
        B.solve_device(0, 0, active=[0])  # null requests
    import torch
    reqs = torch.zeros((2, M.REQ_DOUBLES), dtype=torch.float64, device="cuda")
    with pytest.raises(M.MppiError):
        B.solve_device(reqs.data_ptr(), 0, active=[0, 0])
    with pytest.raises(M.MppiError):
        B.solve_device(reqs.data_ptr(), 0, active=[5])
    B.close()


def test_autotuner_picks_a_valid_shape(tmp_path):
    import json

    import torch
    say("autotune")
    inst = make_instances(8, seed=4)
    S = [solver_for(w, M.FP32) for w in inst]
    B = M.Batch(S)
    reqs = torch.zeros((len(S), M.REQ_DOUBLES), dtype=torch.float64, device="cuda")
    for i, w in enumerate(inst):
        reqs[i, :13] = torch.from_numpy(w["x0"])
    u0s = torch.zeros((len(S), 4), dtype=torch.float64, device="cuda")
    before = [sv.get_warm() for sv in S]
    cache = str(tmp_path / "tune.json")
    best, ms, hit = B.autotune(reqs.data_ptr(), u0s.data_ptr(), reps=2, cache_path=cache)
    say("  best", best, ms, hit)
    assert not hit and best["rollout_waves"] in (1, 2, 3, 4) and best["rollout_groups"] > 0 and ms > 0
    assert best["regen_average"] in (0, 1) and (best["rollout_waves"] >= 3 or best["regen_average"] == 0)
    got = B.get_cfg()
    assert got["rollout_waves"] == best["rollout_waves"] and got["regen_average"] == best["regen_average"]
    # the timed steps left every context's warm state as it was
    for sv, wb in zip(S, before):
        wa = sv.get_warm()
        assert wa.solve_index == wb.solve_index and wa.warm == wb.warm
        assert list(wa.U) == list(wb.U)
    # the cache holds the choice: a second tuner applies it without timing
    data = json.load(open(cache))
    assert len(data) == 1 and list(data.values())[0]["rollout_waves"] == best["rollout_waves"]
    B.set_cfg()
    best2, ms2, hit2 = B.autotune(reqs.data_ptr(), u0s.data_ptr(), reps=2, cache_path=cache)
    assert hit2 and best2 == best and ms2 == pytest.approx(ms, rel=1e-5)
    assert B.get_cfg()["rollout_waves"] == best["rollout_waves"]
    B.close()


def test_chunk_sizes_give_the_same_bits(monkeypatch):
    """Four-wave rollouts with 4-step chunks and with 2-step chunks compute
    the same bits: the small contexts run alone with 4-step chunks (at most
    one tile per CU); the first has more tiles than CUs and so 2-step chunks,
    the contexts disagree, and the batch (more tiles than CUs in total) runs
    them all with 2-step chunks, two workgroups per CU."""
    import torch
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    monkeypatch.setenv("MPPI_ROLLOUT_WAVES", "4")
    say("chunk sizes", "CUs", n_cu)
    inst = []
    for i, (K, obj) in enumerate([(n_cu * 64 + 100, "gate"), (2000, "contour"), (3000, "track"), (700, "gate")]):
        inst.append(synth.single_solve_workload(K=K, N=24, objective=obj, seed=300 + i, track_seed=300 + i,
                                                **{"lambda": 20.0}))
    solo = [solver_for(w, M.FP32) for w in inst]
    bat = [solver_for(w, M.FP32) for w in inst]
    B = M.Batch(bat, rollout_waves=4, use_graph=True)
    n = len(inst)
    reqs = torch.zeros((n, M.REQ_DOUBLES), dtype=torch.float64, device="cuda")
    u0s = torch.zeros((n, 4), dtype=torch.float64, device="cuda")
    for step in range(2):
        for i, w in enumerate(inst):
            reqs[i, :13] = torch.from_numpy(w["x0"])
            reqs[i, 13] = step * w["params"]["dt"]
        torch.cuda.synchronize()
        B.solve_device(reqs.data_ptr(), u0s.data_ptr())
        torch.cuda.synchronize()
        got = u0s.cpu().numpy()
        for i, w in enumerate(inst):
            u0, U, info = solo[i].solve(w["x0"], step * w["params"]["dt"])
            assert np.array_equal(got[i], u0), (step, i)
            Jb, _ = bat[i].read_samples()
            Js, _ = solo[i].read_samples()
            assert np.array_equal(Jb, Js), (step, i)
    B.close()
    for s in solo + bat:
        s.close()


def _batch_slice():
    """Instances of the 256-instance batch workload (K from {1024..16384},
    N in [30, 150], 5..12 gates, lambda = 1, sigma = 1 N): the first 20, plus
    the first instances with K = 16384 and with the longest horizons."""
    spec = synth.batch_instances(256, seed=3)
    pick = list(range(20))
    pick += [i for i, s in enumerate(spec) if s["K"] == 16384 and i not in pick][:2]
    longest = sorted(range(len(spec)), key=lambda i: -spec[i]["N"])
    pick += [i for i in longest if i not in pick][:2]
    out = []
    for i in pick:
        s = spec[i]
        out.append((i, synth.single_solve_workload(K=s["K"], N=s["N"], seed=s["seed"], track_seed=s["track_seed"],
                                                   n_gates=s["n_gates"])))
    return out


@pytest.mark.parametrize("waves", [0, 1], ids=["automatic", "one-wave"])
def test_batch_against_the_oracle(waves):
    """Batched binary32 solves of the benchmark's uneven instances, each
    compared with the FP64 oracle solving from the same exported warm state:
    a cold and a warm step under a captured graph."""
    import torch
    from tests.parity import compare_result
    sl = _batch_slice()
    say("batch vs oracle", "waves", waves, "instances", [i for i, _ in sl],
        "K", [w["params"]["K"] for _, w in sl], "N", [w["params"]["N"] for _, w in sl])
    assert max(w["params"]["K"] for _, w in sl) == 16384 and max(w["params"]["N"] for _, w in sl) >= 148
    pairs = [build_pair(w, M.FP32) for _, w in sl]
    B = M.Batch([d for d, _ in pairs], rollout_waves=waves, use_graph=True)
    n = len(sl)
    reqs = torch.zeros((n, M.REQ_DOUBLES), dtype=torch.float64, device="cuda")
    u0s = torch.zeros((n, 4), dtype=torch.float64, device="cuda")
    xs = [w["x0"].copy() for _, w in sl]
    worst = 0.0
    for step in range(2):
        wds = [d.get_warm() for d, _ in pairs]
        for i, (_, w) in enumerate(sl):
            reqs[i, :13] = torch.from_numpy(xs[i])
            reqs[i, 13] = step * w["params"]["dt"]
        torch.cuda.synchronize()
        B.solve_device(reqs.data_ptr(), u0s.data_ptr())
        torch.cuda.synchronize()
        got = u0s.cpu().numpy()
        for i, (idx, w) in enumerate(sl):
            dev, orc = pairs[i]
            st, info = dev.read_info()
            assert st == M.OK
            wn = dev.get_warm()
            U = np.array(wn.U[:4 * w["params"]["N"]]).reshape(-1, 4)
            assert np.array_equal(got[i], U[0])
            Jd, _ = dev.read_samples()
            r = compare_result(orc, wds[i], xs[i], step * w["params"]["dt"], M.FP32, got[i], U, info, Jd=Jd, wn=wn)
            worst = max(worst, r["err_U_e2e"])
            xs[i] = M.plant_step(w["quad"], xs[i], got[i], w["params"]["dt"], 2)
        say("  step", step, "layout", B.get_cfg(), "worst end-to-end control error", worst)
    B.close()
    for d, _ in pairs:
        d.close()


@pytest.mark.parametrize("precision", [M.FP32, M.FP64])
@pytest.mark.parametrize("waves", [4, 3])
def test_batch_regenerating_average_equals_stored(precision, waves, monkeypatch):
    """A batch whose rollout writes no sample tensor and whose average draws
    the samples again gives the same first inputs, costs and warm state, bit
    for bit, as the same batch with the stored tensor; with one-wave rollouts
    the setting has no effect."""
    import torch
    say("batch regen vs stored", precision, "waves", waves)
    monkeypatch.setenv("MPPI_ROLLOUT_WAVES", str(waves))
    inst = make_instances(9, seed=11, objectives=("gate", "contour", "track"), precision=precision)
    A = [solver_for(w, precision) for w in inst]
    S = [solver_for(w, precision) for w in inst]
    BA = M.Batch(A, rollout_waves=waves, regen_average=True)
    BS = M.Batch(S, rollout_waves=waves)
    assert BA.get_cfg()["regen_average"] == 1 and BS.get_cfg()["regen_average"] == 0
    n = len(inst)
    reqs = torch.zeros((n, M.REQ_DOUBLES), dtype=torch.float64, device="cuda")
    ua = torch.zeros((n, 4), dtype=torch.float64, device="cuda")
    us = torch.zeros((n, 4), dtype=torch.float64, device="cuda")
    xs = [w["x0"].copy() for w in inst]
    for step in range(3):
        for i, w in enumerate(inst):
            reqs[i, :13] = torch.from_numpy(xs[i])
            reqs[i, 13] = step * w["params"]["dt"]
        BA.solve_device(reqs.data_ptr(), ua.data_ptr())
        BS.solve_device(reqs.data_ptr(), us.data_ptr())
        torch.cuda.synchronize()
        assert torch.equal(ua, us), step
        for i, w in enumerate(inst):
            Ja, _ = A[i].read_samples()
            Js, _ = S[i].read_samples()
            assert np.array_equal(Ja, Js)
            assert list(A[i].get_warm().U) == list(S[i].get_warm().U)
            xs[i] = M.plant_step(w["quad"], xs[i], us[i].cpu().numpy(), w["params"]["dt"], 2)
    # its solves kept no sample tensor to read
    with pytest.raises(M.MppiError):
        A[0].read_samples(want_U=True)
    S[0].read_samples(want_U=True)
    BA.set_cfg(rollout_waves=1, regen_average=True)
    assert BA.get_cfg()["regen_average"] == 0
    BA.close()
    BS.close()
