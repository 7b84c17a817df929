"""Serving: continuous batching of solves from many drones.  Each result of
the mix must equal the same drone's solve sequence run alone (same warm-start
history), with the memory budget forcing admissions to wait."""
import numpy as np
import pytest

from paper_2509_14726_amd import mppi as M
from paper_2509_14726_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)


def drones(n, seed, external):
    rng = np.random.default_rng(seed)
    out = []
    for d in range(n):
        K = int(rng.choice([128, 512, 1024]))
        N = int(rng.choice([20, 40]))
        obj = "gate" if d % 2 == 0 else "contour"
        w = synth.single_solve_workload(K=K, N=N, objective=obj, seed=400 + d, track_seed=400 + d,
                                        **{"lambda": 30.0})
        if external:
            w["params"] = dict(w["params"], flags=M.FLAG_EXTERNAL_WORKSPACE)
        out.append(w)
    return out


def solver(w, prec=M.FP32):
    return M.Solver(w["quad"], w["params"], gates=w["gates"], path=w.get("path"),
                    path_len=w.get("path_len", 0.0), precision=prec)


@pytest.mark.parametrize("budget_mb,slots", [(512.0, 2), (2.0, 3)])
def test_alone_vs_mix(budget_mb, slots):
    say("alone vs mix", budget_mb, slots)
    n = 10
    ws = drones(n, 7, external=True)
    wa = drones(n, 7, external=False)
    served = [solver(w) for w in ws]
    alone = [solver(w) for w in wa]
    S = M.Server(served, budget_bytes=budget_mb * 2 ** 20, n_slots=slots, max_batch=4)
    rng = np.random.default_rng(3)
    steps = 4
    # each drone: a fixed sequence of requests (states from its own plant)
    xs = [w["x0"].copy() for w in wa]
    expected = {}
    reqs = []
    for k in range(steps):
        for d in range(n):
            t = k * 0.02
            u0, _, _ = alone[d].solve(xs[d], t)
            expected[(d, k)] = u0
            reqs.append((rng.uniform(0, 1) + k, d, xs[d].copy(), t, k))
            xs[d] = M.plant_step(wa[d]["quad"], xs[d], u0, 0.02, 2)
    reqs.sort(key=lambda r: r[0])
    tick = {}
    for i, (ta, d, x, t, k) in enumerate(reqs):
        tick[S.submit(d, x, t, ta)] = (d, k)
        if i % 5 == 0:
            S.progress(float(i))
    S.drain(1e9)
    res = S.poll()
    assert len(res) == n * steps
    seen = set()
    for r in res:
        d, k = tick[r["ticket"]]
        assert r["drone"] == d and r["status"] == M.OK
        assert np.array_equal(np.array(r["u0"]), expected[(d, k)]), (d, k)
        seen.add((d, k))
    assert len(seen) == n * steps
    st = S.stats()
    say("  stats", st)
    assert st["completed"] == n * steps and st["queued"] == 0 and st["in_flight"] == 0
    assert st["peak_bytes_in_flight"] <= budget_mb * 2 ** 20
    S.close()


def test_server_rejects_oversized_and_plain_contexts():
    say("server args")
    ws = drones(2, 8, external=True)
    served = [solver(w) for w in ws]
    with pytest.raises(M.MppiError):
        M.Server([solver(drones(1, 9, external=False)[0])], budget_bytes=1 << 20)
    S = M.Server(served, budget_bytes=4096)
    with pytest.raises(M.MppiError) as e:
        S.submit(0, ws[0]["x0"], 0.0, 0.0)
    assert e.value.status == M.E_NOMEM
    S.close()
    with pytest.raises(M.MppiError):
        served[0].solve(ws[0]["x0"], 0.0)  # no workspace of its own


@pytest.mark.parametrize("contour_input", ["thrust", "rate"])
def test_served_solves_against_the_oracle(contour_input):
    """Drones of the serving workload (K in {2048, 8192}, N in {50, 100},
    gate objective with thrust as the input, contouring with thrust or the
    rate input model, lambda = 10): every served
    solve over three rounds of requests compared with the FP64 oracle from
    the drone's exported warm state.  A served solve's workspace is lent
    back to the server when it retires, so its sample costs (needed to replay
    a decision within the ambiguity margin) come from a twin context of the
    same drone stepped alone, whose result must equal the served one bit for
    bit (a launch holds drones of one rollout layout, here the thrust drones'
    four-wave or the rate drones' one-wave layout)."""
    from oracle import oracle as O
    from paper_2509_14726_amd import serving
    from tests.parity import EPS_DEC, compare_result
    ws = serving.drone_workloads(6, contour_input=contour_input)
    shapes = [(w["params"]["K"], w["params"]["N"], w["params"]["objective"]) for w in ws]
    say("served vs oracle", contour_input, shapes)
    assert {K for K, _, _ in shapes} == {2048, 8192} and {N for _, N, _ in shapes} == {50, 100}
    served = [solver(w) for w in ws]
    twins = [solver(dict(w, params=dict(w["params"], flags=0))) for w in ws]
    orcs = [O.Problem(w["quad"], dict(w["params"], eps_dec=EPS_DEC[M.FP32], n_threads=8), gates=w["gates"],
                      path=w.get("path"), path_len=w.get("path_len", 0.0)) for w in ws]
    S = M.Server(served, budget_bytes=64 * 2 ** 20, n_slots=2, max_batch=3)
    xs = [w["x0"].copy() for w in ws]
    worst = 0.0
    n_amb = 0
    for k in range(3):
        wds = [sv.get_warm() for sv in served]
        t = k * 0.02
        tick = {S.submit(d, xs[d], t, float(d)): d for d in range(len(ws))}
        S.drain(1e9)
        res = S.poll()
        assert len(res) == len(ws)
        for r in res:
            d = tick[r["ticket"]]
            assert r["status"] == M.OK
            u0 = np.array(r["u0"])
            st, info = served[d].read_info()
            assert st == M.OK
            wn = served[d].get_warm()
            U = np.array(wn.U[:4 * ws[d]["params"]["N"]]).reshape(-1, 4)
            assert np.array_equal(u0, U[0])
            u0_t, U_t, _ = twins[d].solve(xs[d], t)
            assert np.array_equal(u0, u0_t) and np.array_equal(U, U_t), (k, d)
            Jd, _ = twins[d].read_samples()
            c = compare_result(orcs[d], wds[d], xs[d], t, M.FP32, u0, U, info, Jd=Jd, wn=wn)
            worst = max(worst, c["err_U_e2e"])
            n_amb += c["n_amb"]
            plant = M.plant_step_rate if xs[d].size == 17 else M.plant_step
            xs[d] = plant(ws[d]["quad"], xs[d], u0, 0.02, 4)
        say("  round", k, "worst end-to-end control error", worst, "ambiguous samples so far", n_amb)
    S.close()
    for sv in served + twins:
        sv.close()
