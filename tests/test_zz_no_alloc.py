"""The allocation-free solve entry point (mppi_solve_device_noalloc) against
mppi_solve_device, through the C ABI.

Both run the same kernels on the same inputs; only the per-solve workspace
differs (the library's fixed per-GPU array instead of the context's own), so
the first input, the report and the warm state handed on must agree bit for
bit.  Two workloads run back to back on the one fixed array, the second
smaller than the first, so stale contents of a larger solve would show.
"""
import sys

import numpy as np
import pytest

from paper_2509_14726_amd import mppi as M
from paper_2509_14726_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def _solver(w, precision, stream, flags=0):
    prm = dict(w["params"], flags=flags)
    return M.Solver(w["quad"], prm, gates=w["gates"], path=w.get("path"), path_len=w.get("path_len", 0.0),
                    xref=w.get("xref"), ref_dt=w.get("ref_dt", 0.0), precision=precision, stream=stream,
                    allocator=M.TorchAllocator(0))


def _warm_arrays(sv):
    wm = sv.get_warm()
    return (wm.warm, wm.g0, wm.solve_index, list(wm.allow), np.array(wm.U[:4 * sv.N]),
            np.array(wm.V[:sv.N]), wm.theta0)


def _run_pair(w, precision, steps, flags_b):
    import torch
    stream = torch.cuda.current_stream().cuda_stream
    a = _solver(w, precision, stream, flags=flags_b & ~M.FLAG_EXTERNAL_WORKSPACE)
    b = _solver(w, precision, stream, flags=flags_b)
    req = torch.zeros(M.REQ_DOUBLES, dtype=torch.float64, device="cuda")
    ua = torch.zeros(4, dtype=torch.float64, device="cuda")
    ub = torch.zeros(4, dtype=torch.float64, device="cuda")
    x = w["x0"].copy()
    dt = w["params"]["dt"]
    for step in range(steps):
        req[:13] = torch.from_numpy(x)
        req[13] = step * dt
        a.solve_device(req.data_ptr(), ua.data_ptr())
        b.solve_device_noalloc(req.data_ptr(), ub.data_ptr())
        sa, ia = a.read_info()
        sb, ib = b.read_info()
        assert sa == M.OK and sb == M.OK, (sa, sb, M.last_error(b.ctx))
        u_a = ua.cpu().numpy()
        u_b = ub.cpu().numpy()
        assert np.array_equal(u_a, u_b), (step, u_a, u_b)
        assert ia == ib, (step, ia, ib)
        wa, wb = _warm_arrays(a), _warm_arrays(b)
        for xa, xb in zip(wa, wb):
            assert np.array_equal(np.asarray(xa), np.asarray(xb)), step
        say("  step", step, "u0", np.round(u_a, 6), "J_min", ia["J_min"], "layout", ia["rollout_waves"])
        x = M.plant_step(w["quad"], x, u_a, dt, 2)
    a.close()
    b.close()


@pytest.mark.parametrize("precision", [M.FP32, M.FP64], ids=["fp32", "fp64"])
def test_noalloc_matches_device_entry_point(precision):
    """Benchmark-sized gate solve (K = 8192, N = 100), then a smaller
    contouring solve (K = 1000, N = 37) on a context without a workspace of
    its own, each over three warm-started steps."""
    say("noalloc: gate K=8192 N=100", precision)
    w1 = synth.single_solve_workload(K=8192, N=100, objective="gate", seed=2, track_seed=1)
    _run_pair(w1, precision, 3, flags_b=0)
    say("noalloc: contour K=1000 N=37 (external workspace context)", precision)
    w2 = synth.single_solve_workload(K=1000, N=37, objective="contour", seed=3, track_seed=2,
                                     **{"lambda": 20.0})
    _run_pair(w2, precision, 3, flags_b=M.FLAG_EXTERNAL_WORKSPACE)


def test_noalloc_tracking_after_larger_solve():
    """A tracking solve with the regenerating average (K = 333, N = 9) after
    a larger one has filled the array."""
    say("noalloc: track K=333 N=9 regen")
    w = synth.single_solve_workload(K=333, N=9, objective="track", seed=4, track_seed=3,
                                    **{"lambda": 5.0})
    _run_pair(w, M.FP32, 3, flags_b=M.FLAG_REGEN_AVERAGE)


def test_noalloc_rejects_workspace_above_limit():
    """K = 262144, N = 200 needs 839 MB of workspace: refused before any launch."""
    import torch
    say("noalloc: oversize refused")
    w = synth.single_solve_workload(K=262144, N=200, objective="gate", seed=1, track_seed=5, n_gates=12,
                                    dt=0.01)
    b = _solver(w, M.FP32, torch.cuda.current_stream().cuda_stream, flags=M.FLAG_EXTERNAL_WORKSPACE)
    req = torch.zeros(M.REQ_DOUBLES, dtype=torch.float64, device="cuda")
    req[:13] = torch.from_numpy(w["x0"])
    u0 = torch.zeros(4, dtype=torch.float64, device="cuda")
    with pytest.raises(M.MppiError) as e:
        b.solve_device_noalloc(req.data_ptr(), u0.data_ptr())
    assert e.value.status == M.E_INVAL
    assert "exceeds the fixed workspace" in str(e.value)
    b.close()
