"""CPU checks of the C ABI boundary: the library loads, exports every entry
point that include/mppi.h declares, the binding mirrors the header's structs,
and the host-only paths (argument validation, status strings, plant step)
behave as documented.  No compute call needs a GPU here."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2509_14726_amd import mppi as M
from paper_2509_14726_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "mppi.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mppi_[a-z_]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert len(names) >= 13
    lib = C.CDLL(M.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(M.EXPORTS) == names


def test_struct_sizes_match_header_layout():
    # sizes implied by the C declarations (x86-64 ABI)
    assert C.sizeof(M.mppi_quad) == 8 * 13
    assert C.sizeof(M.mppi_info) == 5 * 8 + 8 * 4
    assert C.sizeof(M.mppi_warm) == 4 * 4 + 9 * 4 + 4 + 8 + 13 * 8 + 8 + 256 * 4 * 8 + 256 * 8 + 8
    assert M.mppi_params.R_dT.offset == 4 * 4 + 8 * 2 + 8 * 4 + 8 + 8 + 8 * 3 + 13 * 8 * 2
    # the variants and the input model follow the flags
    off = M.mppi_params.flags.offset + 4
    assert M.mppi_params.n_iter.offset == off and M.mppi_params.ctrl_cost.offset == off + 8  # padded to 8
    assert M.mppi_params.input_model.offset == off + 16 and M.mppi_params.rate_lim.offset == off + 24
    assert C.sizeof(M.mppi_params) == off + 24 + 32
    assert M.REQ_DOUBLES == 24 and M.REQ_THRUST == 16


def test_status_strings():
    assert M.lib.mppi_status_string(M.E_NONFINITE) == b"MPPI_E_NONFINITE"
    assert M.lib.mppi_status_string(M.OK) == b"MPPI_OK"
    assert M.lib.mppi_status_string(-99) == b"MPPI_E_UNKNOWN"


@pytest.mark.parametrize("over,frag", [
    (dict(K=0), "K=0"), (dict(N=0), "N=0"), (dict(N=257), "N=257"), (dict(dt=0.0), "dt"),
    (dict(**{"lambda": -1.0}), "lambda"), (dict(sigma=(1.0, -1.0, 1.0, 1.0)), "sigma[1]"),
    (dict(objective=7), "objective"), (dict(n_iter=65), "n_iter"), (dict(ctrl_cost=-1.0), "ctrl_cost"),
    (dict(input_model=5), "input model"), (dict(input_model=1, rate_lim=(1.0, 10.0)), "bounds"),
])
def test_create_rejects_invalid_parameters_before_touching_the_device(over, frag):
    w = synth.single_solve_workload(K=64, N=10)
    prm = dict(w["params"], **over)
    with pytest.raises(M.MppiError) as e:
        M.Solver(w["quad"], prm, gates=w["gates"])
    assert e.value.status == M.E_INVAL
    assert frag in str(e.value)


def test_create_rejects_missing_problem_data():
    w = synth.single_solve_workload(K=64, N=10)
    with pytest.raises(M.MppiError):
        M.Solver(w["quad"], w["params"])  # gate objective without gates
    prm = dict(w["params"], objective=M.OBJ_CONTOUR)
    with pytest.raises(M.MppiError):
        M.Solver(w["quad"], prm, gates=w["gates"])  # no path
    with pytest.raises(M.MppiError):
        M.Solver(w["quad"], prm, path=np.zeros((10, 6)), path_len=1.0)  # v_max dt >= L


def test_create_rejects_more_gates_than_the_bound():
    w = synth.single_solve_workload(K=64, N=10)
    g = np.zeros((M.G_MAX + 1, 4))
    g[:, 0] = np.arange(M.G_MAX + 1)
    with pytest.raises(M.MppiError) as e:
        M.Solver(w["quad"], w["params"], gates=g)
    assert e.value.status == M.E_INVAL and "gates" in str(e.value)


def test_plant_step_free_fall_and_hover():
    q = synth.QUAD
    x = np.zeros(13); x[6] = 1.0; x[2] = 10.0; x[3] = 1.0
    y = M.plant_step(q, x, np.zeros(4), 0.1, 3)
    np.testing.assert_allclose(y[0:3], [0.1, 0.0, 10.0 - 0.5 * 9.81 * 0.01], atol=1e-13)
    h = synth.hover_thrust()
    x = np.zeros(13); x[6] = 1.0
    np.testing.assert_allclose(M.plant_step(q, x, np.full(4, h), 0.02, 1), x, atol=1e-14)
    with pytest.raises(M.MppiError):
        M.plant_step(q, x, np.zeros(4), 0.02, 0)


def test_destroy_null_is_a_no_op():
    M.lib.mppi_destroy(None)
    M.lib.mppi_batch_destroy(None)
    M.lib.mppi_server_destroy(None)


# device blocks mppi_create asks its allocator for, gate objective: warm
# state, warm U, warm V, head values, report, request record, per-solve
# workspace, gate table (binary64 copy, device-precision copy)
N_DEVICE_BLOCKS_GATE = 9


@pytest.mark.parametrize("fail_at", range(1, N_DEVICE_BLOCKS_GATE + 1))
def test_failing_allocator_gives_nomem_and_frees_what_it_got(fail_at):
    """An allocator callback that fails on its fail_at-th call: mppi_create
    returns MPPI_E_NOMEM, leaves *out NULL and hands back every block it was
    given.  The allocations come before the first HIP call, so this runs on a
    host without a GPU; the fake blocks are never dereferenced."""
    w = synth.single_solve_workload(K=64, N=10)
    calls, live, freed = [0], {}, []

    def alloc(nbytes, user):
        calls[0] += 1
        if calls[0] == fail_at:
            return None
        buf = C.create_string_buffer(int(nbytes) + 256)
        ptr = (C.addressof(buf) + 255) // 256 * 256
        live[ptr] = buf
        return ptr

    def free(ptr, user):
        freed.append(int(ptr))
        live.pop(int(ptr))

    af, ff = M.ALLOC_FN(alloc), M.FREE_FN(free)
    al = M.mppi_allocator(af, ff, None)
    quad = M.make_quad(w["quad"])
    prm = M.make_params(w["params"], M.FP32)
    pb = M.mppi_problem()
    g = np.ascontiguousarray(w["gates"], dtype=np.float64)
    pb.gates = g.ctypes.data_as(C.POINTER(C.c_double)); pb.n_gates = g.shape[0]; pb.gate_size = 1.5
    out = C.c_void_p(1234)
    st = M.lib.mppi_create(C.byref(prm), C.byref(quad), C.byref(pb), None, C.byref(al), C.byref(out))
    assert st == M.E_NOMEM, (st, M.last_error(None))
    assert out.value is None
    assert calls[0] == fail_at
    assert len(freed) == fail_at - 1 and not live
    assert "allocation" in M.last_error(None)


def test_allocator_needs_both_callbacks():
    w = synth.single_solve_workload(K=64, N=10)
    al = M.mppi_allocator(M.ALLOC_FN(lambda n, u: None), M.FREE_FN(), None)
    quad = M.make_quad(w["quad"])
    prm = M.make_params(w["params"], M.FP32)
    pb = M.mppi_problem()
    g = np.ascontiguousarray(w["gates"], dtype=np.float64)
    pb.gates = g.ctypes.data_as(C.POINTER(C.c_double)); pb.n_gates = g.shape[0]; pb.gate_size = 1.5
    out = C.c_void_p()
    st = M.lib.mppi_create(C.byref(prm), C.byref(quad), C.byref(pb), None, C.byref(al), C.byref(out))
    assert st == M.E_INVAL and out.value is None


def test_rate_plant_reduces_to_the_thrust_plant_and_saturates():
    """mppi_plant_step_rate (host, binary64): a zero rate is the thrust
    plant at the held thrusts; a rate that would carry a thrust past its
    bound stops it there; the closed-form cubic climb of a thrust ramp."""
    import numpy as np
    q = synth.QUAD
    rng = np.random.default_rng(2)
    x = np.concatenate([rng.normal(size=6), [1.0, 0.0, 0.0, 0.0], rng.normal(size=3), rng.uniform(1, 6, 4)])
    xr = M.plant_step_rate(q, x, np.zeros(4), 0.02, 4)
    np.testing.assert_array_equal(xr[:13], M.plant_step(q, x[:13], x[13:], 0.02, 4))
    np.testing.assert_array_equal(xr[13:], x[13:])
    x[13:] = [6.9, 0.1, 3.0, 3.0]
    xr = M.plant_step_rate(q, x, np.array([50.0, -50.0, 1.0, -1.0]), 0.02, 4)
    np.testing.assert_allclose(xr[13:], [q["t_max"], q["t_min"], 3.02, 2.98], rtol=0, atol=1e-12)
    T0, r, t = 1.7, 3.0, 0.4
    x = np.array([0, 0, 1.0, 0, 0, 0.5, 1, 0, 0, 0, 0, 0, 0, T0, T0, T0, T0], float)
    xr = M.plant_step_rate(q, x, np.full(4, r), t, 40)
    m, g = q["mass"], q["gravity"]
    z = 1.0 + 0.5 * t + (4 * T0 / m - g) * t * t / 2 + (4 * r / m) * t ** 3 / 6
    assert abs(xr[2] - z) < 1e-12
