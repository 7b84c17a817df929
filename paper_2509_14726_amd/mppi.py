"""ctypes binding of libmppi.so (the HIP C ABI of include/mppi.h).

Argument marshalling only: every step of a solve runs in the library's HIP
kernels.  The module raises at import when the library is missing; there is
no CPU fallback.  PyTorch, when used, only provides device memory (through
the allocator callbacks) and streams.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# MPPI_LIBRARY names another build of the same library (the host-sanitizer
# build of paper_2509_14726_amd.sanitize); by default the in-tree one.
LIB_PATH = os.environ.get("MPPI_LIBRARY") or os.path.join(HERE, "libmppi.so")

N_MAX = 256
K_MAX = 1 << 24
G_MAX = 256
MASK_WORDS = 9
REQ_DOUBLES = 24
REQ_THRUST = 16      # request slots of the measured thrusts (rate model)
SCRATCH_BYTES = 32 << 20
OK, E_INVAL, E_NOMEM, E_DEVICE, E_NONFINITE = 0, -1, -2, -3, -4
OBJ_GATE, OBJ_CONTOUR, OBJ_TRACK = 0, 1, 2
FP32, FP64 = 0, 1
INPUT_THRUST, INPUT_RATE = 0, 1

EXPORTS = ["mppi_create", "mppi_destroy", "mppi_solve", "mppi_solve_device",
           "mppi_solve_device_noalloc", "mppi_read_info",
           "mppi_read_samples", "mppi_get_warm", "mppi_set_warm", "mppi_last_error",
           "mppi_status_string", "mppi_plant_step", "mppi_plant_step_rate", "mppi_set_profiling",
           "mppi_read_profile", "mppi_autotune",
           "mppi_batch_create", "mppi_batch_solve_device", "mppi_batch_set_cfg", "mppi_batch_get_cfg",
           "mppi_batch_autotune", "mppi_batch_destroy", "mppi_batch_last_error",
           "mppi_server_create", "mppi_server_submit", "mppi_server_progress", "mppi_server_poll",
           "mppi_server_drain", "mppi_server_get_stats", "mppi_server_destroy", "mppi_server_last_error"]


class MppiError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{status}: {msg}")
        self.status = status


class mppi_quad(C.Structure):
    _fields_ = [("mass", C.c_double), ("arm", C.c_double), ("inertia", C.c_double * 3),
                ("c_tau", C.c_double), ("drag", C.c_double * 3), ("gravity", C.c_double),
                ("t_min", C.c_double), ("t_max", C.c_double), ("w_max", C.c_double)]


class mppi_params(C.Structure):
    _fields_ = [("K", C.c_int32), ("N", C.c_int32), ("objective", C.c_int32),
                ("precision", C.c_int32), ("dt", C.c_double), ("lam", C.c_double),
                ("sigma", C.c_double * 4), ("sigma_v", C.c_double), ("seed", C.c_uint64),
                ("w_lim", C.c_double), ("q_near", C.c_double), ("r_near", C.c_double),
                ("Q", C.c_double * 13), ("QN", C.c_double * 13), ("R_dT", C.c_double * 4),
                ("q_l", C.c_double), ("q_c", C.c_double), ("Q_w", C.c_double * 3),
                ("r_dv", C.c_double), ("mu", C.c_double), ("v_max", C.c_double),
                ("proj_window", C.c_int32), ("flags", C.c_int32), ("n_iter", C.c_int32),
                ("ctrl_cost", C.c_double), ("input_model", C.c_int32), ("pad_", C.c_int32),
                ("rate_lim", C.c_double * 2), ("dv_lim", C.c_double * 2)]


FLAG_EXTERNAL_WORKSPACE = 1
FLAG_REGEN_AVERAGE = 2
TUNE_FORCE = 1


class mppi_problem(C.Structure):
    _fields_ = [("gates", C.POINTER(C.c_double)), ("n_gates", C.c_int32),
                ("gate_size", C.c_double), ("path", C.POINTER(C.c_double)),
                ("n_path", C.c_int32), ("path_len", C.c_double),
                ("xref", C.POINTER(C.c_double)), ("n_ref", C.c_int32), ("ref_dt", C.c_double)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class mppi_allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p)]


class mppi_info(C.Structure):
    _fields_ = [("J_min", C.c_double), ("S", C.c_double), ("ess", C.c_double),
                ("J_nom", C.c_double), ("theta0", C.c_double), ("status", C.c_int32),
                ("g0", C.c_int32), ("i0", C.c_int32), ("shift", C.c_int32),
                ("solve_index", C.c_uint32), ("rollout_waves", C.c_int32),
                ("regen_average", C.c_int32), ("rollout_draw", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class mppi_warm(C.Structure):
    _fields_ = [("warm", C.c_int32), ("g0", C.c_int32), ("solve_index", C.c_uint32),
                ("N", C.c_int32), ("allow", C.c_uint32 * MASK_WORDS), ("t_prev", C.c_double),
                ("x_prev", C.c_double * 13), ("theta0", C.c_double),
                ("U", C.c_double * (N_MAX * 4)), ("V", C.c_double * N_MAX), ("vtheta", C.c_double)]


class mppi_batch_cfg(C.Structure):
    _fields_ = [("rollout_waves", C.c_int32), ("rollout_groups", C.c_int32),
                ("sample_groups", C.c_int32), ("use_graph", C.c_int32), ("regen_average", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class mppi_tune_result(C.Structure):
    _fields_ = [("regen_average", C.c_int32), ("from_cache", C.c_int32), ("ms_stored", C.c_double),
                ("ms_regen", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class mppi_server_cfg(C.Structure):
    _fields_ = [("budget_bytes", C.c_double), ("n_slots", C.c_int32), ("max_batch", C.c_int32),
                ("use_graph", C.c_int32), ("pad_", C.c_int32)]


class mppi_result(C.Structure):
    _fields_ = [("ticket", C.c_uint64), ("drone", C.c_int32), ("status", C.c_int32),
                ("u0", C.c_double * 4), ("t_arrival", C.c_double), ("t_launch", C.c_double),
                ("t_done", C.c_double)]


class mppi_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64), ("launches", C.c_uint64),
                ("queued", C.c_int64), ("in_flight", C.c_int64), ("arena_bytes", C.c_double),
                ("peak_bytes_in_flight", C.c_double), ("rollout_steps", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_D = C.POINTER(C.c_double)
_P = C.c_void_p


def _load():
    # PyTorch ships its own HIP runtime under the same soname as ROCm's.  Load
    # it first so that this library binds to it and the process holds one HIP
    # runtime (a second one cannot open the device).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(there is no CPU fallback)")
    L = C.CDLL(LIB_PATH)
    L.mppi_create.argtypes = [C.POINTER(mppi_params), C.POINTER(mppi_quad),
                              C.POINTER(mppi_problem), _P, C.POINTER(mppi_allocator),
                              C.POINTER(_P)]
    L.mppi_create.restype = C.c_int
    L.mppi_destroy.argtypes = [_P]
    L.mppi_destroy.restype = None
    L.mppi_solve.argtypes = [_P, _D, C.c_double, _D, _D, C.POINTER(mppi_info)]
    L.mppi_solve.restype = C.c_int
    L.mppi_solve_device.argtypes = [_P, _P, _P]
    L.mppi_solve_device.restype = C.c_int
    L.mppi_solve_device_noalloc.argtypes = [_P, _P, _P]
    L.mppi_solve_device_noalloc.restype = C.c_int
    L.mppi_read_info.argtypes = [_P, C.POINTER(mppi_info)]
    L.mppi_read_info.restype = C.c_int
    L.mppi_read_samples.argtypes = [_P, _D, _D]
    L.mppi_read_samples.restype = C.c_int
    L.mppi_get_warm.argtypes = [_P, C.POINTER(mppi_warm)]
    L.mppi_get_warm.restype = C.c_int
    L.mppi_set_warm.argtypes = [_P, C.POINTER(mppi_warm)]
    L.mppi_set_warm.restype = C.c_int
    L.mppi_last_error.argtypes = [_P]
    L.mppi_last_error.restype = C.c_char_p
    L.mppi_status_string.argtypes = [C.c_int]
    L.mppi_status_string.restype = C.c_char_p
    L.mppi_plant_step.argtypes = [C.POINTER(mppi_quad), _D, _D, C.c_double, C.c_int32, _D]
    L.mppi_plant_step.restype = C.c_int
    L.mppi_plant_step_rate.argtypes = [C.POINTER(mppi_quad), _D, _D, C.c_double, C.c_int32, _D]
    L.mppi_plant_step_rate.restype = C.c_int
    L.mppi_set_profiling.argtypes = [_P, C.c_int32]
    L.mppi_set_profiling.restype = C.c_int
    L.mppi_read_profile.argtypes = [_P, _D, C.POINTER(C.c_int32)]
    L.mppi_read_profile.restype = C.c_int
    L.mppi_batch_create.argtypes = [C.POINTER(_P), C.c_int32, _P, C.POINTER(mppi_batch_cfg),
                                    C.POINTER(_P)]
    L.mppi_batch_create.restype = C.c_int
    L.mppi_batch_solve_device.argtypes = [_P, C.POINTER(C.c_int32), C.c_int32, _P, _P]
    L.mppi_batch_solve_device.restype = C.c_int
    L.mppi_batch_set_cfg.argtypes = [_P, C.POINTER(mppi_batch_cfg)]
    L.mppi_batch_set_cfg.restype = C.c_int
    L.mppi_batch_get_cfg.argtypes = [_P, C.POINTER(mppi_batch_cfg)]
    L.mppi_batch_get_cfg.restype = C.c_int
    L.mppi_batch_autotune.argtypes = [_P, _P, _P, C.c_int32, C.c_char_p, C.c_int32, C.POINTER(mppi_batch_cfg), _D,
                                      C.POINTER(C.c_int32)]
    L.mppi_autotune.argtypes = [_P, _P, C.c_int32, C.c_char_p, C.c_int32, C.POINTER(mppi_tune_result)]
    L.mppi_autotune.restype = C.c_int
    L.mppi_batch_autotune.restype = C.c_int
    L.mppi_batch_destroy.argtypes = [_P]
    L.mppi_batch_destroy.restype = None
    L.mppi_batch_last_error.argtypes = [_P]
    L.mppi_batch_last_error.restype = C.c_char_p
    L.mppi_server_create.argtypes = [C.POINTER(_P), C.c_int32, C.POINTER(mppi_server_cfg),
                                     C.POINTER(_P)]
    L.mppi_server_create.restype = C.c_int
    L.mppi_server_submit.argtypes = [_P, C.c_int32, _D, C.c_double, C.c_double,
                                     C.POINTER(C.c_uint64)]
    L.mppi_server_submit.restype = C.c_int
    L.mppi_server_progress.argtypes = [_P, C.c_double, C.POINTER(C.c_int32)]
    L.mppi_server_progress.restype = C.c_int
    L.mppi_server_poll.argtypes = [_P, C.POINTER(mppi_result), C.c_int32, C.POINTER(C.c_int32)]
    L.mppi_server_poll.restype = C.c_int
    L.mppi_server_drain.argtypes = [_P, C.c_double]
    L.mppi_server_drain.restype = C.c_int
    L.mppi_server_get_stats.argtypes = [_P, C.POINTER(mppi_server_stats)]
    L.mppi_server_get_stats.restype = C.c_int
    L.mppi_server_destroy.argtypes = [_P]
    L.mppi_server_destroy.restype = None
    L.mppi_server_last_error.argtypes = [_P]
    L.mppi_server_last_error.restype = C.c_char_p
    return L


lib = _load()


def _dp(a):
    return None if a is None else a.ctypes.data_as(_D)


def _f64(x, n=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def make_quad(q: dict) -> mppi_quad:
    s = mppi_quad()
    s.mass = q["mass"]; s.arm = q["arm"]; s.inertia[:] = list(q["inertia"]); s.c_tau = q["c_tau"]
    s.drag[:] = list(q.get("drag", (0.0, 0.0, 0.0))); s.gravity = q["gravity"]
    s.t_min = q["t_min"]; s.t_max = q["t_max"]; s.w_max = q["w_max"]
    return s


def make_params(p: dict, precision: int) -> mppi_params:
    s = mppi_params()
    s.K = p["K"]; s.N = p["N"]; s.objective = p["objective"]; s.precision = precision
    s.dt = p["dt"]; s.lam = p["lambda"]; s.sigma[:] = list(p["sigma"])
    s.sigma_v = p.get("sigma_v", 0.0); s.seed = p["seed"]
    s.w_lim = p.get("w_lim", 0.0); s.q_near = p.get("q_near", 0.0); s.r_near = p.get("r_near", 0.0)
    s.Q[:] = list(p.get("Q", [0.0] * 13)); s.QN[:] = list(p.get("QN", [0.0] * 13))
    s.R_dT[:] = list(p.get("R_dT", [0.0] * 4))
    s.q_l = p.get("q_l", 0.0); s.q_c = p.get("q_c", 0.0); s.Q_w[:] = list(p.get("Q_w", [0.0] * 3))
    s.r_dv = p.get("r_dv", 0.0); s.mu = p.get("mu", 0.0); s.v_max = p.get("v_max", 0.0)
    s.proj_window = p.get("proj_window", 64)
    s.flags = p.get("flags", 0)
    s.n_iter = p.get("n_iter", 1)
    s.ctrl_cost = p.get("ctrl_cost", 0.0)
    s.input_model = p.get("input_model", INPUT_THRUST)
    s.rate_lim[:] = list(p.get("rate_lim", (-10.0, 10.0)))
    s.dv_lim[:] = list(p.get("dv_lim", (-20.0, 20.0)))
    return s


def last_error(ctx=None) -> str:
    return lib.mppi_last_error(ctx).decode()


def _check(st: int, ctx=None):
    if st != OK:
        raise MppiError(st, f"{lib.mppi_status_string(st).decode()}: {last_error(ctx)}")


class TorchAllocator:
    """Device memory for a context from PyTorch's caching allocator."""

    def __init__(self, device: int = 0):
        import torch
        self._torch = torch
        self._device = device
        self._live = {}
        self._alloc = ALLOC_FN(self._do_alloc)
        self._free = FREE_FN(self._do_free)
        self.struct = mppi_allocator(self._alloc, self._free, None)

    def _do_alloc(self, nbytes, user):
        t = self._torch.empty(int(nbytes) + 256, dtype=self._torch.uint8,
                              device=f"cuda:{self._device}")
        ptr = t.data_ptr()
        ptr = (ptr + 255) // 256 * 256
        self._live[ptr] = t
        return ptr

    def _do_free(self, ptr, user):
        self._live.pop(int(ptr), None)


class Solver:
    """One solver context (mppi_create ... mppi_destroy)."""

    def __init__(self, quad: dict, params: dict, gates=None, path=None, path_len: float = 0.0,
                 xref=None, ref_dt: float = 0.0, precision: int = FP32, stream=None,
                 allocator: TorchAllocator | None = None):
        self.N = params["N"]
        self.K = params["K"]
        self.objective = params["objective"]
        self.nx = 17 if params.get("input_model", INPUT_THRUST) == INPUT_RATE else 13
        self._quad = make_quad(quad)
        self._prm = make_params(params, precision)
        pb = mppi_problem()
        self._keep = []
        if gates is not None:
            g = _f64(gates).reshape(-1, 4).copy(); self._keep.append(g)
            pb.gates = _dp(g); pb.n_gates = g.shape[0]; pb.gate_size = params.get("gate_size", 1.5)
        if path is not None:
            p = _f64(path).reshape(-1, 6).copy(); self._keep.append(p)
            pb.path = _dp(p); pb.n_path = p.shape[0]; pb.path_len = float(path_len)
        if xref is not None:
            r = _f64(xref).reshape(-1, 13).copy(); self._keep.append(r)
            pb.xref = _dp(r); pb.n_ref = r.shape[0]; pb.ref_dt = float(ref_dt)
        self._allocator = allocator
        ctx = _P()
        st = lib.mppi_create(C.byref(self._prm), C.byref(self._quad), C.byref(pb),
                             _P(stream) if stream else None,
                             C.byref(allocator.struct) if allocator else None, C.byref(ctx))
        _check(st, None)
        self.ctx = ctx

    def close(self):
        if getattr(self, "ctx", None):
            lib.mppi_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, x0, t_now: float = 0.0, want_U: bool = True):
        """x0: 13 states, 17 for the rate model (the thrusts last)."""
        x = _f64(x0, self.nx)
        u0 = np.zeros(4)
        U = np.zeros((self.N, 4)) if want_U else None
        info = mppi_info()
        st = lib.mppi_solve(self.ctx, _dp(x), float(t_now), _dp(u0), _dp(U), C.byref(info))
        _check(st, self.ctx)
        return u0, U, info.as_dict()

    def solve_device(self, d_req: int, d_u0: int):
        _check(lib.mppi_solve_device(self.ctx, _P(d_req), _P(d_u0)), self.ctx)

    def autotune(self, d_req: int, reps: int = 5, cache_path=None, force=False) -> dict:
        """mppi_autotune: stored or regenerating weighted average for this
        context's later solves (the warm state is restored afterwards)."""
        r = mppi_tune_result()
        path = cache_path.encode() if cache_path else None
        _check(lib.mppi_autotune(self.ctx, _P(d_req), int(reps), path, TUNE_FORCE if force else 0, C.byref(r)),
               self.ctx)
        return r.as_dict()

    def solve_device_noalloc(self, d_req: int, d_u0: int):
        """mppi_solve_device on the library's fixed per-GPU workspace."""
        _check(lib.mppi_solve_device_noalloc(self.ctx, _P(d_req), _P(d_u0)), self.ctx)

    def read_info(self):
        info = mppi_info()
        st = lib.mppi_read_info(self.ctx, C.byref(info))
        return st, info.as_dict()

    def read_samples(self, want_U: bool = False):
        J = np.zeros(self.K)
        U = np.zeros((self.N, self.K, 4)) if want_U else None
        _check(lib.mppi_read_samples(self.ctx, _dp(J), _dp(U)), self.ctx)
        return J, U

    def set_profiling(self, enable: bool = True):
        _check(lib.mppi_set_profiling(self.ctx, 1 if enable else 0), self.ctx)

    def read_profile(self):
        """Mean (sample, rollout, average) kernel durations in ms and the solve count."""
        ms = np.zeros(3)
        n = C.c_int32()
        _check(lib.mppi_read_profile(self.ctx, _dp(ms), C.byref(n)), self.ctx)
        return ms, n.value

    def get_warm(self) -> mppi_warm:
        w = mppi_warm()
        _check(lib.mppi_get_warm(self.ctx, C.byref(w)), self.ctx)
        return w

    def set_warm(self, w: mppi_warm):
        _check(lib.mppi_set_warm(self.ctx, C.byref(w)), self.ctx)


def plant_step(quad: dict, x, u, dt: float, substeps: int = 1):
    q = make_quad(quad)
    x = _f64(x, 13); u = _f64(u, 4); out = np.zeros(13)
    _check(lib.mppi_plant_step(C.byref(q), _dp(x), _dp(u), float(dt), int(substeps), _dp(out)))
    return out


def plant_step_rate(quad: dict, x, tdot, dt: float, substeps: int = 1):
    """The rate model's host plant: 17 states, thrust rates held over dt."""
    q = make_quad(quad)
    x = _f64(x, 17); u = _f64(tdot, 4); out = np.zeros(17)
    _check(lib.mppi_plant_step_rate(C.byref(q), _dp(x), _dp(u), float(dt), int(substeps), _dp(out)))
    return out


def _bcheck(st: int, b=None):
    if st != OK:
        raise MppiError(st, f"{lib.mppi_status_string(st).decode()}: {lib.mppi_batch_last_error(b).decode()}")


class Batch:
    """A batch of registered solvers stepped together (mppi_batch_*)."""

    def __init__(self, solvers, stream=None, rollout_waves=0, rollout_groups=0, sample_groups=0,
                 use_graph=True, regen_average=False):
        self.solvers = list(solvers)
        arr = (_P * len(self.solvers))(*[sv.ctx.value if hasattr(sv.ctx, "value") else sv.ctx
                                         for sv in self.solvers])
        cfg = mppi_batch_cfg(rollout_waves, rollout_groups, sample_groups, 1 if use_graph else 0,
                             1 if regen_average else 0)
        b = _P()
        _bcheck(lib.mppi_batch_create(arr, len(self.solvers), _P(stream) if stream else None,
                                      C.byref(cfg), C.byref(b)))
        self.b = b

    def solve_device(self, d_reqs: int, d_u0s: int, active=None):
        n = len(self.solvers)
        if active is None:
            _bcheck(lib.mppi_batch_solve_device(self.b, None, n, _P(d_reqs), _P(d_u0s)), self.b)
        else:
            a = (C.c_int32 * len(active))(*[int(i) for i in active])
            _bcheck(lib.mppi_batch_solve_device(self.b, a, len(active), _P(d_reqs), _P(d_u0s)), self.b)

    def set_cfg(self, rollout_waves=0, rollout_groups=0, sample_groups=0, use_graph=True, regen_average=False):
        cfg = mppi_batch_cfg(rollout_waves, rollout_groups, sample_groups, 1 if use_graph else 0,
                             1 if regen_average else 0)
        _bcheck(lib.mppi_batch_set_cfg(self.b, C.byref(cfg)), self.b)

    def get_cfg(self) -> dict:
        cfg = mppi_batch_cfg()
        _bcheck(lib.mppi_batch_get_cfg(self.b, C.byref(cfg)), self.b)
        return cfg.as_dict()

    def autotune(self, d_reqs: int, d_u0s: int, reps: int = 3, cache_path=None, force=False):
        """mppi_batch_autotune: (best launch shape, its mean step ms, whether
        it came from the cache)."""
        best = mppi_batch_cfg()
        ms = C.c_double()
        hit = C.c_int32()
        path = cache_path.encode() if cache_path else None
        _bcheck(lib.mppi_batch_autotune(self.b, _P(d_reqs), _P(d_u0s), int(reps), path,
                                        TUNE_FORCE if force else 0, C.byref(best), C.byref(ms), C.byref(hit)),
                self.b)
        return best.as_dict(), ms.value, bool(hit.value)

    def close(self):
        if getattr(self, "b", None):
            lib.mppi_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _scheck(st: int, srv=None):
    if st != OK:
        raise MppiError(st, f"{lib.mppi_status_string(st).decode()}: {lib.mppi_server_last_error(srv).decode()}")


class Server:
    """Continuous-batching server over drone contexts (mppi_server_*).  The
    solvers must be created with params["flags"] = FLAG_EXTERNAL_WORKSPACE."""

    def __init__(self, solvers, budget_bytes: float, n_slots: int = 2, max_batch: int = 0,
                 use_graph: bool = True):
        self.solvers = list(solvers)
        arr = (_P * len(self.solvers))(*[sv.ctx.value if hasattr(sv.ctx, "value") else sv.ctx
                                         for sv in self.solvers])
        cfg = mppi_server_cfg(float(budget_bytes), int(n_slots), int(max_batch), 1 if use_graph else 0, 0)
        s = _P()
        _scheck(lib.mppi_server_create(arr, len(self.solvers), C.byref(cfg), C.byref(s)))
        self.s = s
        self._buf = (mppi_result * 4096)()

    def submit(self, drone: int, x0, t_now: float, t_arrival: float) -> int:
        x = _f64(x0, self.solvers[drone].nx)
        t = C.c_uint64()
        _scheck(lib.mppi_server_submit(self.s, int(drone), _dp(x), float(t_now), float(t_arrival),
                                       C.byref(t)), self.s)
        return t.value

    def progress(self, now: float) -> int:
        n = C.c_int32()
        _scheck(lib.mppi_server_progress(self.s, float(now), C.byref(n)), self.s)
        return n.value

    def drain(self, now: float):
        _scheck(lib.mppi_server_drain(self.s, float(now)), self.s)

    def poll(self):
        out = []
        while True:
            n = C.c_int32()
            _scheck(lib.mppi_server_poll(self.s, self._buf, len(self._buf), C.byref(n)), self.s)
            for i in range(n.value):
                r = self._buf[i]
                out.append(dict(ticket=r.ticket, drone=r.drone, status=r.status, u0=list(r.u0),
                                t_arrival=r.t_arrival, t_launch=r.t_launch, t_done=r.t_done))
            if n.value < len(self._buf):
                return out

    def stats(self) -> dict:
        st = mppi_server_stats()
        _scheck(lib.mppi_server_get_stats(self.s, C.byref(st)), self.s)
        return st.as_dict()

    def close(self):
        if getattr(self, "s", None):
            lib.mppi_server_destroy(self.s)
            self.s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
