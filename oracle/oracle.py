"""ctypes binding of the FP64 CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  The product library never calls it.  Parity status of
each exported function (what pins it) is documented in the test files under
tests/ that start with ``test_oracle``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIBRARY names another build of the oracle (the host-sanitizer build);
# by default the in-tree one.
BUILD_PATH = os.path.join(HERE, "liborc.so")
LIB_PATH = os.environ.get("ORACLE_LIBRARY") or BUILD_PATH
SRC = os.path.join(HERE, "mppi_oracle.c")
COUNT_LIB_PATH = os.path.join(HERE, "liborc_count.so")
COUNT_SRC = os.path.join(HERE, "opcount.cpp")

NMAX = 256
MASK_WORDS = 9
OBJ_GATE, OBJ_CONTOUR, OBJ_TRACK = 0, 1, 2
INPUT_THRUST, INPUT_RATE = 0, 1
OK, EINVAL, ENONFINITE = 0, -1, -4


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C99, no fast-math, no FMA contraction),
    and its op-counting build (the same source as C++ with binary64 counted)."""
    if force or not os.path.exists(BUILD_PATH):
        tmp = BUILD_PATH + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-std=c99", "-Wall", "-fPIC", "-shared", "-fopenmp",
            "-ffp-contract=off", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, BUILD_PATH)
    if force or not os.path.exists(COUNT_LIB_PATH):
        tmp = COUNT_LIB_PATH + ".tmp"
        subprocess.check_call([
            "g++", "-O2", "-std=c++17", "-Wall", "-Wno-unknown-pragmas", "-Wno-unused-variable",
            "-fPIC", "-shared", "-ffp-contract=off", "-o", tmp, COUNT_SRC, "-lm"])
        os.replace(tmp, COUNT_LIB_PATH)
    return BUILD_PATH


class Quad(C.Structure):
    _fields_ = [("mass", C.c_double), ("arm", C.c_double), ("inertia", C.c_double * 3),
                ("c_tau", C.c_double), ("drag", C.c_double * 3), ("gravity", C.c_double),
                ("t_min", C.c_double), ("t_max", C.c_double), ("w_max", C.c_double)]


class Cfg(C.Structure):
    _fields_ = [("K", C.c_int32), ("N", C.c_int32), ("objective", C.c_int32),
                ("n_threads", C.c_int32),
                ("dt", C.c_double), ("lam", C.c_double), ("sigma", C.c_double * 4),
                ("sigma_v", C.c_double), ("seed", C.c_uint64),
                ("w_lim", C.c_double),
                ("q_near", C.c_double), ("r_near", C.c_double), ("eps_dec", C.c_double),
                ("Q", C.c_double * 13), ("QN", C.c_double * 13), ("R_dT", C.c_double * 4),
                ("q_l", C.c_double), ("q_c", C.c_double), ("Q_w", C.c_double * 3),
                ("r_dv", C.c_double), ("mu", C.c_double), ("v_max", C.c_double),
                ("gates", C.POINTER(C.c_double)), ("n_gates", C.c_int32), ("gate_size", C.c_double),
                ("path", C.POINTER(C.c_double)), ("n_path", C.c_int32), ("path_len", C.c_double),
                ("xref", C.POINTER(C.c_double)), ("n_ref", C.c_int32), ("ref_dt", C.c_double),
                ("proj_window", C.c_int32), ("n_iter", C.c_int32), ("ctrl_cost", C.c_double),
                ("input_model", C.c_int32), ("pad3_", C.c_int32), ("rate_lim", C.c_double * 2),
                ("dv_lim", C.c_double * 2)]


class Warm(C.Structure):
    _fields_ = [("warm", C.c_int32), ("g0", C.c_int32), ("s", C.c_uint32), ("pad_", C.c_int32),
                ("allow", C.c_uint32 * MASK_WORDS), ("t_prev", C.c_double),
                ("x_prev", C.c_double * 13), ("theta0", C.c_double),
                ("U", C.c_double * (NMAX * 4)), ("V", C.c_double * NMAX), ("vtheta", C.c_double)]


class Out(C.Structure):
    _fields_ = [("J", C.POINTER(C.c_double)), ("w", C.POINTER(C.c_double)),
                ("U", C.POINTER(C.c_double)), ("V", C.POINTER(C.c_double)),
                ("margin", C.POINTER(C.c_double)), ("Ustar", C.POINTER(C.c_double)),
                ("Vstar", C.POINTER(C.c_double)),
                ("J_min", C.c_double), ("S", C.c_double), ("ess", C.c_double),
                ("J_nom", C.c_double), ("theta0", C.c_double),
                ("g0", C.c_int32), ("i0", C.c_int32), ("shift", C.c_int32), ("n_amb", C.c_int32),
                ("status", C.c_int32), ("pad_", C.c_int32),
                ("allow", C.c_uint32 * MASK_WORDS), ("front", C.c_uint32 * MASK_WORDS),
                ("front_amb", C.c_uint32 * MASK_WORDS), ("absJ", C.POINTER(C.c_double)),
                ("absJ_nom", C.c_double), ("n_amb_earlier", C.c_int32), ("pad2_", C.c_int32)]


_D = C.POINTER(C.c_double)
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                        C.POINTER(C.c_uint32)]
        L.orc_u01.argtypes = [C.c_uint32]
        L.orc_u01.restype = C.c_double
        L.orc_normals.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, _D]
        L.orc_f.argtypes = [C.POINTER(Quad), _D, _D, _D]
        L.orc_rk4.argtypes = [C.POINTER(Quad), _D, _D, C.c_double, _D]
        L.orc_f_rate.argtypes = [C.POINTER(Quad), _D, _D, _D]
        L.orc_rk4_rate.argtypes = [C.POINTER(Quad), _D, _D, C.c_double, _D]
        L.orc_sample_rate.argtypes = [C.POINTER(Cfg), C.POINTER(Quad), _D, _D, C.c_uint32, C.c_uint32,
                                      C.c_int, _D, C.c_double, _D, _D]
        L.orc_gate_cross.argtypes = [_D, _D, _D, C.c_double, _D]
        L.orc_gate_cross.restype = C.c_int
        L.orc_project.argtypes = [C.POINTER(Cfg), _D, C.c_double, C.c_int]
        L.orc_project.restype = C.c_double
        L.orc_sample.argtypes = [C.POINTER(Cfg), C.POINTER(Quad), _D, _D, C.c_uint32, C.c_uint32,
                                 _D, _D]
        L.orc_rollout_cost.argtypes = [C.POINTER(Cfg), C.POINTER(Quad), _D, _D, _D, C.c_int32,
                                       C.POINTER(C.c_uint32), _D, C.c_double, C.c_double,
                                       C.c_int32, _D, C.POINTER(C.c_uint32),
                                       C.POINTER(C.c_uint32)]
        L.orc_rollout_cost.restype = C.c_double
        L.orc_solve.argtypes = [C.POINTER(Quad), C.POINTER(Cfg), C.POINTER(Warm), _D, C.c_double,
                                _D, C.POINTER(C.c_uint8), C.POINTER(Out)]
        L.orc_solve.restype = C.c_int
        L.orc_warm_init.argtypes = [C.POINTER(Warm), C.c_int32]
        _lib = L
    return _lib


_count_lib = None


def count_lib():
    """The op-counting build: the oracle's functions plus orc_ops_reset /
    orc_ops_read (add, mul, div, sqrt, transcendental, other)."""
    global _count_lib
    if _count_lib is None:
        if not os.path.exists(COUNT_LIB_PATH):
            build(force=False)
        L = C.CDLL(COUNT_LIB_PATH)
        L.orc_ops_reset.argtypes = []
        L.orc_ops_read.argtypes = [C.POINTER(C.c_int64)]
        L.orc_normals.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, _D]
        L.orc_f.argtypes = [C.POINTER(Quad), _D, _D, _D]
        L.orc_rk4.argtypes = [C.POINTER(Quad), _D, _D, C.c_double, _D]
        L.orc_sample.argtypes = [C.POINTER(Cfg), C.POINTER(Quad), _D, _D, C.c_uint32, C.c_uint32, _D, _D]
        L.orc_rollout_cost.argtypes = [C.POINTER(Cfg), C.POINTER(Quad), _D, _D, _D, C.c_int32,
                                       C.POINTER(C.c_uint32), _D, C.c_double, C.c_double,
                                       C.c_int32, _D, C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        L.orc_rollout_cost.restype = C.c_double
        _count_lib = L
    return _count_lib


OP_CLASSES = ("add", "mul", "div", "sqrt", "trans", "other")


def counted(call) -> dict:
    """Run call(count_lib()) and return the operations it counted."""
    L = count_lib()
    L.orc_ops_reset()
    call(L)
    out = (C.c_int64 * 6)()
    L.orc_ops_read(out)
    return {k: int(v) for k, v in zip(OP_CLASSES, out)}


def flops(ops: dict) -> int:
    """Floating-point operations of a count: additions, multiplications,
    divisions and square roots (transcendentals are counted apart)."""
    return ops["add"] + ops["mul"] + ops["div"] + ops["sqrt"]


def _dp(a):
    return a.ctypes.data_as(_D) if a is not None else None


def _arr(x, n=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if n is not None:
        assert a.size == n, (a.size, n)
    return a


# --------------------------------------------------------------------------
# thin wrappers over the building blocks

def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xffffffff for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xffffffff for v in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def u01(word):
    return lib().orc_u01(int(word) & 0xffffffff)


def normals(seed, m, k, s, ch=0):
    z = np.zeros(4)
    lib().orc_normals(int(seed), int(m), int(k), int(s), int(ch), _dp(z))
    return z


def make_quad(p: dict) -> Quad:
    q = Quad()
    q.mass = p["mass"]; q.arm = p["arm"]
    q.inertia[:] = list(p["inertia"])
    q.c_tau = p["c_tau"]
    q.drag[:] = list(p.get("drag", (0.0, 0.0, 0.0)))
    q.gravity = p["gravity"]; q.t_min = p["t_min"]; q.t_max = p["t_max"]; q.w_max = p["w_max"]
    return q


def f(quad: dict, x, T):
    x = _arr(x, 13); T = _arr(T, 4); xd = np.zeros(13)
    q = make_quad(quad)
    lib().orc_f(C.byref(q), _dp(x), _dp(T), _dp(xd))
    return xd


def rk4(quad: dict, x, T, dt):
    x = _arr(x, 13); T = _arr(T, 4); xn = np.zeros(13)
    q = make_quad(quad)
    lib().orc_rk4(C.byref(q), _dp(x), _dp(T), float(dt), _dp(xn))
    return xn


def rk4_rate(quad: dict, x, Tdot, dt):
    """One RK4 step of the paper's 17-state model (thrusts last), rate held."""
    x = _arr(x, 17); Td = _arr(Tdot, 4); xn = np.zeros(17)
    q = make_quad(quad)
    lib().orc_rk4_rate(C.byref(q), _dp(x), _dp(Td), float(dt), _dp(xn))
    return xn


def gate_cross(pa, pb, gate, size):
    pa = _arr(pa, 3); pb = _arr(pb, 3); g = _arr(gate, 4); m = np.zeros(1)
    r = lib().orc_gate_cross(_dp(pa), _dp(pb), _dp(g), float(size), _dp(m))
    return bool(r), float(m[0])


class Problem:
    """Owns the ctypes config plus the numpy buffers it points into."""

    def __init__(self, quad: dict, prm: dict, gates=None, path=None, path_len=0.0,
                 xref=None, ref_dt=0.0):
        self.quad_d = quad
        self.quad = make_quad(quad)
        self.prm = prm
        c = Cfg()
        c.K = prm["K"]; c.N = prm["N"]; c.objective = prm["objective"]
        c.n_threads = prm.get("n_threads", 1)
        c.dt = prm["dt"]; c.lam = prm["lambda"]
        c.sigma[:] = list(prm["sigma"])
        c.sigma_v = prm.get("sigma_v", 0.0)
        c.seed = prm["seed"]
        c.w_lim = prm.get("w_lim", 0.0)
        c.q_near = prm.get("q_near", 0.0); c.r_near = prm.get("r_near", 0.0)
        c.eps_dec = prm.get("eps_dec", 0.0)
        c.Q[:] = list(prm.get("Q", [0.0] * 13)); c.QN[:] = list(prm.get("QN", [0.0] * 13))
        c.R_dT[:] = list(prm.get("R_dT", [0.0] * 4))
        c.q_l = prm.get("q_l", 0.0); c.q_c = prm.get("q_c", 0.0)
        c.Q_w[:] = list(prm.get("Q_w", [0.0] * 3))
        c.r_dv = prm.get("r_dv", 0.0); c.mu = prm.get("mu", 0.0); c.v_max = prm.get("v_max", 0.0)
        c.proj_window = prm.get("proj_window", 64)
        c.n_iter = prm.get("n_iter", 1)
        c.ctrl_cost = prm.get("ctrl_cost", 0.0)
        c.input_model = prm.get("input_model", INPUT_THRUST)
        c.rate_lim[:] = list(prm.get("rate_lim", (-10.0, 10.0)))
        c.dv_lim[:] = list(prm.get("dv_lim", (-20.0, 20.0)))
        self.nx = 17 if c.input_model == INPUT_RATE else 13
        self.gates = None if gates is None else _arr(gates).reshape(-1, 4).copy()
        self.path = None if path is None else _arr(path).reshape(-1, 6).copy()
        self.xref = None if xref is None else _arr(xref).reshape(-1, 13).copy()
        if self.gates is not None:
            c.gates = _dp(self.gates); c.n_gates = self.gates.shape[0]
            c.gate_size = prm.get("gate_size", 1.5)
        if self.path is not None:
            c.path = _dp(self.path); c.n_path = self.path.shape[0]; c.path_len = float(path_len)
        if self.xref is not None:
            c.xref = _dp(self.xref); c.n_ref = self.xref.shape[0]; c.ref_dt = float(ref_dt)
        self.cfg = c

    def warm(self, g0: int = 0) -> Warm:
        w = Warm()
        lib().orc_warm_init(C.byref(w), int(g0))
        return w

    def project(self, p, theta_prev=0.0, global_search=True):
        p = _arr(p, 3)
        return lib().orc_project(C.byref(self.cfg), _dp(p), float(theta_prev), int(global_search))

    def sample_rate(self, Ustar, Vstar, m, s, T0, v0=0.0, noisy=True):
        """Rate-model samples (clipped rates) of sample m from thrusts T0."""
        N = self.cfg.N
        Us = _arr(Ustar, 4 * N); Vs = _arr(Vstar, N); T0 = _arr(T0, 4)
        U = np.zeros(4 * N); V = np.zeros(N)
        lib().orc_sample_rate(C.byref(self.cfg), C.byref(self.quad), _dp(Us), _dp(Vs), int(m), int(s),
                              1 if noisy else 0, _dp(T0), float(v0), _dp(U), _dp(V))
        return U.reshape(N, 4), V

    def sample(self, Ustar, Vstar, m, s):
        N = self.cfg.N
        Us = _arr(Ustar, 4 * N); Vs = _arr(Vstar, N)
        U = np.zeros(4 * N); V = np.zeros(N)
        lib().orc_sample(C.byref(self.cfg), C.byref(self.quad), _dp(Us), _dp(Vs), int(m), int(s),
                         _dp(U), _dp(V))
        return U.reshape(N, 4), V

    def rollout_cost(self, x0, U, V=None, g0=0, allow=None, u_prev=None, v_prev=0.0, theta0=0.0,
                     i0=0, nominal=False):
        N = self.cfg.N
        x0 = _arr(x0, self.nx); U = _arr(U, 4 * N)
        V = _arr(np.zeros(N) if V is None else V, N)
        if allow is None:
            allow = [0xffffffff] * MASK_WORDS
        al = (C.c_uint32 * MASK_WORDS)(*allow)
        up = _arr(np.full(4, self.quad_d["mass"] * self.quad_d["gravity"] / 4.0)
                  if u_prev is None else u_prev, 4)
        mg = np.zeros(1)
        fr = (C.c_uint32 * MASK_WORDS)() if nominal else None
        fa = (C.c_uint32 * MASK_WORDS)() if nominal else None
        J = lib().orc_rollout_cost(C.byref(self.cfg), C.byref(self.quad), _dp(x0), _dp(U), _dp(V),
                                   int(g0), al, _dp(up), float(v_prev), float(theta0), int(i0),
                                   _dp(mg), fr, fa)
        if nominal:
            return J, float(mg[0]), list(fr), list(fa)
        return J, float(mg[0])

    def rollout_step_ops(self, x0, n_samples: int = 64, s: int = 0) -> dict:
        """Operations per rollout step of a cold solve from x0 (nominal at
        hover thrust), counted by the op-counting build over samples
        0..n_samples-1: 'sample' (Eq. (3): normals, perturbation, clipping)
        and 'rollout' (Eq. (2) integrated with the objective's cost), each the
        mean count per sample and step, plus their flops."""
        N = self.cfg.N
        hover = self.quad_d["mass"] * self.quad_d["gravity"] / 4.0
        Us = np.full(4 * N, hover)
        Vs = np.zeros(N)
        x0 = _arr(x0, 13)
        theta0 = self.project(x0[:3]) if self.cfg.objective == OBJ_CONTOUR else 0.0
        al = (C.c_uint32 * MASK_WORDS)(*([0xffffffff] * MASK_WORDS))
        up = np.full(4, hover)
        samples = []
        for m in range(n_samples):
            U = np.zeros(4 * N)
            V = np.zeros(N)
            samples.append((U, V))

        def do_sample(L):
            for m, (U, V) in enumerate(samples):
                L.orc_sample(C.byref(self.cfg), C.byref(self.quad), _dp(Us), _dp(Vs), m, s, _dp(U), _dp(V))

        def do_rollout(L):
            for U, V in samples:
                L.orc_rollout_cost(C.byref(self.cfg), C.byref(self.quad), _dp(x0), _dp(U), _dp(V), 0, al,
                                   _dp(up), 0.0, float(theta0), 0, None, None, None)

        per = float(n_samples * N)
        out = {}
        for name, fn in (("sample", do_sample), ("rollout", do_rollout)):
            ops = counted(fn)
            d = {k: v / per for k, v in ops.items()}
            d["flops"] = flops(ops) / per
            out[name] = d
        out["flops_per_step"] = out["sample"]["flops"] + out["rollout"]["flops"]
        return out

    def solve(self, warm: Warm, x0, t_now=0.0, J_rep=None, rep_mask=None):
        """One MPPI step; returns a dict of outputs.  warm is updated in place."""
        K, N = self.cfg.K, self.cfg.N
        J = np.zeros(K); w = np.zeros(K); U = np.zeros(4 * N); V = np.zeros(N)
        mg = np.zeros(K); Us = np.zeros(4 * N); Vs = np.zeros(N)
        o = Out()
        A = np.zeros(K)
        o.J = _dp(J); o.w = _dp(w); o.U = _dp(U); o.V = _dp(V); o.margin = _dp(mg); o.absJ = _dp(A)
        o.Ustar = _dp(Us); o.Vstar = _dp(Vs)
        x0 = _arr(x0, self.nx)
        jr = _arr(J_rep, K) if J_rep is not None else None
        rm = (np.ascontiguousarray(np.asarray(rep_mask, dtype=np.uint8))
              if rep_mask is not None else None)
        st = lib().orc_solve(C.byref(self.quad), C.byref(self.cfg), C.byref(warm), _dp(x0),
                             float(t_now), _dp(jr),
                             rm.ctypes.data_as(C.POINTER(C.c_uint8)) if rm is not None else None,
                             C.byref(o))
        return dict(status=st, J=J, w=w, U=U.reshape(N, 4), V=V, margin=mg, absJ=A,
                    Ustar=Us.reshape(N, 4), Vstar=Vs, J_min=o.J_min, S=o.S, ess=o.ess,
                    J_nom=o.J_nom, absJ_nom=o.absJ_nom, theta0=o.theta0, g0=o.g0, i0=o.i0, shift=o.shift,
                    n_amb=o.n_amb, n_amb_earlier=o.n_amb_earlier, allow=list(o.allow), front=list(o.front),
                    front_amb=list(o.front_amb))


def mask_bits(words, n):
    """Unpack the first n bits of a little-endian word mask into a bool array."""
    return np.array([(words[j >> 5] >> (j & 31)) & 1 for j in range(n)], dtype=bool)
