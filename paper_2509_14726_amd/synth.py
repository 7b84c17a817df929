"""Seeded synthetic inputs for the MPPI step (tracks, paths, references, params).

This module holds no arithmetic of the method itself: it only produces the
inputs that Alg. 1 of the paper takes (waypoints W, arc-length path P_arc,
time-parameterised reference tau_ref) and the parameter sets of the
workloads.  Both the device path and the oracle consume what it returns.

The paper's tracks (Circle, Figure-8, Split-S; Sec. V-A) have no published
layouts, so seeded random tracks with the same gate size stand in for them.
"""
from __future__ import annotations

import math

import numpy as np

# Quadrotor of the single-solve workload: 0.85 kg, 0.15 m arm, inertia
# diag(1e-3, 1e-3, 1.7e-3), four rotors with thrust in [0, 7] N.  The yaw
# torque coefficient and the drag matrix are not given by the paper
# (Sec. III-A names them only); 0.01 m and zero are this project's values.
# The body-rate bound 10 rad/s is the one of Table I.
QUAD = dict(mass=0.85, arm=0.15, inertia=(1e-3, 1e-3, 1.7e-3), c_tau=0.01,
            drag=(0.0, 0.0, 0.0), gravity=9.81, t_min=0.0, t_max=7.0, w_max=10.0)

OBJ_GATE, OBJ_CONTOUR, OBJ_TRACK = 0, 1, 2
OBJECTIVES = {"gate": OBJ_GATE, "contour": OBJ_CONTOUR, "track": OBJ_TRACK}

# MPPI parameters shared by every workload: dt 0.02 s, lambda 1, 1 N noise per
# rotor.  The cost weights are not printed in the paper; these are this
# project's choices (they change behaviour, not parity).
BASE = dict(dt=0.02, **{"lambda": 1.0}, sigma=(1.0, 1.0, 1.0, 1.0), sigma_v=2.0, w_lim=100.0,
            q_near=5.0, r_near=1.0, gate_size=1.5,
            Q=(100.0, 100.0, 100.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 0.1, 0.1, 0.1),
            QN=(100.0, 100.0, 100.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 0.1, 0.1, 0.1),
            R_dT=(1e-5, 1e-5, 1e-5, 1e-5),
            q_l=100.0, q_c=100.0, Q_w=(0.1, 0.1, 0.1), r_dv=1e-4, mu=10.0, v_max=25.0,
            proj_window=64)


def params(K: int, N: int, objective: str = "gate", seed: int = 1, **over) -> dict:
    p = dict(BASE)
    p.update(K=int(K), N=int(N), objective=OBJECTIVES[objective], seed=int(seed))
    p.update(over)
    return p


def hover_thrust(quad: dict = QUAD) -> float:
    return quad["mass"] * quad["gravity"] / 4.0


# --------------------------------------------------------------------------
# tracks

def random_track(seed: int, n_gates: int = 7, box=(30.0, 30.0, 5.0), z0: float = 1.0,
                 min_sep: float = 3.0) -> np.ndarray:
    """G x 4 gates (cx, cy, cz, yaw): centres uniform in a box_x x box_y x box_z
    slab lifted by z0, pairwise at least min_sep apart, yaw uniform in [-pi, pi]."""
    rng = np.random.default_rng(seed)
    gates = []
    while len(gates) < n_gates:
        c = np.array([rng.uniform(-box[0] / 2, box[0] / 2), rng.uniform(-box[1] / 2, box[1] / 2),
                      z0 + rng.uniform(0.0, box[2])])
        if all(np.linalg.norm(c - g[:3]) >= min_sep for g in gates):
            gates.append(np.array([c[0], c[1], c[2], rng.uniform(-math.pi, math.pi)]))
    return np.array(gates)


def loop_track(seed: int, n_gates: int = 7, radius=(9.0, 14.0), height=(1.5, 4.0)) -> np.ndarray:
    """G x 4 gates of a closed circuit: centres at jittered angles around the
    origin (radius and height uniform in the given ranges), each gate facing
    along the closed spline through the centres, so that flying the spline
    passes every gate front to back."""
    rng = np.random.default_rng(seed)
    step = 2.0 * math.pi / n_gates
    ang = np.arange(n_gates) * step + rng.uniform(-0.25 * step, 0.25 * step, n_gates)
    r = rng.uniform(radius[0], radius[1], n_gates)
    c = np.column_stack([r * np.cos(ang), r * np.sin(ang), rng.uniform(height[0], height[1], n_gates)])
    sp, _ = _periodic_spline(c)
    d = sp(sp.x[:-1], 1)
    return np.column_stack([c, np.arctan2(d[:, 1], d[:, 0])])


def start_state(gates: np.ndarray, back: float = 2.0) -> np.ndarray:
    """Hover `back` metres in front of gate 0, facing through it."""
    c, yaw = gates[0, :3], gates[0, 3]
    n = np.array([math.cos(yaw), math.sin(yaw), 0.0])
    x = np.zeros(13)
    x[0:3] = c - back * n
    x[6] = math.cos(yaw / 2.0)
    x[9] = math.sin(yaw / 2.0)
    return x


# --------------------------------------------------------------------------
# arc-length path through the gate centres (contouring input)

def _periodic_spline(points: np.ndarray):
    from scipy.interpolate import CubicSpline
    pts = np.vstack([points, points[:1]])
    chord = np.linalg.norm(np.diff(pts, axis=0), axis=1)
    u = np.concatenate([[0.0], np.cumsum(chord)])
    return CubicSpline(u, pts, bc_type="periodic"), u[-1]


def path_table(gates: np.ndarray, n_points: int = 2000, dense: int = 200000):
    """Closed cubic spline (chord-length knots) through the gate centres,
    resampled at n_points points uniform in arc length.  Returns (table P x 6
    = position and unit tangent, total length L)."""
    sp, umax = _periodic_spline(gates[:, :3])
    uu = np.linspace(0.0, umax, dense + 1)
    d = sp(uu, 1)
    speed = np.linalg.norm(d, axis=1)
    s = np.concatenate([[0.0], np.cumsum(0.5 * (speed[1:] + speed[:-1]) * np.diff(uu))])
    L = float(s[-1])
    s_target = np.arange(n_points) * (L / n_points)
    u_target = np.interp(s_target, s, uu)
    pos = sp(u_target)
    tan = sp(u_target, 1)
    tan /= np.linalg.norm(tan, axis=1, keepdims=True)
    return np.hstack([pos, tan]), L


def reference_table(gates: np.ndarray, speed: float = 5.0, dt: float = 0.02, n_rows: int = 1101,
                    gravity: float = 9.81) -> np.ndarray:
    """Full-state reference sampled every dt along the spline at constant
    speed: p = path(speed t), v = speed * tangent, attitude from the thrust
    direction a + g e_z with yaw along the tangent, zero body rates."""
    from scipy.spatial.transform import Rotation
    sp, umax = _periodic_spline(gates[:, :3])
    dense = 200000
    uu = np.linspace(0.0, umax, dense + 1)
    d1 = sp(uu, 1)
    sp_len = np.linalg.norm(d1, axis=1)
    s = np.concatenate([[0.0], np.cumsum(0.5 * (sp_len[1:] + sp_len[:-1]) * np.diff(uu))])
    L = s[-1]
    sr = (speed * np.arange(n_rows) * dt) % L
    u = np.interp(sr, s, uu)
    p = sp(u)
    du = sp(u, 1)
    ddu = sp(u, 2)
    nd = np.linalg.norm(du, axis=1, keepdims=True)
    t = du / nd
    # d^2 p / ds^2 = (ddu - (t . ddu) t) / |du|^2
    kappa = (ddu - np.sum(t * ddu, axis=1, keepdims=True) * t) / (nd * nd)
    zb = speed * speed * kappa + np.array([0.0, 0.0, gravity])
    zb /= np.linalg.norm(zb, axis=1, keepdims=True)
    yaw = np.arctan2(t[:, 1], t[:, 0])
    xc = np.column_stack([np.cos(yaw), np.sin(yaw), np.zeros(n_rows)])
    yb = np.cross(zb, xc)
    yb /= np.linalg.norm(yb, axis=1, keepdims=True)
    xb = np.cross(yb, zb)
    R = np.stack([xb, yb, zb], axis=2)            # columns are the body axes
    qxyzw = Rotation.from_matrix(R).as_quat()      # (x, y, z, w)
    q = np.column_stack([qxyzw[:, 3], qxyzw[:, 0], qxyzw[:, 1], qxyzw[:, 2]])
    q *= np.where(q[:, :1] < 0.0, -1.0, 1.0)
    out = np.zeros((n_rows, 13))
    out[:, 0:3] = p
    out[:, 3:6] = speed * t
    out[:, 6:10] = q
    return out


# --------------------------------------------------------------------------
# workloads

def single_solve_workload(K: int = 1024, N: int = 50, seed: int = 1, track_seed: int = 1,
                          n_gates: int = 7, objective: str = "gate", dt: float = 0.02,
                          **over) -> dict:
    """A single MPPI solve on a seeded track.  Contouring gets the 2000-point
    arc-length table of the spline through the gate centres, tracking the 5 m/s
    full-state reference on the same spline."""
    gates = random_track(track_seed, n_gates)
    prm = params(K, N, objective, seed, dt=dt, **over)
    w = dict(quad=dict(QUAD), params=prm, gates=gates, x0=start_state(gates))
    if objective == "contour":
        path, L = path_table(gates)
        w.update(path=path, path_len=L)
    if objective == "track":
        w.update(xref=reference_table(gates, dt=dt, n_rows=1000 + N + 1), ref_dt=dt)
    return w


def race_workload(K: int = 8192, N: int = 20, objective: str = "gate", seed: int = 1, track_seed: int = 1,
                  n_gates: int = 7, dt: float = 0.03, steps: int = 1000, **over) -> dict:
    """A closed-loop race on a seeded circuit (`loop_track`): the solver's
    parameters, the start 2 m in front of gate 0, and for contouring and
    tracking the path table and the 5 m/s reference of the same circuit
    (rows for `steps` control steps plus a horizon)."""
    gates = loop_track(track_seed, n_gates)
    prm = params(K, N, objective, seed, dt=dt, **over)
    w = dict(quad=dict(QUAD), params=prm, gates=gates, x0=start_state(gates))
    if objective == "contour":
        path, L = path_table(gates)
        w.update(path=path, path_len=L)
    if objective == "track":
        w.update(xref=reference_table(gates, dt=dt, n_rows=steps + N + 1), ref_dt=dt)
    return w


def batch_instances(n: int = 256, seed: int = 3):
    """Uneven instances: K from {1024..16384}, N uniform in [30, 150], 5..12
    gates, each on its own seeded track."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        K = int(rng.choice([1024, 2048, 4096, 8192, 16384]))
        N = int(rng.integers(30, 151))
        G = int(rng.integers(5, 13))
        out.append(dict(K=K, N=N, n_gates=G, track_seed=3000 + i, seed=3000 + i))
    return out
