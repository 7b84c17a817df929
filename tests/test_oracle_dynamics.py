"""Pins of the oracle's dynamics f(x, u) and RK4 step (Sec. III-A, Eq. (2)).

Every expected value here comes from a closed form of rigid-body motion, not
from the oracle's own formulas: free fall and hover, a tilted hovering thrust,
a constant yaw spin, a constant yaw torque, the torque map of the X layout,
conservation laws of the torque-free body, and drag in a rotated frame.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_14726_amd.synth import QUAD

G = QUAD["gravity"]
M = QUAD["mass"]
HOVER = M * G / 4.0


def state(p=(0, 0, 0), v=(0, 0, 0), q=(1, 0, 0, 0), w=(0, 0, 0)):
    return np.array(list(p) + list(v) + list(q) + list(w), dtype=float)


def roll(x, T, dt, n, quad=QUAD):
    for _ in range(n):
        x = O.rk4(quad, x, T, dt)
    return x


def test_free_fall_polynomial_exact():
    # zero thrust, no rotation: p(t) = p0 + v0 t - g t^2/2 e_z (RK4 is exact
    # for this quadratic), attitude arbitrary
    q = np.array([0.9, 0.1, -0.3, 0.2]); q /= np.linalg.norm(q)
    x0 = state(p=(1.0, -2.0, 3.0), v=(0.5, 0.25, 4.0), q=q)
    dt, n = 0.02, 100
    x = roll(x0, np.zeros(4), dt, n)
    t = dt * n
    np.testing.assert_allclose(x[0:3], [1.0 + 0.5 * t, -2.0 + 0.25 * t, 3.0 + 4.0 * t - 0.5 * G * t * t],
                               atol=1e-12)
    np.testing.assert_allclose(x[3:6], [0.5, 0.25, 4.0 - G * t], atol=1e-12)
    np.testing.assert_allclose(x[6:10], q, atol=1e-15)


def test_hover_is_stationary():
    x0 = state(p=(3.0, 4.0, 5.0))
    x = roll(x0, np.full(4, HOVER), 0.02, 200)
    np.testing.assert_allclose(x, x0, atol=1e-12)


def test_tilted_thrust_single_evaluation():
    # body rolled by phi about x: thrust axis (0, -sin phi, cos phi).  With
    # collective thrust m g / cos phi the vertical acceleration vanishes and
    # the lateral one is -g tan phi.
    phi = 0.3
    x = state(q=(math.cos(phi / 2), math.sin(phi / 2), 0, 0))
    F = M * G / math.cos(phi)
    xd = O.f(QUAD, x, np.full(4, F / 4))
    np.testing.assert_allclose(xd[3:6], [0.0, -G * math.tan(phi), 0.0], atol=1e-12)
    # pitch about y: thrust axis (sin th, 0, cos th)
    th = -0.4
    x = state(q=(math.cos(th / 2), 0, math.sin(th / 2), 0))
    xd = O.f(QUAD, x, np.full(4, M * G / math.cos(th) / 4))
    np.testing.assert_allclose(xd[3:6], [G * math.tan(th), 0.0, 0.0], atol=1e-12)


def test_yaw_spin_matches_rotation():
    # w = (0, 0, wz), uniform thrust: no torque, J_x = J_y so w stays constant,
    # q(t) = (cos(wz t / 2), 0, 0, sin(wz t / 2)), position hovers
    wz, dt, n = 3.0, 0.02, 100
    x = roll(state(p=(1, 1, 1), w=(0, 0, wz)), np.full(4, HOVER), dt, n)
    t = dt * n
    np.testing.assert_allclose(x[10:13], [0, 0, wz], atol=1e-12)
    # q' = A q has eigenvalues +-i wz/2; RK4's phase error per step is
    # (wz dt / 2)^5 / 120, accumulated over n steps (2e-8 here)
    bound = 2.0 * n * (wz * dt / 2) ** 5 / 120.0
    np.testing.assert_allclose(x[6:10], [math.cos(wz * t / 2), 0, 0, math.sin(wz * t / 2)],
                               atol=bound)
    np.testing.assert_allclose(x[0:6], [1, 1, 1, 0, 0, 0], atol=1e-12)


def test_roll_spin_sign():
    # positive body-x rate rolls the thrust axis toward -y
    wx, dt, n = 1.0, 0.01, 50
    x = roll(state(w=(wx, 0, 0)), np.full(4, HOVER), dt, n)
    ang = wx * dt * n
    np.testing.assert_allclose(x[6:10], [math.cos(ang / 2), math.sin(ang / 2), 0, 0], atol=1e-10)


def test_constant_yaw_torque():
    # T = (a+d, a-d, a+d, a-d): tau = (0, 0, 4 c_tau d); w_z = 4 c_tau d t / J_z
    # exactly (linear in t), yaw angle psi = 2 c_tau d t^2 / J_z
    a, d, dt, n = HOVER, 0.01, 0.01, 100
    T = np.array([a + d, a - d, a + d, a - d])
    x = roll(state(), T, dt, n)
    t = dt * n
    Jz = QUAD["inertia"][2]
    wz = 4 * QUAD["c_tau"] * d * t / Jz
    np.testing.assert_allclose(x[10:13], [0, 0, wz], atol=1e-12)
    psi = 2 * QUAD["c_tau"] * d * t * t / Jz
    np.testing.assert_allclose(x[6:10], [math.cos(psi / 2), 0, 0, math.sin(psi / 2)], atol=1e-8)
    np.testing.assert_allclose(x[0:6], np.zeros(6), atol=1e-12)


@pytest.mark.parametrize("rotor,sign", [(0, (1, -1, 1)), (1, (1, 1, -1)), (2, (-1, 1, 1)),
                                        (3, (-1, -1, -1))])
def test_torque_map_of_x_layout(rotor, sign):
    # Eq. (2): tau = (l/sqrt2 (T1+T2-T3-T4), l/sqrt2 (-T1+T2+T3-T4), c_tau (T1-T2+T3-T4));
    # one rotor at a time, zero body rates, so w' = tau / J
    T = np.zeros(4); T[rotor] = 2.0
    xd = O.f(QUAD, state(), T)
    a = QUAD["arm"] / math.sqrt(2.0)
    tau = np.array([sign[0] * a * 2.0, sign[1] * a * 2.0, sign[2] * QUAD["c_tau"] * 2.0])
    np.testing.assert_allclose(xd[10:13], tau / np.array(QUAD["inertia"]), rtol=1e-14)
    # thrust of a level body is vertical: v' = (0, 0, F/m - g)
    np.testing.assert_allclose(xd[3:6], [0, 0, 2.0 / M - G], atol=1e-14)


def test_torque_free_body_conserves_energy_and_momentum():
    # Euler's equations without torque conserve 1/2 w^T J w and |J w|;
    # an asymmetric inertia exercises every gyroscopic term
    quad = dict(QUAD, inertia=(1.0e-3, 2.0e-3, 3.0e-3))
    J = np.array(quad["inertia"])
    x = state(w=(2.0, -1.0, 1.5))
    e0 = 0.5 * np.sum(J * x[10:13] ** 2)
    h0 = np.linalg.norm(J * x[10:13])
    x = roll(x, np.full(4, HOVER), 0.005, 400, quad)
    assert abs(0.5 * np.sum(J * x[10:13] ** 2) - e0) < 1e-9 * e0
    assert abs(np.linalg.norm(J * x[10:13]) - h0) < 1e-9 * h0
    # and the rates did change (the gyroscopic coupling is active)
    assert np.linalg.norm(x[10:13] - np.array([2.0, -1.0, 1.5])) > 0.1


def test_world_angular_momentum_direction_fixed():
    # torque-free: the world-frame angular momentum R(q) J w is constant
    quad = dict(QUAD, inertia=(1.0e-3, 2.0e-3, 3.0e-3))
    J = np.array(quad["inertia"])

    def world_h(x):
        w_, x_, y_, z_ = x[6:10]
        R = np.array([[1 - 2 * (y_ * y_ + z_ * z_), 2 * (x_ * y_ - w_ * z_), 2 * (x_ * z_ + w_ * y_)],
                      [2 * (x_ * y_ + w_ * z_), 1 - 2 * (x_ * x_ + z_ * z_), 2 * (y_ * z_ - w_ * x_)],
                      [2 * (x_ * z_ - w_ * y_), 2 * (y_ * z_ + w_ * x_), 1 - 2 * (x_ * x_ + y_ * y_)]])
        return R @ (J * x[10:13])

    x = state(w=(2.0, -1.0, 1.5))
    h0 = world_h(x)
    x = roll(x, np.full(4, HOVER), 0.002, 1000, quad)
    np.testing.assert_allclose(world_h(x), h0, atol=1e-8)


def test_quaternion_unit_after_step():
    rng = np.random.default_rng(1)
    for _ in range(20):
        q = rng.normal(size=4); q /= np.linalg.norm(q)
        x = state(v=rng.normal(size=3), q=q, w=rng.normal(size=3) * 5)
        xn = O.rk4(QUAD, x, rng.uniform(0, 7, 4), 0.02)
        assert abs(np.linalg.norm(xn[6:10]) - 1.0) < 1e-15


def test_drag_in_rotated_frame():
    # level body yawed by 90 deg: body x is world y, so D = diag(d1, d2, d3)
    # acts as diag(d2, d1, d3) on world velocity; with hover thrust
    # v' = -diag(d2, d1, d3) v
    quad = dict(QUAD, drag=(0.1, 0.3, 0.5))
    x = state(v=(1.0, 2.0, -1.0), q=(math.cos(math.pi / 4), 0, 0, math.sin(math.pi / 4)))
    xd = O.f(quad, x, np.full(4, HOVER))
    np.testing.assert_allclose(xd[3:6], [-0.3 * 1.0, -0.1 * 2.0, -0.5 * -1.0], atol=1e-14)
