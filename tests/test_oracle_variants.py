"""Pins of the two standard MPPI variants the oracle offers besides the
paper's literal method (both off by default): the control-cost term of
information-theoretic MPPI (Williams et al., the line of work the paper's
Sec. II-A builds on) and several MPPI iterations per control step.

With every state cost switched off, a sample's cost is the control-cost term
alone, gamma * sum U* (U - U*) / sigma^2, and the weights exp(-J / lambda)
tilt each Gaussian perturbation by exp(-a e) with a = (gamma / lambda) U* /
sigma^2.  The mean of a tilted N(0, sigma^2) is -a sigma^2, so the update
moves U* to (1 - gamma / lambda) U*; n iterations compound the factor.  These
properties, not the formula, are what the tests check.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_14726_amd import synth

DT = 0.02


def _zero_cost_tracking(K, N, **over):
    """Tracking objective with every state and rate weight zero: the rollout
    cost of every sample is exactly 0."""
    w = synth.single_solve_workload(K=K, N=N, objective="track", seed=21)
    prm = dict(w["params"], Q=[0.0] * 13, QN=[0.0] * 13, R_dT=[0.0] * 4, w_lim=0.0, eps_dec=0.0, n_threads=8)
    prm.update(over)
    pb = O.Problem(w["quad"], prm, xref=w["xref"], ref_dt=w["ref_dt"])
    return pb, w


def _warm_with(pb, U, t_prev):
    wm = pb.warm(0)
    wm.warm = 1
    wm.t_prev = t_prev
    for k in range(U.shape[0]):
        for i in range(4):
            wm.U[4 * k + i] = U[k, i]
    return wm


def _statistical_check(r, want, sigma):
    """|U - want| within 5 standard errors of a weighted mean of ESS samples."""
    se = sigma / np.sqrt(r["ess"])
    assert np.all(np.abs(r["U"] - want) < 5.0 * se), (r["U"], want, se, r["ess"])
    return se


def test_control_cost_tilts_the_update_toward_zero():
    N, K, sig, gamma = 2, 40000, 0.5, 0.1
    pb, w = _zero_cost_tracking(K, N, sigma=(sig,) * 4, ctrl_cost=gamma, **{"lambda": 1.0})
    U = np.array([[2.5, 3.0, 3.5, 4.0]] * N)
    r = pb.solve(_warm_with(pb, U, -DT), w["x0"], 0.0)
    assert r["status"] == O.OK and r["shift"] == 1
    se = _statistical_check(r, (1.0 - gamma) * U, sig)
    # the tilt itself is far outside the noise of the estimate
    assert np.all(np.abs(r["U"] - U) > 10.0 * se)


def test_control_cost_is_linear_in_gamma_and_needs_noise():
    N, K = 12, 64
    base = dict(sigma=(0.4, 0.0, 0.9, 0.2), **{"lambda": 3.0})
    J = {}
    for g in (0.0, 1.0, 2.5):
        pb, w = _zero_cost_tracking(K, N, ctrl_cost=g, **base)
        U = np.tile([2.0, 3.0, 4.0, 5.0], (N, 1)) + 0.1 * np.arange(N)[:, None]
        r = pb.solve(_warm_with(pb, U, -DT), w["x0"], 0.0)
        assert r["status"] == O.OK
        J[g] = r["J"]
        if g == 0.0:
            assert np.all(r["J"] == 0.0)
    d1, d25 = J[1.0] - J[0.0], J[2.5] - J[0.0]
    assert np.abs(d1).max() > 1.0
    np.testing.assert_allclose(d25, 2.5 * d1, rtol=1e-12, atol=1e-12)
    # without noise every sample is the nominal: no perturbation, no term
    pb, w = _zero_cost_tracking(K, N, ctrl_cost=5.0, sigma=(0.0,) * 4)
    r = pb.solve(_warm_with(pb, np.full((N, 4), 3.0), -DT), w["x0"], 0.0)
    assert np.all(r["J"] == 0.0)


def test_two_iterations_compound_the_tilt_without_shifting():
    """Iteration 1 shifts the warm start by one step, iteration 2 (same time)
    does not shift: U* varies along the horizon, so a second shift would
    show as U*_{k+1} in place of U*_k."""
    N, K, sig, gamma = 3, 60000, 0.5, 0.1
    pb, w = _zero_cost_tracking(K, N, sigma=(sig,) * 4, ctrl_cost=gamma, n_iter=2, **{"lambda": 1.0})
    U = np.array([[2.0, 2.5, 3.0, 3.5]]) + 0.6 * np.arange(N)[:, None]
    wm = _warm_with(pb, U, -DT)
    s0 = wm.s
    r = pb.solve(wm, w["x0"], 0.0)
    assert r["status"] == O.OK and r["shift"] == 0 and r["n_amb_earlier"] == 0
    # the first iteration's warm start, shifted by one step (last row repeated)
    Ustar1 = U[[min(k + 1, N - 1) for k in range(N)]]
    _statistical_check(r, (1.0 - gamma) ** 2 * Ustar1, sig)
    assert wm.s == s0 + 2 and wm.t_prev == 0.0


def test_zero_noise_iterations_are_idempotent_and_keep_the_applied_input():
    """Without noise every iteration returns its nominal.  The rate term of
    Eq. (8) then sees the same sequence in every iteration, measured from the
    input applied before the control step (the warm start's first row), so
    the cost of the last iteration equals the single iteration's: had an
    inner iteration taken its predecessor's first input as the last applied
    one, the first rate term would change."""
    N = 8
    U = np.array([[2.0, 2.5, 3.0, 3.5]]) + 0.3 * np.arange(N)[:, None]
    out = {}
    for n_iter in (1, 3):
        pb, w = _zero_cost_tracking(4, N, sigma=(0.0,) * 4, R_dT=[1e-3] * 4, n_iter=n_iter)
        wm = _warm_with(pb, U, -DT)
        r = pb.solve(wm, w["x0"], 0.0)
        assert r["status"] == O.OK
        out[n_iter] = (r["U"].copy(), r["J_min"], wm.s)
    np.testing.assert_array_equal(out[1][0], out[3][0])
    assert out[1][1] == out[3][1] and out[1][1] > 1.0
    assert out[3][2] == out[1][2] + 2


def test_invalid_variant_settings_rejected():
    pb, w = _zero_cost_tracking(4, 5, n_iter=65)
    assert pb.solve(pb.warm(), w["x0"], 0.0)["status"] == O.EINVAL
    pb, w = _zero_cost_tracking(4, 5, ctrl_cost=-1.0)
    assert pb.solve(pb.warm(), w["x0"], 0.0)["status"] == O.EINVAL
