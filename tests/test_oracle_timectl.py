"""Pins of the oracle's a-posteriori time-step control: the local error
estimates against the exact one-step error of y' = λy (constants, signs and
the variable-step ratio), the derivative f against the scheme's own
identity, and the controller's invariants on a small problem."""

import numpy as np
import pytest

from oracle import assemble, make_mesh, solve, time_levels
from oracle.stepper import rhs, system_matrix
from oracle.timectl import (RANNACHER, STALL, f_eval, land, local_error, retry_factor, solve_adaptive,
                            solve_levels, step_factor, step_theta)
from oracle.stepper import step
from problems import continuity_cfg, sample


def theta_step(y0, lam, dt, theta):
    """One θ-step of y' = λy."""
    return y0 * (1.0 + (1.0 - theta) * lam * dt) / (1.0 - theta * lam * dt)


@pytest.mark.parametrize("theta", [1.0, 0.75, 0.6])
@pytest.mark.parametrize("r", [1.0, 1.5, 0.7])
def test_first_order_estimate_matches_the_local_error(theta, r):
    """θ ≠ 1/2: the estimate is (θ - 1/2)Δt(f1 - f0); starting from the exact
    value, the step's error y1 - y(t+Δt) and the estimate agree to O(Δt)."""
    lam, t = -2.0, 0.3
    for dt in (2e-3, 1e-3):
        y0 = np.exp(lam * t)
        y1 = theta_step(y0, lam, dt, theta)
        true = y1 - np.exp(lam * (t + dt))
        d, q = local_error(np.array([y1]), np.array([y0]), np.array([lam * y1]), np.array([lam * y0]),
                           np.array([lam * np.exp(lam * (t - dt / r))]), dt, dt / r, theta)
        assert q == 1
        assert abs(d[0] / true - 1.0) < 5 * abs(lam) * dt, (dt, d[0], true)


@pytest.mark.parametrize("r", [1.0, 1.5, 0.6])
def test_tr_ab2_estimate_matches_the_local_error(r):
    """θ = 1/2: the TR-AB2 estimate with a previous step Δt/r reproduces the
    trapezoidal rule's local error Δt³ y'''/12 to O(Δt)."""
    lam, t = -3.0, 0.2
    for dt in (4e-3, 2e-3):
        dtp = dt / r
        y0 = np.exp(lam * t)
        ym1 = np.exp(lam * (t - dtp))
        y1 = theta_step(y0, lam, dt, 0.5)
        true = y1 - np.exp(lam * (t + dt))
        d, q = local_error(np.array([y1]), np.array([y0]), np.array([lam * y1]), np.array([lam * y0]),
                           np.array([lam * ym1]), dt, dtp, 0.5)
        assert q == 2
        assert abs(d[0] / true - 1.0) < 8 * abs(lam) * dt, (r, dt, d[0], true)


def small_system(seed=4101, m=10, n=24, theta=0.5):
    pb = continuity_cfg(seed, m, n, theta, 1.3)
    me = make_mesh(m, n, 1, 1.3)
    return assemble(me, sample(pb, *me.sample_points()))


@pytest.mark.parametrize("theta", [0.5, 1.0])
def test_f_satisfies_the_scheme_identity(theta):
    """(x1 - x0)/Δt = (1-θ) f(t0, x0) + θ f(t1, x1) for the exact step."""
    S = small_system(theta=theta)
    x0 = S.initial()
    t0, t1 = 0.01, 0.0137
    x1 = np.linalg.solve(system_matrix(S, t1 - t0, theta).toarray(), rhs(S, x0, t0, t1, theta))
    lhs = (x1 - x0) / (t1 - t0)
    r = (1 - theta) * f_eval(S, x0, t0) + theta * f_eval(S, x1, t1)
    assert np.max(np.abs(lhs - r)) <= 1e-9 * np.max(np.abs(lhs))


def test_landing():
    assert land(0.9, 0.2, 1.0) == pytest.approx(0.1)
    assert land(0.7, 0.2, 1.0) == pytest.approx(0.15)   # would leave 0.1 < one step: half-way
    assert land(0.0, 0.2, 1.0) == 0.2


@pytest.mark.parametrize("theta", [0.5, 1.0])
def test_controller_invariants_and_error_follows_tolerance(theta):
    S = small_system(theta=theta)
    T, dt_min, dt_max = 0.05, 1e-5, 1e-2
    ref = solve(S, time_levels(T, 4096), theta)
    errs = []
    for tol in (1e-4, 1e-5):
        x, lv, steps, rej = solve_adaptive(S, theta, T, 1e-4, tol, dt_min, dt_max)
        dts = np.diff(lv)
        assert lv[0] == 0.0 and lv[-1] == T and np.all(dts > 0)
        assert np.all(dts <= dt_max * (1 + 1e-12))
        assert np.all(dts[2:-2] >= dt_min * (1 - 1e-12))
        assert np.all(dts[1:-2] / dts[:-3] <= 2.0 * (1 + 1e-12))    # growth (the last steps may land)
        assert all(e <= 2 * tol for dt, e in steps[1:] if dt > dt_min)
        # replaying the accepted levels gives the same state
        assert np.max(np.abs(solve_levels(S, lv, theta, adaptive_start=True) - x)) <= 1e-12 * np.max(np.abs(x))
        errs.append(np.max(np.abs(x - ref)) / np.max(np.abs(ref)))
    assert errs[1] < errs[0]


@pytest.mark.parametrize("q", [1, 2])
def test_step_factor_at_hand_computed_errors(q):
    """0.9 (tol/e)^{1/(q+1)} equals a chosen g at e = tol (0.9/g)^{q+1}:
    inside [1/2, 2] the factor is g itself, and it sits on each clamp at the
    error that reaches it.  An exponent 1/q instead of 1/(q+1) fails."""
    tol = 3e-7
    for g in (1.5, 1.0, 0.7):
        e = tol * (0.9 / g) ** (q + 1)
        assert step_factor(e, tol, q) == pytest.approx(g, rel=1e-12)
    assert step_factor(tol * (0.9 / 2.0) ** (q + 1), tol, q) == pytest.approx(2.0, rel=1e-12)
    assert step_factor(0.5 * tol * (0.9 / 2.0) ** (q + 1), tol, q) == 2.0     # clamped above
    assert step_factor(tol * 1.8 ** (q + 1), tol, q) == pytest.approx(0.5, rel=1e-12)
    assert step_factor(2.0 * tol * 1.8 ** (q + 1), tol, q) == 0.5              # clamped below
    assert step_factor(0.0, tol, q) == 2.0


@pytest.mark.parametrize("q", [1, 2])
def test_retry_factor_at_hand_computed_errors(q):
    """A rejected step shrinks by 0.9 (tol/e)^{1/(q+1)}, at least to 1/4."""
    tol = 1e-6
    for g in (0.8, 0.4):
        assert retry_factor(tol * (0.9 / g) ** (q + 1), tol, q) == pytest.approx(g, rel=1e-12)
    assert retry_factor(tol * 3.6 ** (q + 1), tol, q) == pytest.approx(0.25, rel=1e-12)
    assert retry_factor(10.0 * tol * 3.6 ** (q + 1), tol, q) == 0.25


def test_crank_nicolson_starts_with_backward_euler_steps():
    """An adaptive Crank-Nicolson solve takes its first RANNACHER steps with
    θ = 1: its first levels equal plain backward-Euler steps over the same
    levels, and other θ are left alone."""
    assert RANNACHER == 2
    assert [step_theta(0.5, k) for k in range(4)] == [1.0, 1.0, 0.5, 0.5]
    assert [step_theta(0.7, k) for k in range(3)] == [0.7, 0.7, 0.7]
    S = small_system(theta=0.5)
    x, lv, steps, rej = solve_adaptive(S, 0.5, 0.01, 1e-4, 1e-5, 1e-6, 1e-2)
    y = S.initial()
    for k in range(RANNACHER):
        y = step(S, y, lv[k], lv[k + 1], 1.0)
    x2 = solve_levels(S, lv[:RANNACHER + 1], 0.5, adaptive_start=True)
    assert np.max(np.abs(x2 - y)) <= 1e-13 * np.max(np.abs(y))
    # with Crank-Nicolson throughout the second level differs
    x2cn = solve_levels(S, lv[:RANNACHER + 1], 0.5)
    assert np.max(np.abs(x2cn - y)) > 1e-9 * np.max(np.abs(y))


def test_solve_stops_when_tolerance_is_out_of_reach_at_dt_min():
    """A tolerance that even dt_min cannot meet: after STALL steps forced
    through at dt_min the solve stops before T."""
    S = small_system(theta=1.0)
    dt_min = 1e-3
    x, lv, steps, rej = solve_adaptive(S, 1.0, 1.0, dt_min, 1e-14, dt_min, 1e-2)
    assert lv[-1] < 1.0
    assert len(steps) == STALL + 1      # the first step (accepted as is) and STALL stalled ones
    assert all(e > 2e-14 for _, e in steps[1:])
