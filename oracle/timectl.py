"""A-posteriori time-step control of the θ-scheme (oracle; test infrastructure only).

The paper advances on time levels fixed in advance (§2.1 Δt = T/K, the time
stretch of §3.1) and leaves adaptive stepping to tuning.  This module is the
reading the library implements for its adaptive mode, written out plainly.

The scheme is the θ-method for the semi-discrete system x' = f(t, x) with

    f(t, x) = -L x + S(t) - c_bnd N(t)

(the right-hand side of (2.11) divided into its two time levels):

    (x_{k+1} - x_k)/Δt = (1-θ) f(t_k, x_k) + θ f(t_{k+1}, x_{k+1}).

Local error estimates, from Taylor expansion of both sides:

* θ ≠ 1/2: x_{k+1} - x(t_{k+1}) = (θ - 1/2) Δt² x'' + O(Δt³); with
  x'' ≈ (f_{k+1} - f_k)/Δt the estimate is d = (θ - 1/2) Δt (f_{k+1} - f_k),
  order q = 1.
* θ = 1/2 (trapezoidal rule): its error Δt³ x'''/12 is estimated against the
  variable-step second-order Adams-Bashforth predictor
  x^P = x_k + Δt ((1 + r/2) f_k - (r/2) f_{k-1}), r = Δt/Δt_prev, as
  d = (x_{k+1} - x^P) / (3 (1 + Δt_prev/Δt)), order q = 2 (the TR-AB2 pair).

Controller (relative L2 error e = ||d|| / ||x_{k+1}||, tolerance tol):

* the first step is taken with Δt_0 and accepted, and the second is also
  tried with Δt_0 (the TR-AB2 pair needs the derivatives of two earlier
  levels; every θ is treated alike);
* a step is rejected when e > 2 tol and Δt > dt_min (its level lies beyond
  the level a dt_min step reaches): it is retaken with
  Δt max(1/4, 0.9 (tol/e)^{1/(q+1)}) (at least dt_min);
* after an accepted step the next is Δt clamp(0.9 (tol/e)^{1/(q+1)}, 1/2, 2)
  (2 when e = 0), clamped to [dt_min, dt_max];
* landing on T: a step that would pass T ends at T, and one that would leave
  less than a step ends half-way;
* a Crank-Nicolson solve (θ = 1/2) takes its first RANNACHER steps with
  backward Euler (θ = 1, first-order estimate).  Crank-Nicolson carries the
  stiff components of the initial state undamped (its amplification tends
  to -1), and the TR-AB2 estimate multiplies them by λΔt: on the 256 x 512
  graded mesh at tol 1e-7 it held Δt at dt_min for thousands of steps,
  while two backward-Euler steps first brought the run to 62 steps;
* after STALL steps in a row forced through at dt_min with e > 2 tol, the
  tolerance is out of reach and the solve stops before T.
"""

from __future__ import annotations

import numpy as np

from .stepper import rhs, solve_system, step

RANNACHER = 2
STALL = 20


def f_eval(sys, x, t):
    """f(t, x) = -L x + S(t) - c_bnd N(t)."""
    return -(sys.L @ x) + sys.source(t) - sys.bnd_term(t)


def local_error(x1, x0, f1, f0, fm1, dt, dt_prev, theta):
    """Estimate d of the local error of the step t_k -> t_k + dt, and its
    order q.  fm1 (f at t_{k-1}) and dt_prev are used for θ = 1/2 only."""
    if theta != 0.5:
        return (theta - 0.5) * dt * (f1 - f0), 1
    r = dt / dt_prev
    xp = x0 + dt * ((1.0 + 0.5 * r) * f0 - 0.5 * r * fm1)
    return (x1 - xp) / (3.0 * (1.0 + dt_prev / dt)), 2


def step_factor(e, tol, q):
    """Growth factor of the next step after an accepted one."""
    if e <= 0.0:
        return 2.0
    return min(2.0, max(0.5, 0.9 * (tol / e) ** (1.0 / (q + 1))))


def retry_factor(e, tol, q):
    """Shrink factor of a rejected step."""
    return max(0.25, 0.9 * (tol / e) ** (1.0 / (q + 1)))


def next_level(t, dt, T):
    """The time level a step dt from t reaches (exactly T when it lands)."""
    return T if dt >= T - t else t + dt


def land(t, dt, T):
    """Step from t that neither passes T nor leaves less than a step before it."""
    rem = T - t
    if dt >= rem:
        return rem
    if dt > 0.5 * rem:
        return 0.5 * rem
    return dt


def step_theta(theta, k):
    """θ of adaptive step k (0-based): backward Euler for the first
    RANNACHER steps of a Crank-Nicolson solve."""
    return 1.0 if (theta == 0.5 and k < RANNACHER) else theta


def solve_adaptive(sys, theta, T, dt0, tol, dt_min, dt_max, t0=0.0, x0=None, max_steps=100000):
    """Adaptive θ-scheme from t0 to t0 + T.  Returns (x, accepted time levels,
    per-step (dt, error estimate), number of rejected attempts).  Each
    attempted step is solved exactly (sparse LU).  A solve that stalls at
    dt_min stops early (its last level is then before t0 + T)."""
    x = sys.initial() if x0 is None else np.array(x0, float)
    t_end = t0 + T
    t = t0
    f_prev = None
    f_cur = f_eval(sys, x, t)
    dt_prev = None
    dt = land(t, min(max(dt0, dt_min), dt_max), t_end)
    levels, steps, rejected, stall = [t], [], 0, 0
    while t < t_end and len(steps) < max_steps and stall < STALL:
        th = step_theta(theta, len(steps))
        t1 = next_level(t, dt, t_end)
        x1 = solve_system(sys, t1 - t, th, rhs(sys, x, t, t1, th))
        f1 = f_eval(sys, x1, t1)
        if f_prev is None:
            e, q, accept = 0.0, (2 if th == 0.5 else 1), True   # first step: accepted as is
        else:
            d, q = local_error(x1, x, f1, f_cur, f_prev, t1 - t, dt_prev, th)
            e = float(np.linalg.norm(d) / max(np.linalg.norm(x1), 1e-300))
            # "longer than dt_min" compares levels: the step's level against
            # the one a dt_min step reaches (t1 - t itself may round above
            # dt_min, which would reject a step at dt_min again and again)
            accept = not (e > 2.0 * tol and t1 > next_level(t, dt_min, t_end))
        if not accept:
            rejected += 1
            dt = land(t, max(dt_min, (t1 - t) * retry_factor(e, tol, q)), t_end)
            continue
        stall = stall + 1 if (f_prev is not None and e > 2.0 * tol) else 0
        steps.append((t1 - t, e))
        dt_prev = t1 - t
        f_prev, f_cur = f_cur, f1
        x, t = x1, t1
        levels.append(t)
        if len(sys.lu_cache) > 4:
            sys.lu_cache.clear()
        nxt = dt_prev * step_factor(e, tol, q) if len(steps) > 1 else dt_prev
        dt = land(t, min(max(nxt, dt_min), dt_max), t_end)
    return x, np.array(levels), steps, rejected


def solve_levels(sys, levels, theta, x0=None, adaptive_start=False):
    """Re-runs a given sequence of time levels (e.g. one logged by the GPU);
    adaptive_start: the levels come from an adaptive solve, whose first
    steps follow step_theta."""
    x = sys.initial() if x0 is None else np.array(x0, float)
    for k in range(len(levels) - 1):
        t0, t1 = float(levels[k]), float(levels[k + 1])
        x = step(sys, x, t0, t1, step_theta(theta, k) if adaptive_start else theta)
        if len(sys.lu_cache) > 4:
            sys.lu_cache.clear()
    return x
