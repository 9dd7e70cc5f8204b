"""θ-weighted time stepping with a sparse direct LU (oracle; test
infrastructure only).

Scheme (2.5) of §2.1 and its Ch. 3 form (§3.2.1), written with the implicit
weight θ = 1 - a (a is the weight of the old level):

    (n^{k+1} - n^k)/Δt_{k+1} + (1-θ) L_h n^k + θ L_h n^{k+1}
        = (1-θ) S(t_k) + θ S(t_{k+1}),

where L_h includes the Dirichlet coupling c_bnd N(t) of the outer ring.
Rearranged as the linear system (2.11)/(2.12):

    (I/Δt + θ L) n^{k+1} = (I/Δt - (1-θ) L) n^k + (1-θ) S^k + θ S^{k+1}
                           - (1-θ) c_bnd N^k - θ c_bnd N^{k+1}.

Each distinct (Δt, θ) is factored once with SuperLU and reused.  Every
solve takes one step of iterative refinement, x <- x + LU^{-1}(b - A x), so
that the result is the solution of the system to FP64 working accuracy: on
the 1024 x 2048 graded mesh, where the rows next to the origin carry
coefficients near 1/(r_1 Δθ)² ~ 1e13, the plain LU solve left a scaled
residual ||D^{-1}(b - A x)|| / ||D^{-1} b|| of 2.5e-14 and errors of 4e-11
after 20 levels; one refinement brings the residual to 6e-15 (a second
changes nothing).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .operator import OracleSystem


def system_matrix(sys: OracleSystem, dt: float, theta: float):
    return (sp.identity(sys.N, format="csc") / dt + theta * sys.L.tocsc()).tocsc()


def rhs(sys: OracleSystem, x, t0: float, t1: float, theta: float):
    dt = t1 - t0
    return (x / dt - (1.0 - theta) * (sys.L @ x)
            + (1.0 - theta) * sys.source(t0) + theta * sys.source(t1)
            - (1.0 - theta) * sys.bnd_term(t0) - theta * sys.bnd_term(t1))


def _lu(sys: OracleSystem, dt: float, theta: float):
    """(LU factors, matrix) of I/Δt + θ L, cached by (Δt, θ)."""
    key = (float(dt), float(theta))
    hit = sys.lu_cache.get(key)
    if hit is None:
        A = system_matrix(sys, dt, theta)
        hit = (spla.splu(A), A.tocsr())
        sys.lu_cache[key] = hit
    return hit


def solve_system(sys: OracleSystem, dt: float, theta: float, b):
    """x with (I/Δt + θ L) x = b: LU solve plus one refinement step."""
    lu, A = _lu(sys, dt, theta)
    x = lu.solve(b)
    return x + lu.solve(b - A @ x)


def step(sys: OracleSystem, x, t0: float, t1: float, theta: float):
    """One θ-scheme step from level t0 to t1."""
    return solve_system(sys, t1 - t0, theta, rhs(sys, x, t0, t1, theta))


def solve(sys: OracleSystem, t_levels, theta: float, x0=None, keep_all=False,
          max_cached=4):
    """March over t_levels[0] -> t_levels[-1]; returns n^K (and all levels)."""
    x = sys.initial() if x0 is None else np.array(x0, float)
    hist = [x.copy()] if keep_all else None
    for k in range(len(t_levels) - 1):
        x = step(sys, x, float(t_levels[k]), float(t_levels[k + 1]), theta)
        if len(sys.lu_cache) > max_cached:
            sys.lu_cache.clear()
        if keep_all:
            hist.append(x.copy())
    return (x, hist) if keep_all else x
