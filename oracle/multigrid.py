"""θ-semi-coarsening multigrid for the step systems (oracle; test
infrastructure only).

The paper solves each level's system (2.11)/(2.12) directly and names
multigrid-type preconditioners as the way to large grids (§4.2, outlook).
The GPU library offers one, built on its alternating-line preconditioner;
this module states it plainly so that it can be checked.

Hierarchy.  Level 0 is the step system A_0 = I/Δt + θ L in its
volume-weighted form Â_0 = V A_0 (V the control volumes of operator.py).
Level ℓ+1 merges the θ-lines of level ℓ in pairs (2J, 2J+1), the last three
together when n_ℓ is odd: P_ℓ copies the value of coarse line J to every
fine line it covers (and the origin to the origin), and

    Â_{ℓ+1} = P_ℓ^T Â_ℓ P_ℓ,    V_{ℓ+1} = P_ℓ^T V_ℓ,    A_{ℓ+1} = V_{ℓ+1}^{-1} Â_{ℓ+1}

(the Galerkin product: radial faces of a merged cell add up, the angular
face inside it drops out, the volumes add).  Lines are merged while
n_ℓ >= NMIN; below the last such level the next one holds the ring means,
one value per ring and the origin, and is solved directly.

Smoother on level ℓ: one step of the alternating-line preconditioner M_ℓ of
A_ℓ (precond.py, with D_ℓ = diag(A_ℓ)),

    x <- x + M_ℓ^{-1} D_ℓ^{-1} V_ℓ^{-1} (f - Â_ℓ x).

V-cycle(ℓ, f): smooth from x = 0; x <- x + P_ℓ V-cycle(ℓ+1, P_ℓ^T (f - Â_ℓ x))
(a direct solve on the ring-mean level); smooth again.  As the
preconditioner of the Krylov system D^{-1} A (D = diag(A_0)):
z = V-cycle(0, V D y), an approximation of (D^{-1} A)^{-1} y.

Unknowns in the paper's ordering (2.12): the origin first, then (i, j) at
1 + j m + (i - 1).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .operator import OracleSystem
from .precond import LinePreconditioner
from .stepper import system_matrix

NMIN = 16   # θ-lines are merged while a level has at least this many


def line_map(m: int, n: int):
    """(P, n_c): the 0/1 matrix merging θ-lines in pairs (the last three
    when n is odd), from n lines to n_c = n // 2."""
    nc = n // 2
    coarse_line = np.minimum(np.arange(n) // 2, nc - 1)
    i = np.arange(1, m + 1)
    rows = [np.array([0])]
    cols = [np.array([0])]
    for j in range(n):
        rows.append(1 + j * m + (i - 1))
        cols.append(1 + coarse_line[j] * m + (i - 1))
    r, c = np.concatenate(rows), np.concatenate(cols)
    return sp.csr_matrix((np.ones(r.size), (r, c)), shape=(m * n + 1, m * nc + 1)), nc


def ring_map(m: int, n: int):
    """The 0/1 matrix from n θ-lines to the ring means (m + 1 values, the
    origin first)."""
    i = np.arange(1, m + 1)
    rows = [np.array([0])] + [1 + j * m + (i - 1) for j in range(n)]
    cols = [np.array([0])] + [i for _ in range(n)]
    r, c = np.concatenate(rows), np.concatenate(cols)
    return sp.csr_matrix((np.ones(r.size), (r, c)), shape=(m * n + 1, m + 1))


class Level:
    """One level: Â (volume-weighted), V, its smoother and the map P to the
    next level."""

    def __init__(self, Ah, V, m: int, n: int):
        self.Ah = sp.csr_matrix(Ah)
        self.V = np.asarray(V, float)
        self.m, self.n = m, n
        A = sp.diags(1.0 / self.V) @ self.Ah
        self.line = LinePreconditioner.of_matrix(A.tocsc(), m)
        self.d = self.line.d
        if n >= NMIN:
            self.P, self.nc = line_map(m, n)
        else:
            self.P, self.nc = ring_map(m, n), 1

    def smooth(self, x, f):
        return x + self.line((f - self.Ah @ x) / (self.V * self.d))


def hierarchy(A0, V, m: int, n: int):
    """(levels, ring-mean matrix) of A0 = I/Δt + θL (module docstring)."""
    levels = []
    Ah, Vl, nl = sp.diags(V) @ A0, np.asarray(V, float), n
    while True:
        lev = Level(Ah, Vl, m, nl)
        levels.append(lev)
        Ah = (lev.P.T @ lev.Ah @ lev.P).tocsr()
        Vl = lev.P.T @ Vl
        if lev.nc == 1:
            return levels, Ah
        nl = lev.nc


class MultigridPreconditioner:
    """z ≈ (D^{-1}A)^{-1} y for the step system of `sys` at (dt, theta)."""

    def __init__(self, sys: OracleSystem, dt: float, theta: float):
        self.A = system_matrix(sys, dt, theta)
        self.levels, self.A_ring = hierarchy(self.A, sys.V, sys.mesh.m, sys.mesh.n)
        self._ring = spla.splu(self.A_ring.tocsc())

    def vcycle(self, l: int, f):
        lev = self.levels[l]
        x = lev.smooth(np.zeros_like(f), f)
        rc = lev.P.T @ (f - lev.Ah @ x)
        e = self.vcycle(l + 1, rc) if l + 1 < len(self.levels) else self._ring.solve(rc)
        return lev.smooth(x + lev.P @ e, f)

    def __call__(self, y):
        l0 = self.levels[0]
        return self.vcycle(0, l0.V * l0.d * np.asarray(y, float))

    def scaled_operator(self, x):
        """D^{-1} A x."""
        return (self.A @ x) / self.levels[0].d
