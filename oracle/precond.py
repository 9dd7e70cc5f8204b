"""The alternating-line preconditioner of the GPU solver, written out from its
definition (oracle; test infrastructure only).

The paper solves each level's system (2.11)/(2.12) directly.  The GPU
library solves it iteratively, with a preconditioner of its own that this
module states plainly so that its sweeps can be checked one by one.  With
A = I/Δt + θ L_h and D = diag(A), the Krylov iteration runs on D^{-1} A and

    M = (I + D^{-1} R)(I + D^{-1} Θ),   z = M^{-1} y = (I + D^{-1}Θ)^{-1} (I + D^{-1}R)^{-1} y,

where R holds the couplings between ring nodes on the same radial line
(the off-diagonal part of the tridiagonal blocks A_j of (2.12)) and Θ the
couplings between nodes of the same ring (periodic in θ) together with the
couplings between the origin and the ring-1 nodes, both ways (the origin
and ring 1 form an arrow system).  Every off-diagonal entry of A belongs to
exactly one of R and Θ.  Each factor is solved with a sparse direct LU.

Unknowns in the paper's ordering (2.12): the origin first, then (i, j) at
1 + j m + (i - 1).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .operator import OracleSystem
from .stepper import system_matrix


def coupling_split(A, m: int):
    """(R, Θ) of the off-diagonal entries of A (module docstring)."""
    C = sp.coo_matrix(A)
    r, c, v = C.row, C.col, C.data
    off = r != c
    line = lambda q: np.where(q == 0, -1, (q - 1) // m)     # θ-line j of a ring node
    ring = lambda q: np.where(q == 0, 0, (q - 1) % m + 1)   # ring i (0: the origin)
    touches_origin = (r == 0) | (c == 0)
    radial = off & ~touches_origin & (line(r) == line(c))
    angular = off & (touches_origin | (ring(r) == ring(c)))
    N = A.shape[0]
    R = sp.csr_matrix((v[radial], (r[radial], c[radial])), shape=(N, N))
    T = sp.csr_matrix((v[angular], (r[angular], c[angular])), shape=(N, N))
    return R, T


class LinePreconditioner:
    """z = M^{-1} y for the step system of `sys` at (dt, theta)."""

    def __init__(self, sys: OracleSystem, dt: float, theta: float):
        self._build(system_matrix(sys, dt, theta), sys.mesh.m)

    @classmethod
    def of_matrix(cls, A, m: int):
        """The same preconditioner for any matrix A of m rings in the paper's
        ordering (the origin, then θ-line after θ-line)."""
        P = cls.__new__(cls)
        P._build(A, m)
        return P

    def _build(self, A, m: int):
        self.A = A
        self.d = A.diagonal()
        Dinv = sp.diags(1.0 / self.d)
        R, T = coupling_split(A, m)
        N = A.shape[0]
        I = sp.identity(N, format="csc")
        self._radial = spla.splu((I + Dinv @ R).tocsc())
        self._angular = spla.splu((I + Dinv @ T).tocsc())

    def __call__(self, y):
        return self._angular.solve(self._radial.solve(np.asarray(y, float)))

    def scaled_operator(self, x):
        """D^{-1} A x."""
        return (self.A @ x) / self.d
