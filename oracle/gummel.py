"""Two carriers coupled through a polar Poisson problem, Gummel's iteration
(oracle; test infrastructure only).

The paper (§3.1) states the continuity equations of electrons n and holes p,
each with the drift of a field E, and then solves one of them with E given.
Coupling them through the field they generate is the natural next step; it
is written out here plainly, in scaled units:

    n_t = ∇·(D_n ∇n) - ∇·(n v_n) + G_n,   v_n = -μ_n 𝓔   (electrons drift against 𝓔),
    p_t = ∇·(D_p ∇p) - ∇·(p v_p) + G_p,   v_p = +μ_p 𝓔,
    -∇·(ε ∇ψ) = p - n + C,                 𝓔 = -∇ψ,

with Dirichlet data on r = 1 for n, p and ψ (or zero flux for the
carriers).  Each carrier is the continuity problem (3.1) with the drift
velocity E = s μ 𝓔 (3.4), s = -1 for electrons and +1 for holes, and is
discretised by the face-flux operator of operator.py.  The face drift comes
from the potential's difference across the face:

    radial face (i+1/2, j):  E_r = s μ (ψ_{i,j} - ψ_{i+1,j}) / h_{i+1},
    angular face (i, j+1/2): E_θ = s μ (ψ_{i,j} - ψ_{i,j+1}) / (r_i μ_{j+1}),

with ψ_{0,j} the origin value and ψ_{m+1,j} the Dirichlet value.  The
Poisson problem is the same operator with D = ε, no drift and no time
derivative.

One time level t_k -> t_{k+1} (Gummel's decoupling): starting from
(n^k, p^k), repeat  ψ <- Poisson(p - n);  (n, p) <- one θ-step from
(n^k, p^k) with the drift of ψ;  until the potential changes by at most
tol relative (max norm) between successive iterations, or for a fixed
number of iterations.  Vectors in the paper's unknown order (2.12).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .mesh import Mesh
from .operator import OracleSystem, assemble, from_vec
from .stepper import step


def poisson_system(mesh: Mesh, psi_data: dict) -> OracleSystem:
    """L of -∇·(ε∇ψ) (psi_data: D = ε, no drift, no reaction)."""
    return assemble(mesh, psi_data)


def boundary_psi(psi_sys: OracleSystem):
    """ψ on r = 1 (the Dirichlet data of the ψ problem, time-independent)."""
    return psi_sys.boundary(0.0)


def solve_poisson(psi_sys: OracleSystem, charge):
    """ψ with L ψ = charge + C - c_bnd ψ_b: the ψ problem's own sources are
    the doping C (its charge slot, mode 0, holds zero in the data)."""
    b = np.asarray(charge, float) + psi_sys.source(0.0) - psi_sys.bnd_term(0.0)
    return spla.spsolve(psi_sys.L.tocsc(), b)


def drift_faces(mesh: Mesh, psi, psi_b, mu_r, mu_t, sign: float):
    """(E_r at radial faces (m+1, n), E_θ at angular faces (m, n)) of a
    carrier with face mobilities mu_r, mu_t and charge sign."""
    m, n = mesh.m, mesh.n
    r, h, mu = mesh.r, mesh.h, mesh.mu
    p0, pg = from_vec(psi, m, n)                       # origin, (m, n)
    ext = np.vstack([np.full((1, n), p0), pg, np.asarray(psi_b, float)[None, :]])   # rings 0..m+1
    Er = sign * np.asarray(mu_r) * (ext[:m + 1] - ext[1:m + 2]) / h[1:m + 2, None]
    Et = sign * np.asarray(mu_t) * (pg - np.roll(pg, -1, axis=1)) / (r[1:m + 1, None] * mu[None, 1:n + 1])
    return Er, Et


def carrier_system(mesh: Mesh, data: dict, psi, psi_b, sign: float, flux: int = 0, bc: int = 0):
    """The carrier's operator with the drift of ψ; its mobility is its
    diffusivity (scaled Einstein relation)."""
    d = dict(data)
    d["Er_r"], d["Et_t"] = drift_faces(mesh, psi, psi_b, data["D_r"], data["D_t"], sign)
    return assemble(mesh, d, flux=flux, bc=bc)


def gummel_step(mesh: Mesh, psi_sys: OracleSystem, n_data: dict, p_data: dict, psi, n, p,
                t0: float, t1: float, theta: float, iters: int, tol: float = 0.0,
                flux: int = 0, bc: int = 0):
    """One time level of the coupled system (module docstring).  Returns
    (ψ, n, p, iterations taken, last relative change of ψ)."""
    psi_b = boundary_psi(psi_sys)
    n0, p0 = np.asarray(n, float), np.asarray(p, float)
    n, p = n0, p0
    psi_prev = np.asarray(psi, float)
    change = np.inf
    for j in range(iters):
        psi = solve_poisson(psi_sys, p - n)
        change = float(np.max(np.abs(psi - psi_prev)) / np.max(np.abs(psi)))
        sn = carrier_system(mesh, n_data, psi, psi_b, -1.0, flux, bc)
        sp_ = carrier_system(mesh, p_data, psi, psi_b, +1.0, flux, bc)
        n = step(sn, n0, t0, t1, theta)
        p = step(sp_, p0, t0, t1, theta)
        if j >= 1 and change <= tol:
            return psi, n, p, j + 1, change
        psi_prev = psi
    return psi, n, p, iters, change
