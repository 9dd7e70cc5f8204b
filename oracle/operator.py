"""Discrete spatial operator L_h as a sparse FP64 matrix (oracle; test
infrastructure only).

Unknowns in the paper's ordering (2.12): index 0 is the origin, and
(i, j), i = 1..m, j = 0..n-1 sits at 1 + j m + (i - 1).

Conservative face-flux form (default).  It writes both PDEs as
n_t + L n = S with L n = -∇·(D∇n) + ∇·(nE) + b n and integrates L over the
control volume of each node:

* ring cell (i, j):  V_ij = r_i (h_i + h_{i+1})/2 · (μ_j + μ_{j+1})/2 -- the
  volume whose reciprocals appear as the prefactors 2/(r_i(h_i+h_{i+1})) and
  2/(r_i²(μ_j+μ_{j+1})) of the stencils in §2.1 and §3.2.1;
* origin: the disk of radius h_1/2, V_0 = π (h_1/2)² (§3.2.2, time term).

Each face carries a conductance G and a drift coefficient K, oriented from
the inner (or lower-θ) node P to the outer (or higher-θ) node Q:
    radial face (i+1/2, j):  G = D(r_{i+1/2}, θ_j) r_{i+1/2} Δθ_j / h_{i+1},
                             K = E_r(r_{i+1/2}, θ_j) r_{i+1/2} Δθ_j,
    angular face (i, j+1/2): G = D(r_i, θ_{j+1/2}) (h_i+h_{i+1})/2 / (r_i μ_{j+1}),
                             K = E_θ(r_i, θ_{j+1/2}) (h_i+h_{i+1})/2,
where Δθ_j = (μ_j + μ_{j+1})/2.  The face i = 0 joins the origin to (1, j)
(r_{1/2} = h_1/2), so the origin row sums all n of its faces -- the
control-volume closure of §3.2.2 with the central average (n_0 + n_1)/2 for
the drift.  The flux P -> Q is
    central:  F = G (n_P - n_Q) + K (n_P + n_Q)/2,
    upwind:   F = G (n_P - n_Q) + max(K, 0) n_P + min(K, 0) n_Q,
and (L n)_P = (1/V_P) Σ_faces F_out + b_P n_P.  With D = 1, E = 0 and a
uniform θ mesh this is exactly ℘_h of §2.1 including its origin row.

The outer face i = m+1/2 touches the Dirichlet value N_j (eq. (2.9) /
(3.2)); its off-diagonal coefficient is returned as ``c_bnd`` so that
(L_h n)_{m,j} = (row of L) · n + c_bnd[j] N_j.  With the zero-flux option
the outer face carries no flux.

The literal form (``assemble_literal``) enters the printed coefficients of
ϖ_h (§3.2.1) and of the origin row of §3.2.2 one by one, with scalar E at
the nodes and one-sided drift differences.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

from .mesh import Mesh


def idx(m: int, i, j):
    """Paper-order position of ring node (i, j), i = 1..m."""
    return 1 + np.asarray(j) * m + (np.asarray(i) - 1)


def to_vec(origin, grid):
    """(origin, (m, n) grid) -> paper-order vector."""
    grid = np.asarray(grid)
    return np.concatenate([[origin], grid.T.reshape(-1)])


def from_vec(v, m, n):
    """paper-order vector -> (origin, (m, n) grid)."""
    v = np.asarray(v)
    return v[0], v[1:].reshape(n, m).T


@dataclass
class OracleSystem:
    mesh: Mesh
    L: sp.csr_matrix
    V: np.ndarray
    c_bnd: np.ndarray
    data: dict
    bc: int = 0
    flux: int = 0
    lu_cache: dict = field(default_factory=dict)

    @property
    def N(self):
        return self.L.shape[0]

    def bnd_rows(self):
        return idx(self.mesh.m, self.mesh.m, np.arange(self.mesh.n))

    def source(self, t):
        d = self.data
        s = np.zeros(self.N)
        for q in range(d["lam"].size):
            tau = (t ** int(d["tpow"][q]) if d["tpow"][q] else 1.0) * np.exp(d["lam"][q] * t)
            s += tau * to_vec(d["g_origin"][q], d["g_grid"][q])
        return s

    def boundary(self, t):
        d = self.data
        nb = np.zeros(self.mesh.n)
        for q in range(d["lam"].size):
            tau = (t ** int(d["tpow"][q]) if d["tpow"][q] else 1.0) * np.exp(d["lam"][q] * t)
            nb += tau * d["nb"][q]
        return nb

    def bnd_term(self, t):
        """Vector c_bnd · N(t) placed on the ring-m rows (zero for zero-flux)."""
        v = np.zeros(self.N)
        if self.bc == 0:
            v[self.bnd_rows()] = self.c_bnd * self.boundary(t)
        return v

    def initial(self):
        return to_vec(self.data["u0_origin"], self.data["u0_grid"])


def _face_split(K, flux):
    if flux == 0:
        return 0.5 * K, 0.5 * K
    return np.maximum(K, 0.0), np.minimum(K, 0.0)


def volumes(mesh: Mesh):
    m, n = mesh.m, mesh.n
    r, h, dth = mesh.r, mesh.h, mesh.dtheta
    ring = r[1:m + 1, None] * 0.5 * (h[1:m + 1, None] + h[2:m + 2, None]) * dth[None, :]
    return to_vec(np.pi * (0.5 * h[1]) ** 2, ring)


def assemble(mesh: Mesh, data: dict, flux: int = 0, bc: int = 0) -> OracleSystem:
    """Conservative face-flux assembly of L_h (module docstring)."""
    m, n = mesh.m, mesh.n
    r, h, rh, mu, dth = mesh.r, mesh.h, mesh.r_half, mesh.mu, mesh.dtheta
    N = m * n + 1
    V = volumes(mesh)
    rows, cols, vals = [], [], []

    def add(P, Q, G, K):
        kp, kq = _face_split(K, flux)
        rows.extend([P, P, Q, Q])
        cols.extend([P, Q, Q, P])
        vals.extend([(G + kp) / V[P], (-G + kq) / V[P], (G - kq) / V[Q], (-G - kp) / V[Q]])

    J = np.arange(n)
    # origin <-> ring 1
    G0 = data["D_r"][0] * rh[0] * dth / h[1]
    K0 = data["Er_r"][0] * rh[0] * dth
    add(np.zeros(n, int), idx(m, 1, J), G0, K0)
    # interior radial faces
    for i in range(1, m):
        G = data["D_r"][i] * rh[i] * dth / h[i + 1]
        K = data["Er_r"][i] * rh[i] * dth
        add(idx(m, i, J), idx(m, i + 1, J), G, K)
    # angular faces (periodic: j = n-1 joins j = 0 through μ_n)
    for i in range(1, m + 1):
        w = 0.5 * (h[i] + h[i + 1])
        G = data["D_t"][i - 1] * w / (r[i] * mu[1:n + 1])
        K = data["Et_t"][i - 1] * w
        add(idx(m, i, J), idx(m, i, (J + 1) % n), G, K)
    # outer face
    Pm = idx(m, m, J)
    c_bnd = np.zeros(n)
    if bc == 0:
        Gb = data["D_r"][m] * rh[m] * dth / h[m + 1]
        Kb = data["Er_r"][m] * rh[m] * dth
        kp, kq = _face_split(Kb, flux)
        rows.extend([Pm])
        cols.extend([Pm])
        vals.extend([(Gb + kp) / V[Pm]])
        c_bnd = (-Gb + kq) / V[Pm]
    # reaction
    b = to_vec(data["b_origin"], data["b_grid"])
    rows.append(np.arange(N))
    cols.append(np.arange(N))
    vals.append(b)
    L = sp.coo_matrix((np.concatenate([np.atleast_1d(np.asarray(v, float)) for v in vals]),
                       (np.concatenate([np.atleast_1d(np.asarray(v)) for v in rows]),
                        np.concatenate([np.atleast_1d(np.asarray(v)) for v in cols]))),
                      shape=(N, N)).tocsr()
    L.sum_duplicates()
    return OracleSystem(mesh, L, V, c_bnd, data, bc=bc, flux=flux)


def assemble_literal(mesh: Mesh, data: dict) -> OracleSystem:
    """ϖ_h of §3.2.1 and the origin row of §3.2.2 entered as printed.

    Non-origin row (i, j), with D at the face points of the flux form and
    the scalar E at the node:
      diag   2/(r_i(h_i+h_{i+1})) (r_{i+1/2}D_{i+1/2,j}/h_{i+1} + r_{i-1/2}D_{i-1/2,j}/h_i)
             + 2/(r_i²(μ_j+μ_{j+1})) (D_{i,j+1/2}/μ_{j+1} + D_{i,j-1/2}/μ_j)
             + E_ij (1/(r_i μ_{j+1}) + 1/h_{i+1})
      (i-1,j) -2 r_{i-1/2} D_{i-1/2,j} / (r_i h_i (h_i+h_{i+1}))
      (i+1,j) -(2 r_{i+1/2} D_{i+1/2,j} / (r_i h_{i+1}(h_i+h_{i+1})) + E_ij/h_{i+1})
      (i,j-1) -2 D_{i,j-1/2} / (r_i² μ_j (μ_j+μ_{j+1}))
      (i,j+1) -(2 D_{i,j+1/2} / (r_i² μ_{j+1}(μ_j+μ_{j+1})) + E_ij/(r_i μ_{j+1}))
    Origin row: (4D_00/h_1² + E_00/h_1) n_00 - (4D_00/(n h_1²) - E_00/(n h_1)) Σ_j n_1j.
    The node (0, j) is the origin; (m+1, j) is the Dirichlet value.  The
    parabolic reaction b, if present, is added to the diagonal (℘_h, §2.1).
    """
    m, n = mesh.m, mesh.n
    r, h, rh, mu = mesh.r, mesh.h, mesh.r_half, mesh.mu
    N = m * n + 1
    E = data.get("E_grid", np.zeros((m, n)))
    E0 = data.get("E_origin", 0.0)
    D0 = data["D_origin"]
    rows, cols, vals = [], [], []
    c_bnd = np.zeros(n)
    for i in range(1, m + 1):
        for j in range(n):
            P = idx(m, i, j)
            jm, jp = (j - 1) % n, (j + 1) % n
            Dp, Dm = data["D_r"][i, j], data["D_r"][i - 1, j]
            Dtp, Dtm = data["D_t"][i - 1, j], data["D_t"][i - 1, jm]
            mj, mj1 = mu[j], mu[j + 1]
            e = E[i - 1, j]
            s = h[i] + h[i + 1]
            diag = (2.0 / (r[i] * s) * (rh[i] * Dp / h[i + 1] + rh[i - 1] * Dm / h[i])
                    + 2.0 / (r[i] ** 2 * (mj + mj1)) * (Dtp / mj1 + Dtm / mj)
                    + e * (1.0 / (r[i] * mj1) + 1.0 / h[i + 1]))
            c_in = -2.0 * rh[i - 1] * Dm / (r[i] * h[i] * s)
            c_out = -(2.0 * rh[i] * Dp / (r[i] * h[i + 1] * s) + e / h[i + 1])
            c_lo = -2.0 * Dtm / (r[i] ** 2 * mj * (mj + mj1))
            c_hi = -(2.0 * Dtp / (r[i] ** 2 * mj1 * (mj + mj1)) + e / (r[i] * mj1))
            rows += [P, P, P, P]
            cols += [P, (0 if i == 1 else idx(m, i - 1, j)), idx(m, i, jm), idx(m, i, jp)]
            vals += [diag, c_in, c_lo, c_hi]
            if i < m:
                rows.append(P)
                cols.append(idx(m, i + 1, j))
                vals.append(c_out)
            else:
                c_bnd[j] = c_out
    rows.append(0)
    cols.append(0)
    vals.append(4.0 * D0 / h[1] ** 2 + E0 / h[1])
    off = -(4.0 * D0 / (n * h[1] ** 2) - E0 / (n * h[1]))
    for j in range(n):
        rows.append(0)
        cols.append(idx(m, 1, j))
        vals.append(off)
    b = to_vec(data["b_origin"], data["b_grid"])
    rows += list(range(N))
    cols += list(range(N))
    vals += list(b)
    L = sp.coo_matrix((np.array(vals, float), (np.array(rows), np.array(cols))),
                      shape=(N, N)).tocsr()
    L.sum_duplicates()
    V = volumes(mesh)
    return OracleSystem(mesh, L, V, c_bnd, data, bc=0, flux=-1)
