"""Pins of the FP64 oracle to things other than itself.

Each test fixes the oracle against something the paper or mathematics
determines: the printed stencil ℘_h (§2.1), a closed-form solution the scheme
must reproduce exactly, discrete conservation of the control-volume scheme,
the maximum principle of the M-matrix (§2.2), convergence order against
manufactured solutions, a brute-force dense solve, and the paper's printed
error tables (Tables 2.1 and 3.1).
"""

import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import assemble, assemble_literal, make_mesh, solve, time_levels
from oracle.operator import from_vec, idx, to_vec, volumes
from oracle.stepper import rhs, step, system_matrix
from problems import (closed_form_quadratic, continuity_cfg, paper_continuity_ex1,
                      paper_parabolic_ex1, parabolic_family, random_positive, sample,
                      zero_flux_random)
from problems.manufactured import exact_at

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def build(pb, m, n, r_kind=0, p=1.0, th_kind=0, q=1.0, flux=0, bc=0, literal=False):
    me = make_mesh(m, n, r_kind, p, th_kind, q)
    d = sample(pb, *me.sample_points())
    return (assemble_literal(me, d) if literal else assemble(me, d, flux=flux, bc=bc)), me


def max_err(x, pb, t, me, skip_origin=False):
    e0, eg = exact_at(pb, t, me.r, me.th)
    ex = to_vec(e0, eg)
    d = np.abs(x - ex)
    return float(np.max(d[1:] if skip_origin else d))


# ----------------------------------------------------------------- mesh

@pytest.mark.parametrize("kind,p", [(0, 1.0), (1, 1.0), (1, 1.3), (1, 0.1), (3, 0.6)])
def test_radial_mesh_endpoints_monotone(kind, p):
    me = make_mesh(37, 64, kind, p, 1, 1.9)
    assert me.r[0] == 0.0 and me.r[-1] == 1.0
    assert np.all(np.diff(me.r) > 0)
    assert me.th[0] == 0.0 and me.th[-1] == 2 * np.pi
    assert np.all(np.diff(me.th) > 0)
    assert abs(me.dtheta.sum() - 2 * np.pi) < 1e-13
    assert np.all(volumes(me) > 0)


def test_stretch_formulas_match_paper():
    # (2.4): υ(s) = sin(s^p π/2); §3.1 angular v(ι) = 2π sin((ι/2π)^q π/2);
    # (2.13): φ(s) = 1 - (1-s)^{p+1}; §3.1 V(t) = T sin((t/T)^l π/2)
    m, n = 9, 12
    me = make_mesh(m, n, 1, 1.7, 1, 2.3)
    s = np.arange(1, m + 1) / (m + 1)
    assert np.allclose(me.r[1:-1], np.sin(s ** 1.7 * np.pi / 2), rtol=0, atol=1e-15)
    io = 2 * np.pi * np.arange(1, n) / n
    assert np.allclose(me.th[1:-1], 2 * np.pi * np.sin((io / (2 * np.pi)) ** 2.3 * np.pi / 2),
                       rtol=0, atol=1e-14)
    me3 = make_mesh(m, n, 3, 0.6)
    assert np.allclose(me3.r[1:-1], 1 - (1 - s) ** 1.6, rtol=0, atol=1e-15)
    t = time_levels(0.05, 100, 1, 1.5)
    assert t[-1] == 0.05 and np.all(np.diff(t) > 0)
    dt = np.diff(t)
    # the cfg2 schedule: steps between 1.38e-5 and 7.08e-4
    assert 1.3e-5 < dt.min() < 1.4e-5 and 7.0e-4 < dt.max() < 7.1e-4


# ----------------------------------------------------------------- P2

def paper_p_h_dense(me, b_grid, b0):
    """℘_h of §2.1 typed from its printed coefficients (uniform θ)."""
    m, n = me.m, me.n
    r, h = me.r, me.h
    rh = me.r_half
    mu = 2 * np.pi / n
    N = m * n + 1
    A = np.zeros((N, N))
    for i in range(1, m + 1):
        for j in range(n):
            P = idx(m, i, j)
            s = h[i] + h[i + 1]
            A[P, P] += (2.0 / (r[i] * s) * (rh[i] / h[i + 1] + rh[i - 1] / h[i])
                        + 2.0 / (r[i] ** 2 * mu ** 2) + b_grid[i - 1, j])
            west = 0 if i == 1 else idx(m, i - 1, j)
            A[P, west] += -2.0 * rh[i - 1] / (r[i] * h[i] * s)
            if i < m:
                A[P, idx(m, i + 1, j)] += -2.0 * rh[i] / (r[i] * h[i + 1] * s)
            A[P, idx(m, i, (j - 1) % n)] += -1.0 / (r[i] ** 2 * mu ** 2)
            A[P, idx(m, i, (j + 1) % n)] += -1.0 / (r[i] ** 2 * mu ** 2)
    A[0, 0] = 4.0 / h[1] ** 2 + b0
    for j in range(n):
        A[0, idx(m, 1, j)] = -4.0 / (n * h[1] ** 2)
    return A


@pytest.mark.parametrize("r_kind,p", [(0, 1.0), (1, 1.0), (1, 1.4), (3, 0.6)])
def test_p2_flux_form_equals_printed_p_h(r_kind, p):
    pb = parabolic_family(1.0, 0.3)
    pb.b = lambda r, th: 0.5 + r * np.cos(th) ** 2
    S, me = build(pb, 7, 12, r_kind, p)
    ref = paper_p_h_dense(me, S.data["b_grid"], S.data["b_origin"])
    got = S.L.toarray()
    scale = np.abs(ref).max()
    assert np.abs(got - ref).max() <= 1e-15 * scale * 8
    # boundary coupling: the (m+1) neighbour of ring m
    m = me.m
    s = me.h[m] + me.h[m + 1]
    cb = -2.0 * me.r_half[m] / (me.r[m] * me.h[m + 1] * s)
    assert np.allclose(S.c_bnd, cb, rtol=1e-14, atol=0)


def test_p2_flux_form_equals_printed_varpi_without_drift():
    # E = 0, uniform θ and D constant on the origin faces: the flux form is
    # the printed ϖ_h of §3.2.1 and the origin row of §3.2.2.
    pb = continuity_cfg(1234, 6, 10)
    pb.Er = pb.Et = None
    pb.E_scalar = lambda r, th: 0.0 * r
    pb.D = lambda r, th: np.where(r < 0.05, 1.0 + 0 * th, 1.0 + 0.3 * r * np.sin(th) + 0.1 * r)
    me = make_mesh(6, 10, 1, 1.2, 0, 1.0)
    d = sample(pb, *me.sample_points())
    d["D_r"][0, :] = d["D_origin"]
    F = assemble(me, d).L.toarray()
    Lit = assemble_literal(me, d).L.toarray()
    assert np.abs(F - Lit).max() <= 1e-14 * np.abs(Lit).max()


# ----------------------------------------------------------------- P1

@pytest.mark.parametrize("m,n,th_kind,q,theta,K", [
    (4, 8, 0, 1.0, 0.5, 5), (8, 16, 1, 1.7, 1.0, 7), (5, 9, 1, 2.5, 0.37, 4), (33, 64, 0, 1.0, 0.6, 10)])
def test_p1_closed_form_is_reproduced_exactly(m, n, th_kind, q, theta, K):
    pb = closed_form_quadratic(0.25)
    S, me = build(pb, m, n, 0, 1.0, th_kind, q)
    t = time_levels(0.3, K, 1, 1.5)        # non-uniform steps too
    x = solve(S, t, theta)
    e0, eg = exact_at(pb, t[-1], me.r, me.th)
    ex = to_vec(e0, eg)
    assert np.max(np.abs(x - ex)) / np.max(np.abs(ex)) < 2e-13


def test_p1_exactness_needs_the_origin_closure():
    # A wrong origin row (factor 4 -> 2) destroys exactness: the pin is sharp.
    pb = closed_form_quadratic(0.25)
    S, me = build(pb, 6, 12)
    L = S.L.tolil()
    L[0, 0] = L[0, 0] * 0.5
    S.L = L.tocsr()
    x = solve(S, time_levels(0.3, 5), 0.5)
    e0, eg = exact_at(pb, 0.3, me.r, me.th)
    assert np.max(np.abs(x - to_vec(e0, eg))) > 1e-4


# ----------------------------------------------------------------- P4

@pytest.mark.parametrize("flux,theta,r_kind,th_kind", [(0, 0.5, 1, 1), (1, 1.0, 1, 0), (0, 1.0, 0, 1),
                                                       (1, 0.5, 3, 1)])
def test_p4_mass_is_conserved_under_zero_flux(flux, theta, r_kind, th_kind):
    pb = zero_flux_random(7)
    S, me = build(pb, 12, 20, r_kind, 1.3 if r_kind == 1 else 0.6, th_kind, 1.6, flux=flux, bc=1)
    t = time_levels(0.02, 6, 1, 1.5)
    x0 = S.initial()
    x = solve(S, t, theta)
    M0, M1 = S.V @ x0, S.V @ x
    assert abs(M1 - M0) / abs(M0) < 1e-13
    # and the column sums of V·L vanish (every face flux leaves one cell and enters another)
    col = np.asarray((sp.diags(S.V) @ S.L).sum(axis=0)).ravel()
    assert np.abs(col).max() < 1e-12 * np.abs(S.L.diagonal() * S.V).max()


def test_p4_conservation_detects_a_non_conservative_origin():
    # The printed origin row (weights 1/n with D_00 at the node) on a
    # non-uniform θ mesh does not conserve mass; the flux form does.
    pb = zero_flux_random(3)
    pb.Er = pb.Et = None
    pb.E_scalar = lambda r, th: 0.0 * r
    me = make_mesh(10, 16, 1, 1.3, 1, 2.0)
    d = sample(pb, *me.sample_points())
    lit = assemble_literal(me, d)
    col = np.asarray((sp.diags(lit.V) @ lit.L).sum(axis=0)).ravel()
    col[lit.bnd_rows()] = 0.0
    assert np.abs(col).max() > 1e-6


# ----------------------------------------------------------------- P5

@pytest.mark.parametrize("seed", [1, 2, 3])
def test_p5_maximum_principle_parabolic_backward_euler(seed):
    pb = random_positive(seed, pde=0)
    pb.modes[0].nb = lambda th: -0.3 + 1.1 * np.cos(2 * th) ** 2
    S, me = build(pb, 14, 24, 1, 1.3, 1, 1.5)
    x = S.initial()
    t = time_levels(0.01, 8, 0)
    for k in range(8):
        g = S.boundary(t[k + 1])
        lo = min(0.0, x.min(), g.min())
        hi = max(0.0, x.max(), g.max())
        x = step(S, x, t[k], t[k + 1], 1.0)
        assert x.min() >= lo - 1e-13 and x.max() <= hi + 1e-13


@pytest.mark.parametrize("seed", [4, 5])
def test_p5_positivity_continuity_upwind_backward_euler(seed):
    pb = random_positive(seed, pde=1)
    S, me = build(pb, 14, 24, 1, 1.3, 1, 1.5, flux=1)
    x = solve(S, time_levels(0.05, 10, 1, 1.5), 1.0)
    assert x.min() >= -1e-14


# ----------------------------------------------------------------- P9

@pytest.mark.parametrize("flux", [0, 1])
def test_p9_m_matrix_structure(flux):
    pb = continuity_cfg(1300, 24, 48)
    S, me = build(pb, 24, 48, 1, 1.3, flux=flux)
    dt, theta = 1e-3, 0.5
    A = system_matrix(S, dt, theta).tocsr()
    off = A - sp.diags(A.diagonal())
    assert off.data.max() <= 0.0
    assert A.diagonal().min() > 0
    col = np.asarray((sp.diags(S.V) @ A).sum(axis=0)).ravel()
    assert np.all(col >= S.V / dt * (1 - 1e-12))


# ----------------------------------------------------------------- P7

def brute_operator(me, d, x, flux):
    """(L x) for every cell by walking its four faces (plain loops)."""
    m, n = me.m, me.n
    r, h = me.r, me.h
    rh, mu, dth = me.r_half, me.mu, me.dtheta
    V = volumes(me)
    o, g = from_vec(x, m, n)
    xv = lambda i, j: o if i == 0 else (0.0 if i == m + 1 else g[i - 1, j % n])
    out = np.zeros_like(x)

    def F(G, K, a, b):
        if flux == 0:
            return G * (a - b) + K * 0.5 * (a + b)
        return G * (a - b) + max(K, 0) * a + min(K, 0) * b

    acc0 = 0.0
    for j in range(n):
        acc0 += F(d["D_r"][0, j] * rh[0] * dth[j] / h[1], d["Er_r"][0, j] * rh[0] * dth[j], o, g[0, j])
    out[0] = acc0 / V[0] + d["b_origin"] * o
    for i in range(1, m + 1):
        for j in range(n):
            tot = 0.0
            # outward through the outer radial face
            tot += F(d["D_r"][i, j] * rh[i] * dth[j] / h[i + 1], d["Er_r"][i, j] * rh[i] * dth[j],
                     xv(i, j), xv(i + 1, j))
            # inner face: flux from (i-1) to (i) counts negatively
            tot -= F(d["D_r"][i - 1, j] * rh[i - 1] * dth[j] / h[i],
                     d["Er_r"][i - 1, j] * rh[i - 1] * dth[j], xv(i - 1, j), xv(i, j))
            w = 0.5 * (h[i] + h[i + 1])
            tot += F(d["D_t"][i - 1, j] * w / (r[i] * mu[j + 1]), d["Et_t"][i - 1, j] * w,
                     xv(i, j), xv(i, j + 1))
            jm = (j - 1) % n
            tot -= F(d["D_t"][i - 1, jm] * w / (r[i] * mu[jm + 1]), d["Et_t"][i - 1, jm] * w,
                     xv(i, jm), xv(i, j))
            out[idx(m, i, j)] = tot / V[idx(m, i, j)] + d["b_grid"][i - 1, j] * xv(i, j)
    return out


@pytest.mark.parametrize("m,n,flux", [(2, 4, 0), (3, 5, 1), (4, 8, 0), (4, 8, 1)])
def test_p7_brute_force_dense(m, n, flux):
    pb = continuity_cfg(1400 + m, m, n)
    pb.b = lambda r, th: 0.2 + 0.1 * np.cos(th)
    me = make_mesh(m, n, 1, 1.3, 1, 1.6)
    d = sample(pb, *me.sample_points())
    S = assemble(me, d, flux=flux)
    N = S.N
    dense = np.column_stack([brute_operator(me, d, e, flux) for e in np.eye(N)])
    assert np.abs(dense - S.L.toarray()).max() <= 1e-13 * np.abs(dense).max()
    # one step: dense solve of (I/dt + θL) vs the sparse LU
    x0 = S.initial()
    dt, theta = 3e-3, 0.5
    b = rhs(S, x0, 0.0, dt, theta)
    xd = np.linalg.solve(np.eye(N) / dt + theta * dense, b)
    xs = step(S, x0, 0.0, dt, theta)
    assert np.abs(xd - xs).max() <= 1e-13 * np.abs(xd).max()


# ----------------------------------------------------------------- P6

def rate(errs, hs):
    return np.polyfit(np.log(hs), np.log(errs), 1)[0]


@pytest.mark.slow
def test_p6_space_order_parabolic_uniform():
    pb = parabolic_family(1.0, 0.5)
    errs, hs = [], []
    for m in (16, 32, 64, 128):
        S, me = build(pb, m, 2 * m)
        x = solve(S, time_levels(0.05, 200), 0.5)
        errs.append(max_err(x, pb, 0.05, me))
        hs.append(1.0 / (m + 1))
    assert 1.85 <= rate(errs, hs) <= 2.15


@pytest.mark.slow
def test_p6_space_order_continuity_graded():
    pb = continuity_cfg(1201, 8, 8)
    errs, hs = [], []
    for m in (16, 32, 64):
        S, me = build(pb, m, 2 * m, 1, 1.3)
        x = solve(S, time_levels(0.02, 80), 0.5)
        errs.append(max_err(x, pb, 0.02, me))
        hs.append(1.0 / (m + 1))
    assert rate(errs, hs) >= 1.7


@pytest.mark.slow
@pytest.mark.parametrize("theta,expect", [(0.5, 2.0), (1.0, 1.0)])
def test_p6_time_order(theta, expect):
    pb = continuity_cfg(1202, 12, 24)
    S, me = build(pb, 12, 24, 1, 1.3)
    T = 0.2
    ref = solve(S, time_levels(T, 8192), theta)
    errs, dts = [], []
    # Crank-Nicolson damps stiff modes poorly, so its rate is asymptotic only
    # once Δt is well below the mesh's stiff time scale: start at T/64.
    for K in (64, 128, 256):
        x = solve(S, time_levels(T, K), theta)
        errs.append(np.max(np.abs(x - ref)))
        dts.append(T / K)
    assert abs(rate(errs, dts) - expect) <= 0.15


# ----------------------------------------------------------------- P3

def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


@pytest.mark.slow
@pytest.mark.parametrize("m", [19, 39, 59])
def test_p3_table_2_1(m):
    g = _golden("table_2_1.json")["rows"][str(m)]
    n = int(np.floor(2 * np.pi * m))
    pb = paper_parabolic_ex1()
    tol = [0.025, 0.005, 0.05]   # (2.4) within 2.5%, uniform r within 0.5%, (2.13) within 5%
    for col, (rk, p) in enumerate([(1, 1.0), (0, 1.0), (3, 0.6)]):
        S, me = build(pb, m, n, rk, p)
        x = solve(S, time_levels(0.1, 10), 0.6)
        e = max_err(x, pb, 0.1, me)
        assert abs(e / g[col] - 1) <= tol[col], (m, col, e, g[col])


@pytest.mark.slow
@pytest.mark.parametrize("m", [19, 39])
def test_p3_table_3_1_literal_stencil(m):
    g = _golden("table_3_1.json")["rows"][str(m)]
    n = int(np.floor(2 * np.pi * m))
    pb = paper_continuity_ex1()
    for col, (rk, p, tk, q) in enumerate([(1, 0.1, 1, 1.9), (1, 0.1, 0, 1.0), (0, 1.0, 1, 1.9)]):
        S, me = build(pb, m, n, rk, p, tk, q, literal=True)
        x = solve(S, time_levels(0.1, 10, 1, 1.5), 0.5)
        e = max_err(x, pb, 0.1, me, skip_origin=True)
        assert abs(e / g[col] - 1) <= 0.01, (m, col, e, g[col])
