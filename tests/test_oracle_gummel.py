"""Pins of the oracle's two-carrier coupling (oracle/gummel.py): the polar
Poisson problem is exact on quadratics, the face drift of a quadratic
potential is the exact field and that of a linear one converges to it at
second order, a more negative charge lowers the potential, the coupled step
conserves each carrier under zero flux, and a converged Gummel step is a
fixed point of its two halves."""

import numpy as np
import pytest

from oracle import make_mesh
from oracle.gummel import boundary_psi, carrier_system, drift_faces, gummel_step, poisson_system, solve_poisson
from oracle.operator import from_vec, to_vec, volumes
from oracle.stepper import step
from problems import Problem, TimeMode, sample, two_carrier


def quad_psi_problem(eps, a, c0):
    """ψ = a r² + c0: -∇·(ε∇ψ) = -4εa, ψ = a + c0 on r = 1."""
    const = lambda v: (lambda r, th: np.full(np.broadcast(r, th).shape, float(v)))
    return Problem(name="quad_psi", pde=1,
                   modes=[TimeMode(0.0, 0, const(0.0), lambda th: np.full(np.shape(th), a + c0)),
                          TimeMode(0.0, 0, const(-4.0 * eps * a), lambda th: np.zeros(np.shape(th)))],
                   u0=const(0.0), D=const(eps))


@pytest.mark.parametrize("m,n,tk,q", [(14, 30, 0, 1.0), (9, 40, 1, 1.6), (21, 16, 1, 0.8)])
def test_poisson_is_exact_on_a_quadratic(m, n, tk, q):
    """On a uniform radial mesh (any angular one) the scheme is exact for
    radial quadratics, the origin row included (as pin P1 for the heat
    operator); a wrong sign of the doping or of the boundary term fails."""
    me = make_mesh(m, n, 0, 1.0, tk, q)
    eps, a, c0 = 0.3, 0.8, -0.2
    S = poisson_system(me, sample(quad_psi_problem(eps, a, c0), *me.sample_points()))
    psi = solve_poisson(S, np.zeros(S.N))
    o, g = from_vec(psi, me.m, me.n)
    assert abs(o - c0) <= 1e-12
    assert np.max(np.abs(g - (a * me.r[1:-1, None] ** 2 + c0))) <= 1e-12


def test_drift_of_a_quadratic_potential_is_the_exact_field():
    """ψ = a r²: the radial face field (ψ_i - ψ_{i+1})/h_{i+1} is -2a r_{i+1/2}
    exactly, and the angular one vanishes."""
    me = make_mesh(10, 20, 1, 1.3, 1, 1.6)
    a, s = 0.7, -1.0
    psi = to_vec(0.0, a * me.r[1:-1, None] ** 2 * np.ones((1, me.n)))
    mu_r = np.full((me.m + 1, me.n), 2.0)
    mu_t = np.full((me.m, me.n), 2.0)
    Er, Et = drift_faces(me, psi, np.full(me.n, a), mu_r, mu_t, s)
    assert np.allclose(Er, s * 2.0 * (-2.0 * a * me.r_half[:, None]), rtol=1e-13, atol=1e-15)
    assert np.all(Et == 0.0)


def test_angular_drift_of_a_linear_potential_converges_at_second_order():
    """ψ = b x = b r cos θ: the exact angular field is -(1/r)∂ψ/∂θ = b sin θ at
    the face θ_{j+1/2}; the face difference approaches it as μ²."""
    b, s = 1.3, 1.0
    errs = []
    for n in (16, 32, 64):
        me = make_mesh(6, n, 0, 1.0, 0, 1.0)
        R, T = me.r[1:-1, None], me.th[None, :-1]
        psi = to_vec(0.0, b * R * np.cos(T))
        _, Et = drift_faces(me, psi, b * np.cos(me.th[:-1]), np.ones((7, n)), np.ones((6, n)), s)
        errs.append(np.max(np.abs(Et - s * b * np.sin(me.th_half[None, :]))))
    rate = np.log(errs[0] / errs[2]) / np.log(4.0)
    assert 1.9 <= rate <= 2.1, errs


def test_more_electrons_lower_the_potential():
    psi_pb, _, _ = two_carrier(21)
    me = make_mesh(12, 24, 1, 1.3)
    S = poisson_system(me, sample(psi_pb, *me.sample_points()))
    base = solve_poisson(S, np.zeros(S.N))
    bump = np.zeros(S.N)
    bump[1:] = 0.1                          # extra electrons: charge p - n lower
    lower = solve_poisson(S, -bump)
    assert np.all(lower < base)


def setup(seed, m=12, n=24, zero_flux=False):
    psi_pb, n_pb, p_pb = two_carrier(seed, zero_flux=zero_flux)
    me = make_mesh(m, n, 1, 1.3)
    pts = me.sample_points()
    dpsi, dn, dp = sample(psi_pb, *pts), sample(n_pb, *pts), sample(p_pb, *pts)
    S = poisson_system(me, dpsi)
    init = [to_vec(d["u0_origin"], d["u0_grid"]) for d in (dpsi, dn, dp)]
    return me, S, dn, dp, init


def test_zero_flux_step_conserves_each_carrier():
    me, S, dn, dp, (psi, n, p) = setup(22, zero_flux=True)
    V = volumes(me)
    psi2, n2, p2, it, _ = gummel_step(me, S, dn, dp, psi, n, p, 0.0, 0.02, 1.0, 4, bc=1)
    assert abs(V @ n2 / (V @ n) - 1) <= 1e-12
    assert abs(V @ p2 / (V @ p) - 1) <= 1e-12
    assert np.max(np.abs(n2 - n)) > 1e-4          # the carriers did move


def test_converged_step_is_a_fixed_point():
    me, S, dn, dp, (psi, n, p) = setup(23)
    psi2, n2, p2, it, change = gummel_step(me, S, dn, dp, psi, n, p, 0.0, 0.01, 0.5, 60, tol=1e-13)
    assert it < 60 and change <= 1e-13
    # ψ solves Poisson with the returned carriers to the stopping tolerance
    psi_fix = solve_poisson(S, p2 - n2)
    assert np.max(np.abs(psi_fix - psi2)) <= 1e-11 * np.max(np.abs(psi2))
    # and each carrier is the θ-step under the drift of that ψ
    psi_b = boundary_psi(S)
    n_fix = step(carrier_system(me, dn, psi2, psi_b, -1.0), n, 0.0, 0.01, 0.5)
    p_fix = step(carrier_system(me, dp, psi2, psi_b, +1.0), p, 0.0, 0.01, 0.5)
    assert np.max(np.abs(n_fix - n2)) <= 1e-11 * np.max(np.abs(n2))
    assert np.max(np.abs(p_fix - p2)) <= 1e-11 * np.max(np.abs(p2))
    # the electrons' drift sign matters: with both carriers drifting alike
    # the result differs
    n_same = step(carrier_system(me, dn, psi2, psi_b, +1.0), n, 0.0, 0.01, 0.5)
    assert np.max(np.abs(n_same - n2)) > 1e-6
