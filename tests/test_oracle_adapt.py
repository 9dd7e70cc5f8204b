"""Pins of the oracle's error indicator, stretch choice and transfer
(closed forms of divided differences, exactness of cubic interpolation,
its fourth order, and that a recommended stretch lowers the indicator)."""

import numpy as np
import pytest

from oracle import make_mesh
from oracle.adapt import choose_stretch, indicator, second_differences, transfer
from oracle.operator import to_vec


def grid_values(me, f):
    R, TH = np.meshgrid(me.r[1:me.m + 1], me.th[:me.n], indexing="ij")
    return f(R, TH)


@pytest.mark.parametrize("rk,p,tk,q", [(0, 1.0, 0, 1.0), (1, 1.3, 0, 1.0), (1, 0.7, 1, 1.4)])
def test_radial_second_difference_of_a_quadratic_is_exact(rk, p, tk, q):
    """δ_r² of a r² + c is 2a on any node spacing (origin value c, boundary a + c)."""
    me = make_mesh(11, 14, rk, p, tk, q)
    a, c = 1.7, -0.4
    x = to_vec(c, grid_values(me, lambda R, T: a * R ** 2 + c))
    d2r, d2t = second_differences(me, x, nb=np.full(me.n, a + c))
    assert np.allclose(d2r, 2 * a, rtol=1e-12, atol=1e-11)
    assert np.allclose(d2t, 0.0, atol=1e-11)


def test_angular_second_difference_closed_form():
    """Uniform θ: δ_θ² cos(kθ) = (2 cos(kμ) - 2)/μ² cos(kθ)."""
    me = make_mesh(6, 20, 0, 1.0)
    k, mu = 3, 2 * np.pi / 20
    x = to_vec(0.0, grid_values(me, lambda R, T: np.cos(k * T)))
    _, d2t = second_differences(me, x, nb=np.zeros(me.n))
    expect = (2 * np.cos(k * mu) - 2) / mu ** 2 * np.cos(k * me.th[:20])
    assert np.allclose(d2t, expect[None, :], rtol=1e-12, atol=1e-12)


def test_indicator_combines_directions():
    me = make_mesh(9, 16, 1, 1.2)
    rng = np.random.default_rng(3)
    x = rng.standard_normal(9 * 16 + 1)
    nb = rng.standard_normal(16)
    eta, kappa = indicator(me, x, nb)
    d2r, d2t = second_differences(me, x, nb)
    h = me.h
    hl = 0.5 * (h[1:10] + h[2:11])
    assert np.allclose(eta, np.maximum(hl[:, None] ** 2 * abs(d2r), me.dtheta[None, :] ** 2 * abs(d2t)))
    assert np.allclose(kappa, abs(d2r).max(axis=1))


def test_transfer_onto_the_same_mesh_is_the_identity():
    me = make_mesh(10, 12, 1, 1.3)
    rng = np.random.default_rng(1)
    x = rng.standard_normal(10 * 12 + 1)
    y = transfer(me, x, me, nb=rng.standard_normal(12))
    assert np.allclose(y, x, rtol=0, atol=1e-13)


@pytest.mark.parametrize("with_boundary", [True, False])
def test_transfer_reproduces_radial_cubics(with_boundary):
    """A cubic in r (constant in θ) is carried exactly to another stretch."""
    old, new = make_mesh(12, 10, 1, 1.0), make_mesh(17, 10, 1, 1.6)
    f = lambda R, T: 1.0 + 2.0 * R - R ** 2 + 0.5 * R ** 3  # noqa: E731
    x = to_vec(1.0, grid_values(old, f))
    nb = np.full(10, f(1.0, 0.0)) if with_boundary else None
    y = transfer(old, x, new, nb)
    assert np.allclose(y, to_vec(1.0, grid_values(new, f)), rtol=0, atol=1e-13)


def test_transfer_is_fourth_order():
    f = lambda R, T: np.exp(-R) * (1 + 0.3 * R * np.cos(T)) + 0.2 * R ** 2 * np.sin(2 * T)  # noqa: E731
    errs = []
    for m in (16, 32, 64):
        old, new = make_mesh(m, 2 * m, 1, 1.1), make_mesh(m + 3, 2 * m + 6, 1, 1.4)
        x = to_vec(f(0.0, 0.0), grid_values(old, f))
        nb = f(1.0, old.th[:old.n])
        y = transfer(old, x, new, nb)
        errs.append(np.max(np.abs(y - to_vec(f(0.0, 0.0), grid_values(new, f)))))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 3.5), rates


def test_recommended_stretch_lowers_the_indicator():
    """A layer at the origin: the recommended exponent grades towards r = 0,
    and the transferred state's largest indicator drops."""
    me = make_mesh(40, 32, 1, 1.0)
    f = lambda R, T: np.exp(-R / 0.05) + 0.1 * np.cos(T) * R  # noqa: E731
    x = to_vec(1.0, grid_values(me, f))
    nb = f(1.0, me.th[:me.n])
    eta, kappa = indicator(me, x, nb)
    p_best, pb, pc, rec = choose_stretch(me, kappa, 1.0, [0.6, 0.8, 1.0, 1.3, 1.6, 2.0, 2.5])
    assert rec and p_best > 1.0 and pb < pc
    new = make_mesh(40, 32, 1, p_best)
    y = transfer(me, x, new, nb)
    eta_new, _ = indicator(new, y, nb)
    assert eta_new.max() < 0.8 * eta.max()
