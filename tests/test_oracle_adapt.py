"""Pins of the oracle's error indicator, stretch choice and transfer
(closed forms of divided differences, exactness of cubic interpolation,
its fourth order, and that a recommended stretch lowers the indicator)."""

import numpy as np
import pytest

from oracle import make_mesh
from oracle.adapt import choose_stretch, indicator, predicted_max, second_differences, transfer
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


def hand_nodes(m, p):
    """Nodes of the stretch (2.4) written out with math.sin, node by node."""
    import math
    h = 1.0 / (m + 1)
    r = [0.0] + [math.sin((k * h) ** p * math.pi / 2.0) for k in range(1, m + 1)] + [1.0]
    return r


@pytest.mark.parametrize("rk,p", [(0, 1.0), (1, 1.3), (1, 0.8)])
def test_indicator_of_a_radial_quadratic(rk, p):
    """n = a r² + c: δ_r² n = 2a exactly and δ_θ² n = 0, so the indicator is
    η_ij = ((r_{i+1} - r_{i-1})/2)² · 2|a| (on a uniform mesh 2|a| h²), and
    κ_i = 2|a|.  A wrong local spacing (h_i or h_{i+1} in place of their
    mean) fails on the graded meshes."""
    m, n, a, c = 13, 10, -1.3, 0.7
    me = make_mesh(m, n, rk, p)
    x = to_vec(c, grid_values(me, lambda R, T: a * R ** 2 + c))
    eta, kappa = indicator(me, x, nb=np.full(n, a + c))
    r = me.r
    for i in range(1, m + 1):
        want = ((r[i + 1] - r[i - 1]) / 2.0) ** 2 * 2.0 * abs(a)
        assert np.allclose(eta[i - 1], want, rtol=1e-9, atol=0), (i, eta[i - 1, 0], want)
    if rk == 0:
        assert np.allclose(eta, 2 * abs(a) / (m + 1) ** 2, rtol=1e-9)
    assert np.allclose(kappa, 2 * abs(a), rtol=1e-9)


def test_indicator_of_r2_cos_k_theta():
    """n = r² cos kθ on a uniform mesh: δ_r² n = 2 cos kθ_j and
    δ_θ² n = r_i² (2 cos kμ - 2)/μ² cos kθ_j exactly, so
    η_ij = |cos kθ_j| max(2 ĥ², r_i² |2 cos kμ - 2|) (ĥ = h, Δθ = μ) and
    κ_i = 2 max_j |cos kθ_j|.  The angular part decides near r = 1, the
    radial part near the origin."""
    m, n, k = 9, 12, 2
    me = make_mesh(m, n, 0, 1.0)
    h, mu = 1.0 / (m + 1), 2 * np.pi / n
    x = to_vec(0.0, grid_values(me, lambda R, T: R ** 2 * np.cos(k * T)))
    thj = 2 * np.pi * np.arange(n) / n
    eta, kappa = indicator(me, x, nb=np.cos(k * thj))
    for i in range(1, m + 1):
        ri = i * h
        want = np.abs(np.cos(k * thj)) * max(2 * h * h, ri * ri * abs(2 * np.cos(k * mu) - 2))
        assert np.allclose(eta[i - 1], want, rtol=1e-9, atol=1e-15), i
    assert np.allclose(kappa, 2 * np.max(np.abs(np.cos(k * thj))), rtol=1e-9)


def test_predicted_max_for_constant_curvature():
    """κ ≡ K0: P(p) = K0 · max_k ((r'_{k+1} - r'_{k-1})/2)² over the nodes
    of the stretch (2.4), computed here node by node.  Using h_{k+1} in
    place of the mean spacing fails."""
    old = make_mesh(20, 8, 0, 1.0)
    K0 = 3.5
    for p, m_new in ((1.0, 20), (1.3, 31), (2.0, 17)):
        r = hand_nodes(m_new, p)
        want = K0 * max(((r[k + 1] - r[k - 1]) / 2.0) ** 2 for k in range(1, m_new + 1))
        got = predicted_max(old.r, np.full(20, K0), m_new, p)
        assert got == pytest.approx(want, rel=1e-12), (p, got, want)


def test_predicted_max_for_linear_curvature():
    """κ linear in r between the outermost old nodes (and constant beyond
    them): P(p) = max_k ĥ'_k² κ(r'_k) with κ evaluated at the new node
    itself.  Sampling κ at a neighbouring node fails."""
    m_old = 25
    old = make_mesh(m_old, 8, 1, 1.1)
    al, be = 0.4, 5.0
    rin = old.r[1:m_old + 1]
    kappa = al + be * rin
    for p, m_new in ((1.3, 25), (0.9, 40)):
        r = hand_nodes(m_new, p)
        vals = []
        for k in range(1, m_new + 1):
            rk = min(max(r[k], rin[0]), rin[-1])
            vals.append(((r[k + 1] - r[k - 1]) / 2.0) ** 2 * (al + be * rk))
        got = predicted_max(old.r, kappa, m_new, p)
        assert got == pytest.approx(max(vals), rel=1e-12), p


def test_choose_stretch_picks_the_smallest_prediction():
    """κ ≡ 1 and candidates 1 and 5: the stretch (2.4) with p = 1 has its
    largest spacing at the origin, about (π/2) h, while p = 5 reaches about
    3 h near s = 0.9, so p = 1 is chosen, and from p = 5 a remesh is
    recommended.  Among equal predictions the first candidate wins, and the
    recommendation needs P(best) <= 0.8 P(current)."""
    me = make_mesh(30, 8, 1, 5.0)
    kap = np.ones(30)
    best, pb, pc, rec = choose_stretch(me, kap, 5.0, [5.0, 1.0])
    h = 1.0 / 31
    assert best == 1.0 and rec
    assert pb == pytest.approx(max(((a - b) / 2) ** 2 for a, b in
                                   zip(hand_nodes(30, 1.0)[2:], hand_nodes(30, 1.0)[:-2])), rel=1e-12)
    assert 1.4 * h < np.sqrt(pb) < 1.6 * h and np.sqrt(pc) > 2.5 * h
    # the first of equal candidates; no recommendation when nothing improves
    best, pb, pc, rec = choose_stretch(me, kap, 1.0, [1.0, 1.0, 5.0])
    assert best == 1.0 and pb == pc and not rec


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
