"""Error indicator, mesh choice and solution transfer (oracle; test
infrastructure only).

The paper builds its adaptivity into the choice of the stretch (2.4): the
exponent p ties the radial grading to the solution's regularity (α = pσ of
Theorem 2.1), and it leaves open how a run should pick or change it (the
outlook of §4.2).  What follows is the plain definition this build reads
into that gap, written out without blocking or fusion:

Indicator at ring node (i, j), i = 1..m, from the second divided
differences of the discrete solution on the non-uniform mesh,
    δ_r² n = 2 [ (n_{i+1,j} - n_{i,j})/h_{i+1} - (n_{i,j} - n_{i-1,j})/h_i ] / (h_i + h_{i+1}),
    δ_θ² n = 2 [ (n_{i,j+1} - n_{i,j})/μ_{j+1} - (n_{i,j} - n_{i,j-1})/μ_j ] / (μ_j + μ_{j+1}),
where ring 0 is the origin value, ring m+1 the Dirichlet value N(t, θ_j)
(for zero flux, ring m+1 repeats ring m) and j wraps around the period;
    η_ij = max( ĥ_i² |δ_r² n|,  Δθ_j² |δ_θ² n| ),   ĥ_i = (h_i + h_{i+1})/2,
                                                    Δθ_j = (μ_j + μ_{j+1})/2,
(a local estimate of the second-order truncation error in each direction,
the angular one measured in arc length r_i Δθ_j against the 1/r² of the
operator).  Radial curvature profile κ_i = max_j |δ_r² n|.

Mesh choice among radial stretches (2.4) with exponents p_c: the predicted
largest radial indicator of the stretch with exponent p is
    P(p) = max_k ĥ'_k² κ(r'_k),
with r'_k its nodes, ĥ'_k its local spacing and κ interpolated linearly in
r from (r_i, κ_i); the choice is the candidate with the smallest P (the
first of equal ones), recommended when P(best) <= 0.8 P(current).

Transfer of a state to another mesh: tensor-product cubic Lagrange
interpolation, first along each old θ-line in r on the nodes r_0 = 0 (the
origin value), r_1..r_m and, for Dirichlet data, r_{m+1} = 1 (the boundary
value), then periodically in θ; each target point uses the four
consecutive nodes whose middle interval holds it (shifted inwards at the
ends of a line).  The origin value is kept.
"""

from __future__ import annotations

import numpy as np

from .mesh import Mesh, radial_nodes
from .operator import from_vec, to_vec


def second_differences(me: Mesh, x, nb=None):
    """(δ_r² n, δ_θ² n) at every ring node, shape (m, n); x in paper order,
    nb the Dirichlet values at r = 1 (None for zero flux)."""
    m, n = me.m, me.n
    n0, U = from_vec(x, m, n)            # U[i-1, j]
    h = me.h
    mu = me.mu
    d2r = np.zeros((m, n))
    d2t = np.zeros((m, n))
    for i in range(1, m + 1):
        for j in range(n):
            c = U[i - 1, j]
            below = n0 if i == 1 else U[i - 2, j]
            if i < m:
                above = U[i, j]
            else:
                above = nb[j] if nb is not None else c
            d2r[i - 1, j] = 2.0 * ((above - c) / h[i + 1] - (c - below) / h[i]) / (h[i] + h[i + 1])
            left = U[i - 1, (j - 1) % n]
            right = U[i - 1, (j + 1) % n]
            d2t[i - 1, j] = 2.0 * ((right - c) / mu[j + 1] - (c - left) / mu[j]) / (mu[j] + mu[j + 1])
    return d2r, d2t


def indicator(me: Mesh, x, nb=None):
    """η (m, n) and the radial curvature profile κ (m)."""
    d2r, d2t = second_differences(me, x, nb)
    h = me.h
    hloc = 0.5 * (h[1:me.m + 1] + h[2:me.m + 2])          # ĥ_i, i = 1..m
    dth = me.dtheta                                        # Δθ_j
    eta = np.maximum(hloc[:, None] ** 2 * np.abs(d2r), dth[None, :] ** 2 * np.abs(d2t))
    kappa = np.abs(d2r).max(axis=1)
    return eta, kappa


def predicted_max(r_old, kappa, m_new, p):
    """P(p): largest ĥ'² κ(r') over the nodes of the stretch (2.4) with exponent p."""
    r = radial_nodes(m_new, 1, p)
    h = np.diff(r)
    hloc = 0.5 * (h[:-1] + h[1:])                          # nodes 1..m
    kap = np.interp(r[1:-1], r_old[1:-1], kappa)
    return float(np.max(hloc ** 2 * kap))


def choose_stretch(me: Mesh, kappa, p_current, candidates, m_new=None):
    """(best p, P(best), P(current), recommended)."""
    m_new = me.m if m_new is None else m_new
    cur = predicted_max(me.r, kappa, m_new, p_current)
    best_p, best = None, np.inf
    for p in candidates:
        v = predicted_max(me.r, kappa, m_new, p)
        if v < best:
            best_p, best = float(p), v
    return best_p, best, cur, bool(best <= 0.8 * cur)


def _lagrange4(xs, ys, x):
    """Cubic Lagrange polynomial through four points, evaluated at x."""
    total = 0.0
    for a in range(4):
        w = 1.0
        for b in range(4):
            if b != a:
                w *= (x - xs[b]) / (xs[a] - xs[b])
        total += w * ys[a]
    return total


def _window(nodes, x):
    """First index of the four consecutive nodes whose middle interval holds x."""
    k = int(np.searchsorted(nodes, x, side="right")) - 1   # nodes[k] <= x < nodes[k+1]
    k = min(max(k, 0), len(nodes) - 2)
    return min(max(k - 1, 0), len(nodes) - 4)


def transfer(me_old: Mesh, x_old, me_new: Mesh, nb=None):
    """State x_old (paper order) on me_old -> paper-order state on me_new."""
    m, n = me_old.m, me_old.n
    n0, U = from_vec(x_old, m, n)
    # each old θ-line as a 1-D node set
    if nb is not None:
        rr = me_old.r.copy()                                # r_0..r_{m+1}
        lines = [np.concatenate([[n0], U[:, j], [nb[j]]]) for j in range(n)]
    else:
        rr = me_old.r[:m + 1].copy()                        # r_0..r_m
        lines = [np.concatenate([[n0], U[:, j]]) for j in range(n)]
    th = me_old.th[:n]
    out = np.zeros((me_new.m, me_new.n))
    for i2 in range(1, me_new.m + 1):
        rq = me_new.r[i2]
        k = _window(rr, rq)
        col = np.array([_lagrange4(rr[k:k + 4], lines[j][k:k + 4], rq) for j in range(n)])
        for j2 in range(me_new.n):
            tq = me_new.th[j2]
            # the old node at or before tq, then four periodic neighbours
            jb = int(np.searchsorted(th, tq, side="right")) - 1
            idx = [(jb - 1 + s) % n for s in range(4)]
            ts = np.array([th[jb - 1 + s - n * ((jb - 1 + s) // n)] + 2 * np.pi * ((jb - 1 + s) // n)
                           for s in range(4)])
            out[i2 - 1, j2] = _lagrange4(ts, col[idx], tq)
    return to_vec(n0, out)
