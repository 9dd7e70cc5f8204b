"""Polar mesh and time levels (oracle; test infrastructure only).

Radial nodes (§2.1, eq. (2.4), and §3.1): h = 1/(m+1), r_i = υ(i h),
i = 0..m+1, with
    kind 0 (uniform):     r_i = i h
    kind 1 (eq. (2.4)):   υ(s) = sin(s^p π/2)
    kind 3 (eq. (2.13)):  φ(s) = 1 - (1 - s)^{p+1}
    kind 2:               explicit values.
r_{i+1/2} = (r_i + r_{i+1})/2, h_i = r_i - r_{i-1}.

Angular nodes (§3.1): μ̃ = 2π/n, θ_j = v(j μ̃), j = 0..n, with
    kind 0 (uniform):     θ_j = j μ̃
    kind 1:               v(ι) = 2π sin((ι/2π)^q π/2)
    kind 2:               explicit values;
μ_j = θ_j - θ_{j-1} (j = 1..n), μ_0 = μ_n; the width of cell j is
(μ_j + μ_{j+1})/2 and its angular faces sit at θ_{j+1/2} = (θ_j + θ_{j+1})/2.

End points are set exactly: r_0 = 0, r_{m+1} = 1, θ_0 = 0, θ_n = 2π.

Time levels (§3.1): t_k = V(k T/K) with V(t) = T sin((t/T)^l π/2), or the
uniform t_k = k Δt of §2.1.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Mesh:
    m: int
    n: int
    r: np.ndarray        # r_0..r_{m+1}
    th: np.ndarray       # θ_0..θ_n

    @property
    def h(self):         # h_1..h_{m+1} stored at index 1..m+1 (index 0 unused)
        out = np.zeros(self.m + 2)
        out[1:] = np.diff(self.r)
        return out

    @property
    def r_half(self):    # r_{i+1/2}, i = 0..m
        return 0.5 * (self.r[:-1] + self.r[1:])

    @property
    def mu(self):        # μ_0..μ_n with μ_0 = μ_n
        mu = np.zeros(self.n + 1)
        mu[1:] = np.diff(self.th)
        mu[0] = mu[self.n]
        return mu

    @property
    def dtheta(self):    # cell widths (μ_j + μ_{j+1})/2, j = 0..n-1
        mu = self.mu
        return 0.5 * (mu[:self.n] + mu[1:self.n + 1])

    @property
    def th_half(self):   # θ_{j+1/2}, j = 0..n-1
        return 0.5 * (self.th[:-1] + self.th[1:])

    def sample_points(self):
        return self.r, self.r_half, self.th, self.th_half


def radial_nodes(m, kind=0, p=1.0, explicit=None):
    h = 1.0 / (m + 1)
    s = np.arange(m + 2) * h
    if kind == 0:
        r = s.copy()
    elif kind == 1:
        r = np.sin(s ** p * np.pi / 2.0)
    elif kind == 3:
        r = 1.0 - (1.0 - s) ** (p + 1.0)
    elif kind == 2:
        r = np.array(explicit, float)
    else:
        raise ValueError(f"unknown radial mesh kind {kind}")
    r[0] = 0.0
    r[-1] = 1.0
    return r


def angular_nodes(n, kind=0, q=1.0, explicit=None):
    s = np.arange(n + 1) / n
    if kind == 0:
        th = 2.0 * np.pi * s
    elif kind == 1:
        th = 2.0 * np.pi * np.sin(s ** q * np.pi / 2.0)
    elif kind == 2:
        th = np.array(explicit, float)
    else:
        raise ValueError(f"unknown angular mesh kind {kind}")
    th[0] = 0.0
    th[-1] = 2.0 * np.pi
    return th


def make_mesh(m, n, r_kind=0, p=1.0, th_kind=0, q=1.0, r_explicit=None, th_explicit=None):
    return Mesh(m, n, radial_nodes(m, r_kind, p, r_explicit),
                angular_nodes(n, th_kind, q, th_explicit))


def time_levels(T, K, t_kind=0, l=1.0, table=None):
    """t_0..t_K: uniform (kind 0), the sine stretch V (kind 1), or a table (kind 2)."""
    if t_kind == 0:
        t = T * np.arange(K + 1) / K
    elif t_kind == 1:
        t = T * np.sin((np.arange(K + 1) / K) ** l * np.pi / 2.0)
    elif t_kind == 2:
        t = np.array(table, float)
    else:
        raise ValueError(f"unknown time kind {t_kind}")
    t[0] = 0.0
    if t_kind != 2:
        t[-1] = T
    return t
