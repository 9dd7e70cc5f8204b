"""Manufactured problems on the unit disk in polar coordinates (r, θ).

A problem is the continuous data of either PDE solved by the method:

* parabolic (Ch. 2, eqs. (2.1)-(2.3)):  u_t - Δu + b u = f,  u = γ on r = 1;
* continuity / drift-diffusion (Ch. 3, eqs. (3.1)-(3.4)):
      n_t = ∇·(D ∇n) - ∇·(n E) + GR,  n = N on r = 1,
  with the mobility folded into E as in (3.4).  E is a vector field with
  polar components (E_r, E_θ).

Both are written as  n_t + 𝓛 n = S(t)  with 𝓛 n = -∇·(D∇n) + ∇·(nE) + b n,
so the parabolic case is D = 1, E = 0.  Time dependence of the source and of
the Dirichlet data is a short sum of modes  τ_q(t) = t^{d_q} exp(λ_q t):

      S(t, r, θ) = Σ_q τ_q(t) g_q(r, θ),      N(t, θ) = Σ_q τ_q(t) nb_q(θ).

Every function here is the *problem*; none of the discretisation lives here.
g_q must be defined at r = 0 (its limit there), because the origin unknown
uses the point value of the source at the origin (Ch. 3, origin source
integral).

Seeds: ``numpy.random.default_rng(seed)`` with the draw order documented in
each constructor.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np
from scipy.special import jn_zeros, jv, jvp

Fn2 = Callable[[np.ndarray, np.ndarray], np.ndarray]


@dataclass
class TimeMode:
    lam: float          # exponent λ_q
    tpow: int           # power d_q of t
    g: Fn2              # source shape g_q(r, θ); must accept r == 0
    nb: Callable[[np.ndarray], np.ndarray]   # Dirichlet shape nb_q(θ)


@dataclass
class Problem:
    name: str
    pde: int                       # 0 parabolic, 1 continuity
    modes: List[TimeMode]
    u0: Fn2
    D: Optional[Fn2] = None        # None -> 1
    Er: Optional[Fn2] = None       # None -> 0
    Et: Optional[Fn2] = None       # None -> 0
    b: Optional[Fn2] = None        # None -> 0 (reaction, parabolic only)
    exact: Optional[Callable[[float, np.ndarray, np.ndarray], np.ndarray]] = None
    # scalar E of the paper's literal Ch. 3 stencil (nodes); only the paper
    # examples define it.
    E_scalar: Optional[Fn2] = None
    mesh: dict = field(default_factory=dict)
    time: dict = field(default_factory=dict)
    meta: dict = field(default_factory=dict)

    def tau(self, q: int, t: float) -> float:
        md = self.modes[q]
        return (t ** md.tpow if md.tpow else 1.0) * np.exp(md.lam * t)


def _const(c):
    return lambda r, th: np.full(np.broadcast(r, th).shape, float(c))


def _bc_const(c):
    return lambda th: np.full(np.shape(th), float(c))


def sample(pb: Problem, r_nodes, r_faces, th_nodes, th_faces) -> dict:
    """Evaluate the problem data at given sample points.

    r_nodes: r_0..r_{m+1};  r_faces: r_{1/2}..r_{m+1/2};
    th_nodes: θ_0..θ_n;     th_faces: θ_{1/2}..θ_{n-1/2}.
    Returns node data split into an origin value and an (m, n) ring grid
    (ring i = 1..m is row i-1, column j = 0..n-1), radial-face data (m+1, n)
    at (r_{i+1/2}, θ_j), i = 0..m, and angular-face data (m, n) at
    (r_i, θ_{j+1/2}), i = 1..m.
    """
    r_nodes = np.asarray(r_nodes, float)
    r_faces = np.asarray(r_faces, float)
    th_nodes = np.asarray(th_nodes, float)
    th_faces = np.asarray(th_faces, float)
    m = r_nodes.size - 2
    n = th_nodes.size - 1
    tn = th_nodes[:n]
    RG, TG = np.meshgrid(r_nodes[1:m + 1], tn, indexing="ij")      # nodes
    RR, TR = np.meshgrid(r_faces, tn, indexing="ij")               # radial faces
    RA, TA = np.meshgrid(r_nodes[1:m + 1], th_faces, indexing="ij")  # angular faces
    zero = np.zeros(1)
    D = pb.D or _const(1.0)
    Er = pb.Er or _const(0.0)
    Et = pb.Et or _const(0.0)
    b = pb.b or _const(0.0)
    out = {
        "m": m, "n": n, "pde": pb.pde,
        "D_r": D(RR, TR), "Er_r": Er(RR, TR),
        "D_t": D(RA, TA), "Et_t": Et(RA, TA),
        "b_grid": b(RG, TG), "b_origin": float(b(zero, zero)[0]),
        "lam": np.array([md.lam for md in pb.modes], float),
        "tpow": np.array([md.tpow for md in pb.modes], np.int32),
        "g_grid": np.stack([md.g(RG, TG) for md in pb.modes]),
        "g_origin": np.array([float(md.g(zero, zero)[0]) for md in pb.modes]),
        "nb": np.stack([md.nb(tn) for md in pb.modes]),
        "u0_grid": pb.u0(RG, TG), "u0_origin": float(pb.u0(zero, zero)[0]),
        "D_origin": float(D(zero, zero)[0]),
    }
    if pb.E_scalar is not None:
        out["E_grid"] = pb.E_scalar(RG, TG)
        out["E_origin"] = float(pb.E_scalar(zero, zero)[0])
    return out


def exact_at(pb: Problem, t: float, r_nodes, th_nodes):
    """Exact solution at the nodes: (origin value, (m, n) grid)."""
    r_nodes = np.asarray(r_nodes, float)
    th_nodes = np.asarray(th_nodes, float)
    m = r_nodes.size - 2
    n = th_nodes.size - 1
    RG, TG = np.meshgrid(r_nodes[1:m + 1], th_nodes[:n], indexing="ij")
    z = np.zeros(1)
    return float(pb.exact(t, z, z)[0]), pb.exact(t, RG, TG)


# ---------------------------------------------------------------- parabolic

def parabolic_family(lam=1.0, beta=0.5, theta0=0.0, name="parabolic"):
    """u = exp(-lam t) φ,  φ = (1 - r²)(1 + β r cos(θ - θ0)),  b = 0.

    In Cartesian form φ = (1 - x² - y²)(1 + β(x cos θ0 + y sin θ0)), so
    Δφ = -4 - 8 β r cos(θ - θ0) and f = exp(-lam t)(-lam φ - Δφ).
    Dirichlet data is 0 on r = 1.
    """
    def phi(r, th):
        return (1.0 - r * r) * (1.0 + beta * r * np.cos(th - theta0))

    def lap(r, th):
        return -4.0 - 8.0 * beta * r * np.cos(th - theta0)

    def g(r, th):
        return -lam * phi(r, th) - lap(r, th)

    return Problem(
        name=name, pde=0,
        modes=[TimeMode(-lam, 0, g, _bc_const(0.0))],
        u0=phi,
        exact=lambda t, r, th: np.exp(-lam * t) * phi(r, th),
        meta={"lam": lam, "beta": beta, "theta0": theta0},
    )


def parabolic_cfg1():
    """32 x 64 uniform mesh, Crank-Nicolson, dt = 1e-3, T = 0.1 (100 steps),
    u = exp(-t)(1 - r²)(1 + r cos θ / 2)."""
    pb = parabolic_family(1.0, 0.5, 0.0, name="parabolic_cfg1")
    pb.mesh = dict(m=32, n=64, r_kind=0, p=1.0, th_kind=0, q=1.0)
    pb.time = dict(theta=0.5, T=0.1, K=100, t_kind=0, l=1.0)
    return pb


def closed_form_quadratic(c=0.25):
    """u = (1 + t) r² + c: Δu = 4, so f = r² - 4(1 + t), γ = 1 + t + c.

    Quadratic in r, constant in θ and linear in t: a conservative 5-point
    scheme on a uniform radial mesh with the origin closure reproduces it
    exactly, and any θ-weighted scheme is exact in time for it.
    """
    return Problem(
        name="closed_form_quadratic", pde=0,
        modes=[TimeMode(0.0, 0, lambda r, th: r * r - 4.0 + 0.0 * th, _bc_const(1.0 + c)),
               TimeMode(0.0, 1, _const(-4.0), _bc_const(1.0))],
        u0=lambda r, th: r * r + c + 0.0 * th,
        exact=lambda t, r, th: (1.0 + t) * r * r + c + 0.0 * th,
    )


def paper_parabolic_ex1():
    """Ch. 2, numerical experiment 1: u = e^{-t} r² + r² (1 - r)^{1/2}.

    The source is the printed one, which agrees with -Δu + u_t of this u
    (a radial function, so the sign of the θ term is irrelevant).
    """
    def g_t(r, th):
        return -r * r - 4.0 + 0.0 * th

    def g_s(r, th):
        s = np.sqrt(1.0 - r)
        return -4.0 * s + 5.0 * r / (2.0 * s) + r * r / (4.0 * s ** 3) + 0.0 * th

    return Problem(
        name="paper_parabolic_ex1", pde=0,
        modes=[TimeMode(-1.0, 0, g_t, _bc_const(1.0)),
               TimeMode(0.0, 0, g_s, _bc_const(0.0))],
        u0=lambda r, th: r * r + r * r * np.sqrt(1.0 - r) + 0.0 * th,
        exact=lambda t, r, th: np.exp(-t) * r * r + r * r * np.sqrt(1.0 - r) + 0.0 * th,
    )


def paper_continuity_ex1():
    """Ch. 3, numerical experiment 1: D = E = r, exact
    n = e^{-t} r + r (1 - r)^{1/2} + r sin²θ, boundary e^{-t} + sin²θ.

    The source is the printed one (with its printed signs), split into the
    e^{-t} part and the time-independent part.  The scalar E of the printed
    stencil is E = r; as a vector field both polar components equal r.
    """
    # At r = 0, D = E = 0 and the exact solution is identically 0, so the
    # equation there reduces to n_t = GR(t, 0) = 0; the printed GR is not
    # continuous at the origin (its limit depends on θ), and the origin
    # source takes the value the exact solution dictates.
    def g_t(r, th):
        return np.where(r > 0, 2.0 * r - 2.0 + 0.0 * th, 0.0)

    def g_s(r, th):
        s = np.sqrt(1.0 - r)
        s2 = np.sin(th) ** 2
        v = (-2.0 * s + 2.0 * r / s - 0.25 * r * r / s ** 3 - 2.0 * s2 - 2.0 * np.cos(2 * th)
             + 3.0 * r * s - 0.5 * r * r / s + 3.0 * r * s2 + r * np.sin(2 * th))
        return np.where(r > 0, v, 0.0)

    return Problem(
        name="paper_continuity_ex1", pde=1,
        modes=[TimeMode(-1.0, 0, g_t, _bc_const(1.0)),
               TimeMode(0.0, 0, g_s, lambda th: np.sin(th) ** 2)],
        u0=lambda r, th: r + r * np.sqrt(1.0 - r) + r * np.sin(th) ** 2,
        D=lambda r, th: r + 0.0 * th,
        Er=lambda r, th: r + 0.0 * th,
        Et=lambda r, th: r + 0.0 * th,
        E_scalar=lambda r, th: r + 0.0 * th,
        exact=lambda t, r, th: (np.exp(-t) * r + r * np.sqrt(1.0 - r) + r * np.sin(th) ** 2),
    )


def paper_continuity_ex2():
    """Ch. 3, numerical experiment 2: D = E = r, exact
    n = e^{-t} r sin²θ + r (1 - r)^{1/2} + r sin²θ, boundary
    e^{-t} sin²θ + sin²θ.

    The source is the printed one, split as for experiment 1 into its
    e^{-t} part, 2 r sin²θ - 2 sin²θ - 2 cos 2θ + r sin 2θ, and its
    time-independent part, which is experiment 1's; the origin source is 0
    (the exact solution vanishes there for all t).
    """
    def g_t(r, th):
        s2 = np.sin(th) ** 2
        return np.where(r > 0, 2.0 * r * s2 - 2.0 * s2 - 2.0 * np.cos(2 * th) + r * np.sin(2 * th), 0.0)

    g_s = paper_continuity_ex1().modes[1].g
    return Problem(
        name="paper_continuity_ex2", pde=1,
        modes=[TimeMode(-1.0, 0, g_t, lambda th: np.sin(th) ** 2),
               TimeMode(0.0, 0, g_s, lambda th: np.sin(th) ** 2)],
        u0=lambda r, th: 2.0 * r * np.sin(th) ** 2 + r * np.sqrt(1.0 - r),
        D=lambda r, th: r + 0.0 * th,
        Er=lambda r, th: r + 0.0 * th,
        Et=lambda r, th: r + 0.0 * th,
        E_scalar=lambda r, th: r + 0.0 * th,
        exact=lambda t, r, th: (np.exp(-t) * r * np.sin(th) ** 2 + r * np.sqrt(1.0 - r) + r * np.sin(th) ** 2),
    )


# --------------------------------------------------------------- continuity

def _per_ring(f, r):
    """f(r) for an array of radii; on a grid whose rows hold one radius each
    (a meshgrid over rings), f is evaluated once per row and broadcast."""
    r = np.asarray(r, float)
    if r.ndim == 2 and r.shape[1] > 1 and np.all(r == r[:, :1]):
        return np.broadcast_to(f(r[:, :1]), r.shape)
    return f(r)


def _bessel_potential(modes):
    """ψ = Σ A J_k(α r) cos(kθ + φ) with α = j_{k,1}; returns callables for
    ψ_r, ψ_θ / r, Δψ, and ∇ψ at the origin (Cartesian)."""
    alph = [float(jn_zeros(k, 1)[0]) for (_, k, _) in modes]

    def J(k, a, r):
        return _per_ring(lambda rr: jv(k, a * rr), r)

    def psi(r, th):
        return sum(A * J(k, a, r) * np.cos(k * th + ph) for (A, k, ph), a in zip(modes, alph))

    def psi_r(r, th):
        return sum(A * a * _per_ring(lambda rr: jvp(k, a * rr, 1), r) * np.cos(k * th + ph)
                   for (A, k, ph), a in zip(modes, alph))

    def psi_t_over_r(r, th):
        # (1/r) ∂ψ/∂θ; J_k(αr)/r -> α/2 (k = 1) or 0 (k != 1) at r = 0
        tot = 0.0
        for (A, k, ph), a in zip(modes, alph):
            if k == 0:
                continue
            lim = (a / 2.0) if k == 1 else 0.0
            jr = _per_ring(lambda rr: np.where(rr > 0, jv(k, a * rr) / np.where(rr > 0, rr, 1.0), lim), r)
            tot = tot - A * k * jr * np.sin(k * th + ph)
        return tot

    def lap_psi(r, th):
        return sum(-(a * a) * A * J(k, a, r) * np.cos(k * th + ph)
                   for (A, k, ph), a in zip(modes, alph))

    def grad0():
        gx = gy = 0.0
        for (A, k, ph), a in zip(modes, alph):
            if k == 1:
                gx += A * a / 2.0 * np.cos(ph)
                gy += -A * a / 2.0 * np.sin(ph)
        return gx, gy

    return psi, psi_r, psi_t_over_r, lap_psi, grad0


def continuity_cfg(seed: int, m=256, n=512, theta=0.5, p=1.3, T=0.05, K=100, l=1.5,
                   t_kind=1, name=None):
    """Drift-diffusion problem with a seeded diffusivity and drift field.

    Draw order from default_rng(seed): k_D ~ U{1..4}; then for q = 1..4:
    A_q ~ U[-2, 2], k_q ~ U{0..4}, φ_q ~ U[0, 2π).

    D = 1 + ½ sin(k_D θ) r²;  ψ = Σ_q A_q J_{k_q}(j_{k_q,1} r) cos(k_q θ + φ_q);
    E = -∇ψ;  exact n = e^{-t} φ, φ = 3/2 + (1 - r²)(1 + ½ r cos θ + ¼ r² sin 2θ).
    In Cartesian form φ = 3/2 + P Q with P = 1 - x² - y², Q = 1 + x/2 + x y/2.
    GR = e^{-t} g,  g = -φ - ∇·(D∇φ) + ∇·(φE) = -φ - ∇D·∇φ - DΔφ - ∇φ·∇ψ - φΔψ.
    """
    rng = np.random.default_rng(seed)
    kD = int(rng.integers(1, 5))
    modes = []
    for _ in range(4):
        A = float(rng.uniform(-2.0, 2.0))
        k = int(rng.integers(0, 5))
        ph = float(rng.uniform(0.0, 2 * np.pi))
        modes.append((A, k, ph))
    psi, psi_r, psi_tr, lap_psi, grad0 = _bessel_potential(modes)

    def cart(r, th):
        return r * np.cos(th), r * np.sin(th)

    def phi_parts(r, th):
        x, y = cart(r, th)
        P = 1.0 - x * x - y * y
        Q = 1.0 + 0.5 * x + 0.5 * x * y
        Px, Py = -2.0 * x, -2.0 * y
        Qx, Qy = 0.5 + 0.5 * y, 0.5 * x
        phi = 1.5 + P * Q
        phx = Px * Q + P * Qx
        phy = Py * Q + P * Qy
        lap = -4.0 * Q + 2.0 * (Px * Qx + Py * Qy)
        return phi, phx, phy, lap

    def Dfun(r, th):
        return 1.0 + 0.5 * np.sin(kD * th) * r * r

    def Er(r, th):
        return -psi_r(r, th)

    def Et(r, th):
        return -psi_tr(r, th)

    def g(r, th):
        r = np.asarray(r, float)
        th = np.asarray(th, float)
        phi, phx, phy, lap = phi_parts(r, th)
        c, s = np.cos(th), np.sin(th)
        ph_r = phx * c + phy * s
        ph_t = -phx * s + phy * c            # (1/r) ∂φ/∂θ
        D_r = r * np.sin(kD * th)
        D_t = 0.5 * r * kD * np.cos(kD * th)  # (1/r) ∂D/∂θ
        gradD_gradphi = D_r * ph_r + D_t * ph_t
        gpsi_gphi = psi_r(r, th) * ph_r + psi_tr(r, th) * ph_t
        val = -phi - gradD_gradphi - Dfun(r, th) * lap - gpsi_gphi - phi * lap_psi(r, th)
        # origin: the Cartesian limit (∇D = 0 and D = 1 there)
        z = np.zeros(1)
        p0, px0, py0, l0 = (v[0] for v in phi_parts(z, z))
        gx, gy = grad0()
        val0 = -p0 - l0 - (px0 * gx + py0 * gy) - p0 * float(lap_psi(z, z)[0])
        return np.where(r > 0, val, val0)

    def phi(r, th):
        return phi_parts(np.asarray(r, float), np.asarray(th, float))[0]

    pb = Problem(
        name=name or f"continuity_seed{seed}", pde=1,
        modes=[TimeMode(-1.0, 0, g, _bc_const(1.5))],
        u0=phi, D=Dfun, Er=Er, Et=Et,
        exact=lambda t, r, th: np.exp(-t) * phi(r, th),
        meta={"seed": seed, "kD": kD, "modes": modes},
    )
    pb.mesh = dict(m=m, n=n, r_kind=1, p=p, th_kind=0, q=1.0)
    pb.time = dict(theta=theta, T=T, K=K, t_kind=t_kind, l=l)
    pb.meta["psi"] = psi
    return pb


# ----------------------------------------------------- property-test problems

def random_positive(seed: int, pde: int = 1):
    """Source-free problem with seeded, oscillatory, non-negative initial
    data and non-negative Dirichlet data (used for positivity / maximum
    principle properties).  Continuity: D in [0.5, 1.5], smooth drift."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.0, 2 * np.pi, size=6)
    a = rng.uniform(0.2, 1.0, size=3)

    def u0(r, th):
        return 1.0 + np.sin(23.0 * r + 5.0 * th + c[0]) * np.cos(17.0 * r * r - 3.0 * th + c[1])

    pb = Problem(
        name=f"random_positive{seed}", pde=pde,
        modes=[TimeMode(0.0, 0, _const(0.0), lambda th: 0.5 + 0.4 * np.sin(3 * th + c[2]))],
        u0=u0,
    )
    if pde == 1:
        pb.D = lambda r, th: 1.0 + 0.5 * np.sin(2 * th + c[3]) * r
        pb.Er = lambda r, th: a[0] * np.cos(th + c[4]) + a[1] * r
        pb.Et = lambda r, th: -a[0] * np.sin(th + c[4]) + a[2] * r * np.cos(2 * th + c[5])
    else:
        pb.b = lambda r, th: a[0] * (1.0 + np.cos(th + c[4]) * r)
    return pb


def zero_flux_random(seed: int):
    """Continuity problem with GR = 0 for mass-conservation checks (used with
    the zero-flux outer boundary): seeded D > 0, seeded drift, positive data."""
    pb = random_positive(seed, pde=1)
    pb.name = f"zero_flux{seed}"
    pb.modes = [TimeMode(0.0, 0, _const(0.0), _bc_const(0.0))]
    return pb


def two_carrier(seed: int, eps: float = 0.5, doping: float = 1.0, zero_flux: bool = False):
    """Electrons n, holes p and the electrostatic potential ψ on the unit
    disk (the two continuity equations of §3.1 with the field of a Poisson
    problem, in scaled units): (ψ problem, n problem, p problem).

    * ψ: D = eps, no drift; mode 0 is the charge slot (g = 0, filled with
      p - n by the coupling; Dirichlet ψ_b(θ) = 0.2 cos(θ + c)), mode 1 the
      doping C(r, θ) = doping (1 - r²)(1 + ½ r cos(2θ + c')); λ = 0.
    * n, p: seeded diffusivities D = d0 (1 + ¼ r² sin(kθ + c)), no drift of
      their own (the coupling sets it from ψ); a steady generation
      g(r, θ) = 0.3 (1 - r²) (λ = 0); Dirichlet data 1 (n) and 0.5 + 0.1 sin θ
      (p), or zero flux with no generation; positive smooth initial data.
    Draw order: c[0..5] ~ U[0, 2π), k ~ U{1..3}."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.0, 2 * np.pi, size=6)
    k = int(rng.integers(1, 4))
    zero = _const(0.0)
    psi = Problem(
        name=f"two_carrier_psi{seed}", pde=1,
        modes=[TimeMode(0.0, 0, zero, lambda th: 0.2 * np.cos(th + c[0])),
               TimeMode(0.0, 0, lambda r, th: doping * (1 - r * r) * (1 + 0.5 * r * np.cos(2 * th + c[1])),
                        _bc_const(0.0))],
        u0=zero, D=_const(eps))

    def carrier(name, d0, nb, u0_amp, phase):
        g = zero if zero_flux else (lambda r, th: 0.3 * (1 - r * r) + 0.0 * th)
        return Problem(
            name=f"two_carrier_{name}{seed}", pde=1,
            modes=[TimeMode(0.0, 0, g, _bc_const(0.0) if zero_flux else nb)],
            u0=lambda r, th: 1.0 + u0_amp * (1 - r * r) * (1 + 0.5 * r * np.cos(th + phase)),
            D=lambda r, th: d0 * (1.0 + 0.25 * r * r * np.sin(k * th + phase)))

    n_pb = carrier("n", 1.0, _bc_const(1.0), 0.5, c[2])
    p_pb = carrier("p", 0.5, lambda th: 0.5 + 0.1 * np.sin(th), 0.3, c[3])
    return psi, n_pb, p_pb
