"""Pins of the oracle's alternating-line preconditioner (oracle/precond.py):
exact inverses where the system has only one kind of coupling, and a dense
brute-force construction, with its own index logic, on tiny meshes."""

import numpy as np
import pytest

from oracle import assemble, make_mesh
from oracle.precond import LinePreconditioner
from oracle.stepper import system_matrix
from problems import continuity_cfg, sample


def system(m, n, seed=5101, edit=None):
    pb = continuity_cfg(seed, m, n, 0.5, 1.3)
    me = make_mesh(m, n, 1, 1.3)
    data = sample(pb, *me.sample_points())
    if edit:
        edit(data)
    return assemble(me, data)


def radial_only(data):
    """No angular faces and an origin decoupled from ring 1."""
    data["D_t"] = np.zeros_like(data["D_t"])
    data["Et_t"] = np.zeros_like(data["Et_t"])
    data["D_r"] = np.array(data["D_r"], copy=True)
    data["Er_r"] = np.array(data["Er_r"], copy=True)
    data["D_r"][0] = 0.0
    data["Er_r"][0] = 0.0


def angular_only(data):
    """No radial faces except those joining the origin to ring 1."""
    data["D_r"] = np.array(data["D_r"], copy=True)
    data["Er_r"] = np.array(data["Er_r"], copy=True)
    data["D_r"][1:] = 0.0
    data["Er_r"][1:] = 0.0


@pytest.mark.parametrize("edit", [radial_only, angular_only])
def test_exact_when_one_coupling_is_missing(edit):
    """With only radial couplings M = I + D^{-1}R = D^{-1}A, with only
    angular (and origin) couplings M = I + D^{-1}Θ = D^{-1}A: M^{-1} D^{-1} A
    is then the identity, whatever the coefficients."""
    S = system(12, 20, edit=edit)
    P = LinePreconditioner(S, 3e-4, 0.7)
    x = np.random.default_rng(1).standard_normal(S.N)
    z = P(P.scaled_operator(x))
    assert np.max(np.abs(z - x)) <= 1e-12 * np.max(np.abs(x))
    # the full system has both couplings: there the preconditioner is not exact
    Sf = system(12, 20)
    Pf = LinePreconditioner(Sf, 3e-4, 0.7)
    assert np.max(np.abs(Pf(Pf.scaled_operator(x)) - x)) > 1e-6 * np.max(np.abs(x))


def brute_force_M(S, dt, theta):
    """Dense M built entry by entry: couplings classified by decoding each
    paper-order index into (ring, line) by hand."""
    A = system_matrix(S, dt, theta).toarray()
    m = S.mesh.m
    N = A.shape[0]
    d = np.diag(A).copy()

    def where(q):   # (ring, line); the origin is ring 0 on no line
        if q == 0:
            return 0, None
        return (q - 1) % m + 1, (q - 1) // m

    R = np.zeros((N, N))
    T = np.zeros((N, N))
    for p in range(N):
        for q in range(N):
            if p == q or A[p, q] == 0.0:
                continue
            (ip, jp), (iq, jq) = where(p), where(q)
            if p == 0 or q == 0 or ip == iq:
                T[p, q] = A[p, q]
            elif jp == jq:
                R[p, q] = A[p, q]
            else:
                raise AssertionError("a five-point operator couples only rings and lines")
    I = np.eye(N)
    Rs, Ts = I + R / d[:, None], I + T / d[:, None]
    return Rs @ Ts, Ts @ Rs


@pytest.mark.parametrize("m,n,theta", [(3, 5, 0.5), (4, 6, 1.0), (2, 8, 0.75)])
def test_matches_a_dense_brute_force(m, n, theta):
    S = system(m, n, seed=5102 + m)
    dt = 2e-3
    M, M_swapped = brute_force_M(S, dt, theta)
    P = LinePreconditioner(S, dt, theta)
    y = np.random.default_rng(m * n).standard_normal(S.N)
    z = np.linalg.solve(M, y)
    assert np.max(np.abs(P(y) - z)) <= 1e-12 * np.max(np.abs(z))
    # the order of the factors matters: the other order is another operator
    zs = np.linalg.solve(M_swapped, y)
    assert np.max(np.abs(P(y) - zs)) > 1e-9 * np.max(np.abs(zs))
