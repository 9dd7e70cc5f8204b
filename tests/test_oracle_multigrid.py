"""Pins of the oracle's θ-semi-coarsening multigrid (oracle/multigrid.py):
the line maps decoded by hand, the ring-mean level against the operator's
own action on ring-constant vectors, exactness where the smoother is exact,
the V-cycle against its error-propagation product, and the contraction and
iteration counts that make it a multigrid method."""

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import assemble, make_mesh
from oracle.multigrid import NMIN, MultigridPreconditioner, hierarchy, line_map, ring_map
from oracle.precond import LinePreconditioner
from oracle.stepper import system_matrix
from problems import continuity_cfg, sample, two_carrier


def where(q, m):
    """(ring, θ-line) of a paper-order index; the origin is (0, None)."""
    return (0, None) if q == 0 else ((q - 1) % m + 1, (q - 1) // m)


@pytest.mark.parametrize("m,n", [(3, 8), (2, 9), (4, 17), (1, 16)])
def test_line_map_merges_pairs_and_the_last_three(m, n):
    P, nc = line_map(m, n)
    assert nc == n // 2 and P.shape == (m * n + 1, m * nc + 1)
    P = P.toarray()
    assert np.array_equal(P.sum(axis=1), np.ones(m * n + 1))     # one coarse value per fine unknown
    for q in range(m * n + 1):
        qc = int(np.argmax(P[q]))
        (i, j), (ic, J) = where(q, m), where(qc, m)
        assert i == ic                                             # rings are kept
        if q:
            expect = min(j // 2, nc - 1)                           # pairs; the last takes three if n is odd
            assert J == expect
    sizes = P.sum(axis=0)[1:].reshape(nc, m)[:, 0]
    assert list(sizes[:-1]) == [2] * (nc - 1) and sizes[-1] == (3 if n % 2 else 2)


@pytest.mark.parametrize("m,n", [(3, 40), (2, 33), (4, 64)])
def test_composed_maps_reach_the_ring_means(m, n):
    """The maps of all θ-levels times the final ring map send (i, j) to ring
    i and the origin to the origin."""
    A = sp.identity(m * n + 1, format="csr")
    V = np.ones(m * n + 1)
    levels, _ = hierarchy(A, V, m, n)
    assert [lv.n for lv in levels][0] == n and levels[-1].n < NMIN and levels[-1].nc == 1
    assert all(a.n // 2 == b.n for a, b in zip(levels, levels[1:]))
    Pt = sp.identity(m * n + 1, format="csr")
    for lv in levels:
        Pt = Pt @ lv.P
    R = np.zeros((m * n + 1, m + 1))
    for q in range(m * n + 1):
        R[q, where(q, m)[0]] = 1.0
    assert np.array_equal(Pt.toarray(), R)
    assert np.array_equal(ring_map(m, n).toarray(), R)


def theta_free_system(m, n, flux=0, bc=0):
    """Coefficients that do not depend on θ on a uniform θ mesh: constant D,
    a radial drift and a reaction that vary with r only."""
    me = make_mesh(m, n, 1, 1.3)
    d = sample(two_carrier(3200)[0], *me.sample_points())
    rr = np.linspace(0.0, 1.0, m + 1)[:, None] * np.ones((1, n))
    d["Er_r"] = 0.7 - 1.3 * rr
    d["b_grid"] = np.outer(0.5 + np.linspace(0, 1, m), np.ones(n))
    d["b_origin"] = 0.5
    return assemble(me, d, flux=flux, bc=bc)


@pytest.mark.parametrize("m,n,flux,bc", [(5, 40, 0, 0), (4, 33, 1, 0), (3, 64, 0, 1)])
def test_ring_mean_level_reproduces_the_operator_on_ring_constants(m, n, flux, bc):
    """With θ-free coefficients A maps ring-constant vectors to ring-constant
    vectors, A (P c) = P (A_red c).  The ring-mean level, built by chaining
    every Galerkin product, must then be diag(V_ring) A_red: a dropped
    face, a wrong merge or a transposed map breaks it."""
    S = theta_free_system(m, n, flux, bc)
    A = system_matrix(S, 3e-3, 0.7)
    levels, A_ring = hierarchy(A, S.V, m, n)
    R = ring_map(m, n)
    V_ring = R.T @ S.V
    c = np.random.default_rng(m * n).standard_normal(m + 1)
    lhs = A @ (R @ c)
    rhs = R @ ((A_ring @ c) / V_ring)
    assert np.max(np.abs(lhs - rhs)) <= 1e-12 * np.max(np.abs(lhs))
    # the same check one level down, on vectors constant over merged pairs
    # only, fails: the property belongs to ring constants
    P1, _ = line_map(m, n)
    c1 = np.random.default_rng(1).standard_normal(P1.shape[1])
    y = A @ (P1 @ c1)
    assert np.max(np.abs(y - P1 @ ((P1.T @ (S.V * y)) / (P1.T @ S.V)))) > 1e-6 * np.max(np.abs(y))


def small(m, n, kind, edit=None):
    me = make_mesh(m, n, 1, 1.3)
    pb = two_carrier(3200)[0] if kind == "psi" else continuity_cfg(1300, m, n, 0.5, 1.3)
    d = sample(pb, *me.sample_points())
    if edit:
        edit(d)
    dt, th = (1e30, 1.0) if kind == "psi" else (2.5e-4, 0.5)
    return assemble(me, d), dt, th


def radial_only(d):
    d["D_t"] = np.zeros_like(d["D_t"])
    d["Et_t"] = np.zeros_like(d["Et_t"])
    d["D_r"] = np.array(d["D_r"], copy=True)
    d["Er_r"] = np.array(d["Er_r"], copy=True)
    d["D_r"][0] = 0.0
    d["Er_r"][0] = 0.0


def angular_only(d):
    d["D_r"] = np.array(d["D_r"], copy=True)
    d["Er_r"] = np.array(d["Er_r"], copy=True)
    d["D_r"][1:] = 0.0
    d["Er_r"][1:] = 0.0


@pytest.mark.parametrize("edit", [radial_only, angular_only])
def test_exact_when_the_smoother_is(edit):
    """With one kind of coupling the fine smoother solves the system: the
    residual after it is zero and the V-cycle returns (D^{-1}A)^{-1} y."""
    S, _, _ = small(10, 36, "cont", edit)
    MG = MultigridPreconditioner(S, 4e-4, 0.7)
    x = np.random.default_rng(3).standard_normal(S.N)
    z = MG(MG.scaled_operator(x))
    assert np.max(np.abs(z - x)) <= 1e-11 * np.max(np.abs(x))


@pytest.mark.parametrize("m,n,kind", [(3, 16, "psi"), (2, 33, "cont"), (3, 34, "psi")])
def test_vcycle_matches_its_error_propagation(m, n, kind):
    """B = the V-cycle as a matrix (applied to unit vectors).  Its error
    propagation I - B Â_0 must equal the product S_ℓ C_ℓ S_ℓ, with the
    smoothing step S_ℓ = I - K_ℓ Â_ℓ, the coarse-grid step
    C_ℓ = I - P_ℓ (I - E_{ℓ+1}) Â_{ℓ+1}^{-1} P_ℓ^T Â_ℓ and E = 0 on the
    directly solved ring-mean level, formed from dense matrices."""
    S, dt, th = small(m, n, kind)
    MG = MultigridPreconditioner(S, dt, th)
    N = S.N
    B = np.column_stack([MG.vcycle(0, e) for e in np.eye(N)])
    E0 = np.eye(N) - B @ MG.levels[0].Ah.toarray()
    E_next = None
    for l in range(len(MG.levels) - 1, -1, -1):
        lv = MG.levels[l]
        Nl = lv.Ah.shape[0]
        Ah, P = lv.Ah.toarray(), lv.P.toarray()
        K = np.column_stack([lv.line(e / (lv.V * lv.d)) for e in np.eye(Nl)])
        Sl = np.eye(Nl) - K @ Ah
        Ac = P.T @ Ah @ P
        inner = np.eye(Ac.shape[0]) if E_next is None else np.eye(Ac.shape[0]) - E_next
        Cl = np.eye(Nl) - P @ inner @ np.linalg.solve(Ac, P.T @ Ah)
        E_next = Sl @ Cl @ Sl
    assert np.max(np.abs(E0 - E_next)) <= 1e-9 * max(1.0, np.max(np.abs(E_next)))


def test_vcycle_contracts_where_the_smoother_alone_stalls():
    """On the steady Poisson problem the V-cycle's error propagation has a
    spectral radius near 0.3; two smoothing steps alone leave 0.86."""
    S, dt, th = small(8, 40, "psi")
    MG = MultigridPreconditioner(S, dt, th)
    N = S.N
    Ah = MG.levels[0].Ah.toarray()
    B = np.column_stack([MG.vcycle(0, e) for e in np.eye(N)])
    l0 = MG.levels[0]
    K = np.column_stack([l0.line(e / (l0.V * l0.d)) for e in np.eye(N)])
    Sm = np.eye(N) - K @ Ah
    rho_mg = max(abs(np.linalg.eigvals(np.eye(N) - B @ Ah)))
    rho_s = max(abs(np.linalg.eigvals(Sm @ Sm)))
    assert rho_mg < 0.45 and rho_s > 0.75


def iterations(A, b, M):
    A = sp.diags(1.0 / A.diagonal()) @ A
    cnt = [0]
    x, info = spla.bicgstab(A, b, M=spla.LinearOperator(A.shape, matvec=M), rtol=1e-10, maxiter=2000,
                            callback=lambda xk: cnt.__setitem__(0, cnt[0] + 1))
    assert info == 0
    return cnt[0], x


@pytest.mark.parametrize("kind", ["psi", "cont"])
def test_cuts_krylov_iterations_and_solves_the_system(kind):
    """Preconditioned BiCGSTAB on D^{-1} A: the V-cycle takes a fraction of
    the line preconditioner's iterations, and both reach the direct solve."""
    m, n = 48, 96
    S, dt, th = small(m, n, kind)
    A = system_matrix(S, dt, th).tocsr()
    b = np.random.default_rng(7).standard_normal(S.N)
    it_line, x_line = iterations(A, b, LinePreconditioner(S, dt, th))
    it_mg, x_mg = iterations(A, b, MultigridPreconditioner(S, dt, th))
    x = spla.spsolve(sp.diags(1.0 / A.diagonal()) @ A, b)
    for y in (x_line, x_mg):
        assert np.max(np.abs(y - x)) <= 1e-7 * np.max(np.abs(x))
    assert it_mg * 3 <= it_line, (it_mg, it_line)
