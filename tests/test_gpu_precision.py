"""Precision configuration at full size: the continuity problem on a
1024 x 2048 graded mesh (2,097,153 unknowns), fixed Δt = 2.5e-4, 200
levels.  The mixed-precision solve (FP32 inner, FP64 outer residual,
origin sum and pivots) stays within 1e-8 (L2) of the all-FP64 GPU solve,
and the FP64 state satisfies the oracle's own equations (its assembled
matrix and right-hand side at this size) for one more level."""

import numpy as np
import pytest

from helpers import l2_rel
from oracle import assemble, make_mesh
from oracle.stepper import rhs, system_matrix
from problems import continuity_cfg, sample

pytestmark = pytest.mark.gpu

M, N, P, DT, K, THETA = 1024, 2048, 1.3, 2.5e-4, 200, 0.5


def say(*a):
    print(*a, flush=True)


def test_cfg3_mixed_matches_fp64_and_fp64_satisfies_oracle_equations():
    from paper_2509_15879_amd import polardisk as pdk
    say("[precision] sampling 1024 x 2048")
    pb = continuity_cfg(1300, M, N, THETA, P)
    md = pdk.mesh_desc(M, N, pdk.MESH_SINE, P)
    data = sample(pb, *pdk.mesh_coords(md))
    a = pdk.Instance(md, data, pdk.PD_FP64)
    b = pdk.Instance(md, data, pdk.PD_MIXED)
    td = pdk.time_desc(THETA, K, DT * K, pdk.TIME_UNIFORM, tol=1e-12)
    say("[precision] 200 levels, FP64 and mixed batched")
    st = pdk.solve_batch([a, b], [td, td])
    xa, xb = a.solution(), b.solution()
    err = l2_rel(xb, xa)
    say(f"  iters/level fp64 {np.mean([s['iters'] for s in st[0]]):.1f}, "
        f"mixed {np.mean([s['iters'] for s in st[1]]):.1f} (+{np.mean([s['refinements'] for s in st[1]]):.2f} "
        f"refinements); L2 mixed vs fp64 {err:.2e}")
    assert err <= 1e-8
    # the initial guesses keep the iteration count low at this size (a guess
    # fitted badly, with the rounding of its normal equations at the scale
    # of the right-hand side, once took 40 iterations per level here)
    assert np.mean([s['iters'] for s in st[0]]) <= 12.0
    # one more FP64 level, checked against the oracle's matrix and right-hand side
    xk = a.solution(pdk.LAYOUT_PAPER)
    t0 = DT * K
    a.solve(pdk.time_desc(THETA, 1, table=[t0, t0 + DT], tol=1e-12))
    xk1 = a.solution(pdk.LAYOUT_PAPER)
    a.close()
    b.close()
    say("[precision] oracle assembly at full size")
    me = make_mesh(M, N, 1, P)
    S = assemble(me, sample(pb, *me.sample_points()))
    A = system_matrix(S, DT, THETA)
    rb = rhs(S, xk, t0, t0 + DT, THETA)
    d = A.diagonal()
    res = np.linalg.norm((rb - A @ xk1) / d) / np.linalg.norm(rb / d)
    say(f"  scaled residual of the GPU state in the oracle's equations {res:.2e}")
    assert res <= 1e-11
