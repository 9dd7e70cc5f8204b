"""The θ-semi-coarsening multigrid preconditioner on the GPU against the
oracle's oracle/multigrid.py: the V-cycle element by element (every level's
line factors are stored in FP32; the coarse correction and the second
smoothing step damp their rounding, measured at most 4e-8, against a bar of
1e-6, while a wrong merge, residual or correction shows as an O(1e-3..1)
difference), solves with it against the oracle's direct solves, its effect
on iteration counts, the coupled system solved with it, and the settings it
refuses."""

import numpy as np
import pytest

from helpers import max_rel
from oracle import assemble, make_mesh, solve, time_levels
from oracle.gummel import gummel_step as oracle_gummel, poisson_system
from oracle.multigrid import MultigridPreconditioner
from oracle.operator import to_vec
from problems import continuity_cfg, sample, two_carrier

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def pair(m, n, kind, seed=7101, bc=0, p=1.3):
    from paper_2509_15879_amd import polardisk as pdk
    pb = two_carrier(seed)[0] if kind == "psi" else continuity_cfg(seed, m, n, 0.5, p)
    me = make_mesh(m, n, 1, p)
    S = assemble(me, sample(pb, *me.sample_points()), bc=bc)
    md = pdk.mesh_desc(m, n, pdk.MESH_SINE, p)
    inst = pdk.Instance(md, sample(pb, *pdk.mesh_coords(md)), pdk.PD_FP64, bc=bc)
    pdk.set_preconditioner(inst, pdk.PRECOND_MG)
    return S, inst


# every level count from none (n < 16: level 0, then the ring means) up;
# odd line counts (three lines merged last); the radial sweep classes
# (m <= 256, <= 512, above) and the four-wave ring sweep (n > 1024) on level 0
CASES = [(20, 12, "cont"), (20, 48, "cont"), (24, 67, "psi"), (40, 130, "cont"), (300, 64, "psi"),
         (600, 32, "cont"), (12, 1100, "cont"), (33, 256, "psi")]


@pytest.mark.parametrize("m,n,kind", CASES)
def test_vcycle_matches_the_oracle(m, n, kind):
    from paper_2509_15879_amd import polardisk as pdk
    dt, theta = (1e30, 1.0) if kind == "psi" else (2.5e-4, 0.5)
    say(f"[mg] {m}x{n} {kind}: GPU V-cycle vs oracle")
    S, inst = pair(m, n, kind, seed=7102 + m)
    MG = MultigridPreconditioner(S, dt, theta)
    y = np.random.default_rng(m + n).standard_normal(S.N)
    z_ref = MG(y)
    before = inst.solution()
    z = inst.precondition(y, dt, theta, layout=pdk.LAYOUT_PAPER)
    err = max_rel(z, z_ref)
    say(f"  levels {[lv.n for lv in MG.levels]}, max-rel {err:.2e}")
    assert err <= 1e-6
    assert inst.time == 0.0 and np.array_equal(inst.solution(), before)
    inst.close()


def test_vcycle_with_zero_flux_boundary():
    from paper_2509_15879_amd import polardisk as pdk
    say("[mg] 30x80 zero-flux continuity: GPU V-cycle vs oracle")
    S, inst = pair(30, 80, "cont", seed=7110, bc=1)
    MG = MultigridPreconditioner(S, 1e-3, 1.0)
    y = np.random.default_rng(3).standard_normal(S.N)
    err = max_rel(inst.precondition(y, 1e-3, 1.0, layout=pdk.LAYOUT_PAPER), MG(y))
    say(f"  max-rel {err:.2e}")
    assert err <= 1e-6
    inst.close()


def test_vcycle_with_upwind_drift():
    """Upwind face pairs (gp and gm not symmetric about G): the merged
    faces and the coarse systems follow them."""
    from paper_2509_15879_amd import polardisk as pdk
    m, n = 28, 90
    say(f"[mg] {m}x{n} upwind continuity: GPU V-cycle vs oracle")
    pb = continuity_cfg(7160, m, n, 0.5, 1.3)
    me = make_mesh(m, n, 1, 1.3)
    S = assemble(me, sample(pb, *me.sample_points()), flux=1)
    md = pdk.mesh_desc(m, n, pdk.MESH_SINE, 1.3)
    inst = pdk.Instance(md, sample(pb, *pdk.mesh_coords(md)), pdk.PD_FP64, flux=1)
    pdk.set_preconditioner(inst, pdk.PRECOND_MG)
    MG = MultigridPreconditioner(S, 5e-4, 0.75)
    y = np.random.default_rng(9).standard_normal(S.N)
    err = max_rel(inst.precondition(y, 5e-4, 0.75, layout=pdk.LAYOUT_PAPER), MG(y))
    say(f"  levels {[lv.n for lv in MG.levels]}, max-rel {err:.2e}")
    assert err <= 1e-6
    inst.close()


def test_adaptive_steps_with_the_vcycle():
    """A-posteriori step control with the V-cycle: its coarse levels are
    refactored whenever Δt moves (the instance's own gate), and the run
    takes the same steps as with the line sweeps (the step control reads
    error estimates of solutions that agree to the solve's tolerance, so
    the levels agree to about 1e-8 relative) and reaches the same state."""
    from paper_2509_15879_amd import polardisk as pdk
    m, n = 40, 100
    say(f"[mg] adaptive steps {m}x{n}: V-cycle vs line sweeps")
    pb = continuity_cfg(7170, m, n, 1.0, 1.3)
    md = pdk.mesh_desc(m, n, pdk.MESH_SINE, 1.3)
    data = sample(pb, *pdk.mesh_coords(md))
    runs = {}
    for kind in (pdk.PRECOND_LINE, pdk.PRECOND_MG):
        inst = pdk.Instance(md, data, pdk.PD_FP64)
        pdk.set_preconditioner(inst, kind)
        st = pdk.taken(inst.solve(pdk.adaptive_time_desc(1.0, 0.02, 1e-5, 1e-6, 1e-6, 2e-3, tol=1e-13)))
        runs[kind] = (np.array([s["t"] for s in st]), sum(s["iters"] for s in st), inst.solution())
        say(f"  precond {kind}: {len(st)} steps, {runs[kind][1]} iterations")
        assert all(s["status"] == 0 for s in st)
        inst.close()
    (t0, i0, x0), (t1, i1, x1) = runs[pdk.PRECOND_LINE], runs[pdk.PRECOND_MG]
    say(f"  levels differ by {np.max(np.abs(t0 - t1)) / t0[-1]:.1e} (relative to T), "
        f"states by {max_rel(x1, x0):.1e}")
    assert len(t0) == len(t1) and np.max(np.abs(t0 - t1)) <= 1e-6 * t0[-1]
    assert max_rel(x1, x0) <= 1e-7
    assert i1 < i0


@pytest.mark.parametrize("form", ["reaction", "printed"])
def test_vcycle_with_a_reaction_term(form):
    """Levels that carry a reaction (volume-averaged when lines merge; the
    origin's is kept): a parabolic problem with b(r, θ), and the printed
    Ch. 3 stencil, whose diagonal beyond its faces is held as a reaction,
    on the angular and radial stretches (C15)."""
    from paper_2509_15879_amd import polardisk as pdk
    from oracle import assemble_literal
    from problems import paper_continuity_ex1
    from problems.manufactured import random_positive
    m, n = 26, 70
    say(f"[mg] {m}x{n} {form}: GPU V-cycle vs oracle")
    if form == "reaction":
        pb, rk, p, tk, q, flux = random_positive(7150, pde=0), 1, 1.3, 0, 1.0, 0
    else:
        pb, rk, p, tk, q, flux = paper_continuity_ex1(), 1, 0.5, 1, 1.9, pdk.FLUX_LITERAL
    me = make_mesh(m, n, rk, p, tk, q)
    od = sample(pb, *me.sample_points())
    S = assemble_literal(me, od) if form == "printed" else assemble(me, od)
    md = pdk.mesh_desc(m, n, rk, p, tk, q)
    inst = pdk.Instance(md, sample(pb, *pdk.mesh_coords(md)), pdk.PD_FP64, flux=flux)
    pdk.set_preconditioner(inst, pdk.PRECOND_MG)
    MG = MultigridPreconditioner(S, 2e-3, 0.5)
    y = np.random.default_rng(5).standard_normal(S.N)
    err = max_rel(inst.precondition(y, 2e-3, 0.5, layout=pdk.LAYOUT_PAPER), MG(y))
    say(f"  levels {[lv.n for lv in MG.levels]}, max-rel {err:.2e}")
    assert err <= 1e-6
    inst.close()


@pytest.mark.parametrize("theta", [0.5, 1.0])
def test_solve_matches_the_oracle_with_fewer_iterations(theta):
    """A graded continuity solve (sine-stretched levels) with the V-cycle
    reaches the oracle's direct solves, in fewer iterations than the line
    preconditioner on the same levels."""
    from paper_2509_15879_amd import polardisk as pdk
    m, n, K = 64, 128, 6
    say(f"[mg] solve 64x128, {K} levels, theta {theta}: multigrid vs line vs oracle")
    pb = continuity_cfg(7120, m, n, theta, 1.3)
    me = make_mesh(m, n, 1, 1.3)
    S = assemble(me, sample(pb, *me.sample_points()))
    ref = solve(S, time_levels(0.05, K, 1, 1.5), theta)
    md = pdk.mesh_desc(m, n, pdk.MESH_SINE, 1.3)
    data = sample(pb, *pdk.mesh_coords(md))
    its = {}
    for kind in (pdk.PRECOND_LINE, pdk.PRECOND_MG):
        inst = pdk.Instance(md, data, pdk.PD_FP64)
        pdk.set_preconditioner(inst, kind)
        stats = inst.solve(pdk.time_desc(theta, K, 0.05, pdk.TIME_SINE, 1.5, tol=1e-13))
        got = inst.solution(layout=pdk.LAYOUT_PAPER)
        its[kind] = [s["iters"] for s in stats]
        say(f"  precond {kind}: iterations {its[kind]}, max-rel {max_rel(got, ref):.2e}")
        assert max_rel(got, ref) <= 1e-10
        assert all(s["status"] == 0 for s in stats)
        inst.close()
    assert sum(its[pdk.PRECOND_MG]) * 2 <= sum(its[pdk.PRECOND_LINE])


def test_gummel_step_in_a_fraction_of_the_iterations():
    """The coupled system solved with the V-cycle for the potential (a
    steady Poisson problem) and both carriers: the Gummel step matches the
    oracle's, with far fewer Krylov iterations than with the line sweeps."""
    from paper_2509_15879_amd import polardisk as pdk
    m, n = 48, 120
    say(f"[mg] Gummel step {m}x{n}: V-cycle vs line sweeps for all three fields vs the oracle")
    psi_pb, n_pb, p_pb = two_carrier(7130)
    me = make_mesh(m, n, 1, 1.3)
    od = [sample(pb, *me.sample_points()) for pb in (psi_pb, n_pb, p_pb)]
    Sp = poisson_system(me, od[0])
    x = [to_vec(d["u0_origin"], d["u0_grid"]) for d in od]
    ref = oracle_gummel(me, Sp, od[1], od[2], x[0], x[1], x[2], 0.0, 0.01, 0.5, 3)
    md = pdk.mesh_desc(m, n, pdk.MESH_SINE, 1.3)
    coords = pdk.mesh_coords(md)
    gd = [sample(pb, *coords) for pb in (psi_pb, n_pb, p_pb)]
    kry = {}
    for kind in (pdk.PRECOND_LINE, pdk.PRECOND_MG):
        psi = pdk.Instance(md, gd[0], pdk.PD_FP64)
        car = [pdk.Instance(md, gd[k], pdk.PD_FP64) for k in (1, 2)]
        for inst, d, sign in zip(car, gd[1:], (-1.0, 1.0)):
            pdk.set_mobility(inst, d["D_r"], d["D_t"], sign)
        for inst in [psi] + car:
            pdk.set_preconditioner(inst, kind)
        st = pdk.gummel_step(psi, car[0], car[1], 0.0, 0.01, 0.5, tol=1e-14, gummel_tol=0.0, max_gummel=3)
        got = [i.solution(pdk.LAYOUT_PAPER) for i in (psi, car[0], car[1])]
        errs = [max_rel(g, r) for g, r in zip(got, ref[:3])]
        kry[kind] = st["krylov_iters"]
        say(f"  precond {kind}: krylov {st['krylov_iters']}, max-rel {max(errs):.2e}")
        assert max(errs) <= 1e-9
        for i in [psi] + car:
            i.close()
    assert kry[pdk.PRECOND_MG] * 4 <= kry[pdk.PRECOND_LINE]


def test_refused_settings_and_batches():
    """Multigrid instances batch with FP64 instances (each keeps its own
    result: the same as solving it alone) and are refused next to a
    mixed-precision one; mixed precision and unknown kinds are refused."""
    from paper_2509_15879_amd import polardisk as pdk
    say("[mg] batches with FP64 instances; refused: mixed precision, an unknown kind")
    pb = continuity_cfg(7140, 16, 40)
    md = pdk.mesh_desc(16, 40)
    data = sample(pb, *pdk.mesh_coords(md))
    mixed = pdk.Instance(md, data, pdk.PD_MIXED)
    with pytest.raises(pdk.PolarDiskError, match="FP64 instances"):
        pdk.set_preconditioner(mixed, pdk.PRECOND_MG)
    with pytest.raises(pdk.PolarDiskError, match="unknown preconditioner"):
        pdk.set_preconditioner(mixed, 7)
    a, b, c = (pdk.Instance(md, data, pdk.PD_FP64) for _ in range(3))
    pdk.set_preconditioner(a, pdk.PRECOND_MG)
    pdk.set_preconditioner(c, pdk.PRECOND_MG)
    td = pdk.time_desc(0.5, 3, 0.01, pdk.TIME_UNIFORM, tol=1e-12)
    with pytest.raises(pdk.PolarDiskError, match="FP64 instances only"):
        pdk.solve_batch([a, mixed], [td, td])
    # a batch of a multigrid, a line and a multigrid instance; each result
    # equals the same instance solved alone with its own preconditioner
    for i in (a, b, c):
        i.set_solution(pdk.ring_vector(data["u0_origin"], data["u0_grid"]), 0.0)
    st = pdk.solve_batch([a, b, c], [td, td, td])
    alone = []
    for kind in (pdk.PRECOND_MG, pdk.PRECOND_LINE):
        d = pdk.Instance(md, data, pdk.PD_FP64)
        pdk.set_preconditioner(d, kind)
        d.solve(td)
        alone.append(d.solution())
        d.close()
    say(f"  batched iterations {[[s['iters'] for s in x] for x in st]}")
    assert np.array_equal(a.solution(), alone[0]) and np.array_equal(c.solution(), alone[0])
    assert np.array_equal(b.solution(), alone[1])
    assert sum(s["iters"] for s in st[0]) < sum(s["iters"] for s in st[1])
    # back to the line sweeps
    pdk.set_preconditioner(a, pdk.PRECOND_LINE)
    a.set_solution(pdk.ring_vector(data["u0_origin"], data["u0_grid"]), 0.0)
    a.solve(td)
    assert np.array_equal(a.solution(), alone[1])
    for i in (mixed, a, b, c):
        i.close()
