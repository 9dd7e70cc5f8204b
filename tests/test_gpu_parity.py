"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bars: FP64 max-relative difference <= 1e-10 (normwise, ||Δ||_∞ / ||n||_∞);
mixed precision L2-relative difference <= 1e-8.  Kernel-level checks (the
operator and the right-hand side) hold to a few ulps of the row sums.
"""

import numpy as np
import pytest

from helpers import DeviceBuffer, gpu_instance, hip_runtime, l2_rel, max_rel, oracle_system
from oracle import solve, time_levels
from oracle.stepper import rhs as oracle_rhs
from oracle.stepper import step as oracle_step
from problems import closed_form_quadratic, continuity_cfg, parabolic_cfg1, parabolic_family

pytestmark = pytest.mark.gpu

FP64_BAR = 1e-10
MIXED_BAR = 1e-8


def say(*a):
    print(*a, flush=True)


CASES = {
    # name: (problem factory, m, n, r_kind, p, th_kind, q, flux, bc)
    "parabolic_4x8": (lambda: parabolic_family(1.0, 0.5), 4, 8, 0, 1.0, 0, 1.0, 0, 0),
    "parabolic_b_33x64": (lambda: _with_b(parabolic_family(0.7, 0.3, 1.0)), 33, 64, 1, 1.0, 0, 1.0, 0, 0),
    "continuity_40x100": (lambda: continuity_cfg(1101, 40, 100), 40, 100, 1, 1.3, 1, 1.9, 0, 0),
    "continuity_up_zf_37x70": (lambda: continuity_cfg(1102, 37, 70), 37, 70, 1, 1.3, 0, 1.0, 1, 1),
    "continuity_2x4": (lambda: continuity_cfg(1103, 2, 4), 2, 4, 0, 1.0, 0, 1.0, 0, 0),
    "continuity_17x130": (lambda: continuity_cfg(1104, 17, 130), 17, 130, 3, 0.6, 1, 2.5, 1, 0),
}


EPS = np.finfo(np.float64).eps


def within_matvec_bound(got, ref, terms, c=64.0, mesh_terms=None, mesh_rel=None):
    """Elementwise forward-error bound of a matrix-vector product:
    |got - ref| <= c ε Σ |terms| (the absolute values of every summand),
    plus, where the two sides' meshes may differ, mesh_rel · mesh_terms."""
    bound = c * EPS * terms + 1e-300
    if mesh_terms is not None:
        bound = bound + mesh_rel * mesh_terms
    worst = float(np.max(np.abs(got - ref) / bound))
    return worst <= 1.0, worst


def mesh_sensitivity(me):
    """Per-row relative perturbation of the stencil coefficients caused by
    one-ulp differences between the two sides' mesh nodes (each side
    evaluates the stretch functions with its own libm): a node spacing δ
    next to a node of size s moves by ~2 ulp(s)/δ, and a coefficient
    carries up to two spacings.  Paper ordering."""
    from oracle.operator import to_vec
    m, n = me.m, me.n
    mu = me.mu
    h = me.h
    ang = 2 * np.spacing(2 * np.pi) / np.minimum(mu[:n], mu[1:n + 1])          # per j
    rad = 2 * np.spacing(1.0) / np.minimum(h[1:m + 1], h[2:m + 2])               # per i
    grid = 4 * (rad[:, None] + ang[None, :])
    return to_vec(4 * 2 * np.spacing(1.0) / h[1] + ang.max(), grid)


def _with_b(pb):
    pb.b = lambda r, th: 0.4 + 0.3 * r * np.cos(th) ** 2
    return pb


def setup_case(name, precision=0):
    f, m, n, rk, p, tk, q, flux, bc = CASES[name]
    pb = f()
    S, me = oracle_system(pb, m, n, rk, p, tk, q, flux, bc)
    inst = gpu_instance(pb, m, n, rk, p, tk, q, precision, flux, bc)
    return pb, S, inst


@pytest.mark.parametrize("name", sorted(CASES))
def test_operator_matches_oracle(name):
    say(f"[operator] {name}")
    pb, S, inst = setup_case(name)
    rng = np.random.default_rng(7)
    for dt, theta in [(1e-3, 0.5), (2.5e-5, 1.0), (0.3, 0.37)]:
        x = rng.standard_normal(S.N)
        got = inst.apply(x, dt, theta, layout=1)
        ref = x / dt + theta * (S.L @ x)
        lx = theta * (abs(S.L) @ np.abs(x))
        ok, worst = within_matvec_bound(got, ref, np.abs(x) / dt + lx, mesh_terms=lx,
                                        mesh_rel=mesh_sensitivity(S.mesh))
        assert ok, (dt, theta, worst)
        assert max_rel(got, ref) <= 1e-12, (dt, theta)
    inst.close()


def test_operator_full_size_cfg2():
    say("[operator] continuity 256x512 graded")
    pb = continuity_cfg(1200, 256, 512)
    S, me = oracle_system(pb, 256, 512, 1, 1.3)
    inst = gpu_instance(pb, 256, 512, 1, 1.3)
    x = np.random.default_rng(3).standard_normal(S.N)
    got = inst.apply(x, 7e-4, 0.5, layout=1)
    ref = x / 7e-4 + 0.5 * (S.L @ x)
    assert max_rel(got, ref) <= 1e-13
    inst.close()


def test_fp32_operator_matches_oracle():
    say("[operator fp32] continuity_40x100")
    pb, S, inst = setup_case("continuity_40x100", precision=1)
    x = np.random.default_rng(8).standard_normal(S.N)
    got = inst.apply(x, 1e-3, 0.5, layout=1, precision=1)
    ref = x / 1e-3 + 0.5 * (S.L @ x)
    assert max_rel(got, ref) <= 1e-5
    inst.close()


@pytest.mark.parametrize("name", ["parabolic_b_33x64", "continuity_40x100", "continuity_up_zf_37x70",
                                  "continuity_17x130"])
def test_rhs_matches_oracle(name):
    say(f"[rhs] {name}")
    pb, S, inst = setup_case(name)
    x0 = S.initial()
    for t0, dt, theta in [(0.0, 1e-3, 0.5), (0.013, 4e-4, 1.0)]:
        inst.set_solution(x0, t0, layout=1)
        got = inst.rhs(t0, dt, theta, layout=1)
        ref = oracle_rhs(S, x0, t0, t0 + dt, theta)
        ax = np.abs(x0)
        lx = (1 - theta) * (abs(S.L) @ ax) + np.abs(S.bnd_term(t0)) + np.abs(S.bnd_term(t0 + dt))
        terms = (ax / dt + lx
                 + (1 - theta) * np.abs(S.source(t0)) + theta * np.abs(S.source(t0 + dt)))
        ok, worst = within_matvec_bound(got, ref, terms, mesh_terms=lx,
                                        mesh_rel=mesh_sensitivity(S.mesh))
        assert ok, (t0, dt, theta, worst)
    inst.close()


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("name", sorted(CASES))
def test_single_step_matches_oracle(name, precision):
    say(f"[step] {name} precision={precision}")
    pb, S, inst = setup_case(name, precision)
    x0 = S.initial()
    for t0, dt, theta in [(0.0, 1e-3, 0.5), (0.001, 2e-5, 1.0)]:
        inst.set_solution(x0, t0, layout=1)
        st = inst.step(t0, dt, theta, tol=1e-13)
        got = inst.solution(layout=1)
        ref = oracle_step(S, x0, t0, t0 + dt, theta)
        if precision == 0:
            assert max_rel(got, ref) <= FP64_BAR, st
        else:
            assert l2_rel(got, ref) <= MIXED_BAR, st
    inst.close()


def test_cfg1_full_solve_fp64():
    say("[solve] parabolic cfg1 32x64, CN, dt=1e-3, 100 steps")
    pb = parabolic_cfg1()
    S, me = oracle_system(pb, 32, 64)
    ref = solve(S, time_levels(0.1, 100), 0.5)
    from paper_2509_15879_amd import polardisk as pdk
    inst = gpu_instance(pb, 32, 64)
    stats = inst.solve(pdk.time_desc(0.5, 100, 0.1, pdk.TIME_UNIFORM, tol=1e-13))
    got = inst.solution(layout=1)
    say(f"  iters/step {np.mean([s['iters'] for s in stats]):.1f}, max-rel {max_rel(got, ref):.2e}")
    assert max_rel(got, ref) <= FP64_BAR
    assert all(s["status"] == 0 for s in stats)
    inst.close()


@pytest.mark.parametrize("precision,theta", [(0, 0.5), (0, 1.0), (1, 0.5), (1, 1.0)])
def test_continuity_graded_solve(precision, theta):
    say(f"[solve] continuity 48x100 graded, V(t), precision={precision}, theta={theta}")
    from paper_2509_15879_amd import polardisk as pdk
    pb = continuity_cfg(1105, 48, 100)
    S, me = oracle_system(pb, 48, 100, 1, 1.3)
    ref = solve(S, time_levels(0.05, 20, 1, 1.5), theta)
    inst = gpu_instance(pb, 48, 100, 1, 1.3, precision=precision)
    stats = inst.solve(pdk.time_desc(theta, 20, 0.05, pdk.TIME_SINE, 1.5, tol=1e-13))
    got = inst.solution(layout=1)
    say(f"  iters/step {np.mean([s['iters'] for s in stats]):.1f}, "
        f"refinements {np.mean([s['refinements'] for s in stats]):.1f}, "
        f"max-rel {max_rel(got, ref):.2e}, l2-rel {l2_rel(got, ref):.2e}")
    if precision == 0:
        assert max_rel(got, ref) <= FP64_BAR
    else:
        assert l2_rel(got, ref) <= MIXED_BAR
    inst.close()


def test_closed_form_exact_on_gpu():
    say("[solve] closed form (1+t) r^2 + c on a uniform radial mesh")
    from paper_2509_15879_amd import polardisk as pdk
    from problems.manufactured import exact_at
    from oracle.operator import to_vec
    pb = closed_form_quadratic(0.25)
    inst = gpu_instance(pb, 20, 36, 0, 1.0, 1, 1.7)
    inst.solve(pdk.time_desc(0.6, 8, 0.3, pdk.TIME_SINE, 1.5, tol=1e-14))
    got = inst.solution(layout=1)
    r, _, th, _ = pdk.mesh_coords(inst.md)
    e0, eg = exact_at(pb, 0.3, r, th)
    assert max_rel(got, to_vec(e0, eg)) <= 1e-12
    inst.close()


def test_zero_flux_conserves_mass_on_gpu():
    say("[solve] zero-flux mass conservation 30x64")
    from paper_2509_15879_amd import polardisk as pdk
    from problems import zero_flux_random
    pb = zero_flux_random(11)
    S, me = oracle_system(pb, 30, 64, 1, 1.3, 1, 1.6, 0, 1)
    inst = gpu_instance(pb, 30, 64, 1, 1.3, 1, 1.6, 0, 0, 1)
    x0 = inst.solution(layout=1)
    inst.solve(pdk.time_desc(0.5, 10, 0.02, pdk.TIME_SINE, 1.5, tol=1e-14))
    x1 = inst.solution(layout=1)
    M0, M1 = S.V @ x0, S.V @ x1
    assert abs(M1 - M0) / abs(M0) <= 1e-12
    inst.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_wide_rings_solve(precision):
    """Rings of more than 1024 nodes run on four waves per ring (k_angw).
    n = 1100 is not a multiple of 8: the last threads own part of a segment
    and part of the fourth wave has no nodes.  Ring 1's arrow closure runs
    in the wide sweep too."""
    m, n, theta = 10, 1100, 0.5
    say(f"[solve] continuity {m}x{n} graded (four waves per ring), precision={precision}")
    from paper_2509_15879_amd import polardisk as pdk
    pb = continuity_cfg(1106, m, n)
    S, me = oracle_system(pb, m, n, 1, 1.3)
    ref = solve(S, time_levels(0.02, 6, 1, 1.5), theta)
    inst = gpu_instance(pb, m, n, 1, 1.3, precision=precision)
    stats = inst.solve(pdk.time_desc(theta, 6, 0.02, pdk.TIME_SINE, 1.5, tol=1e-13))
    got = inst.solution(layout=1)
    say(f"  iters/step {np.mean([s['iters'] for s in stats]):.1f}, "
        f"max-rel {max_rel(got, ref):.2e}, l2-rel {l2_rel(got, ref):.2e}")
    if precision == 0:
        assert max_rel(got, ref) <= FP64_BAR
    else:
        assert l2_rel(got, ref) <= MIXED_BAR
    inst.close()


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("m,n", [(2048, 64), (8, 2048)])
def test_maximum_ring_and_node_counts(m, n, precision):
    """The largest meshes the library accepts along each axis.  2048 rings
    give the radial sweep its longest segments (16 rows per thread, 128
    segments per column); 2048 nodes fill the four-wave ring sweep exactly
    (256 threads of 8 nodes)."""
    theta = 0.5
    say(f"[solve] continuity {m}x{n} graded (maximum counts), precision={precision}")
    from paper_2509_15879_amd import polardisk as pdk
    pb = continuity_cfg(1107, m, n)
    S, me = oracle_system(pb, m, n, 1, 1.3)
    ref = solve(S, time_levels(0.01, 3, 1, 1.5), theta)
    inst = gpu_instance(pb, m, n, 1, 1.3, precision=precision)
    stats = inst.solve(pdk.time_desc(theta, 3, 0.01, pdk.TIME_SINE, 1.5, tol=1e-13))
    got = inst.solution(layout=1)
    say(f"  iters/step {np.mean([s['iters'] for s in stats]):.1f}, "
        f"max-rel {max_rel(got, ref):.2e}, l2-rel {l2_rel(got, ref):.2e}")
    if precision == 0:
        assert max_rel(got, ref) <= FP64_BAR
    else:
        assert l2_rel(got, ref) <= MIXED_BAR
    inst.close()


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("case", ["zero", "constant"])
def test_degenerate_levels_finish_at_the_guess(case, precision):
    """Two problems whose every level is solved by its initial guess.
    "zero": no sources, zero boundary values and initial state; b = 0 at
    every level, the solution is exactly 0.  "constant": pure diffusion with
    zero-flux boundary and a constant initial state; every face flux of a
    constant vanishes exactly, so the state stays exactly at the constant.
    Each level must stop at its begin test with no iteration, and the
    least-squares guess, whose Gram matrix is all zeros or carries only
    rounding, must stay finite."""
    from paper_2509_15879_amd import polardisk as pdk
    from problems import TimeMode
    m, n = 24, 80
    zero = lambda r, th: np.zeros(np.broadcast(r, th).shape)  # noqa: E731
    pb = continuity_cfg(1108, m, n)
    pb.modes = [TimeMode(0.0, 0, zero, lambda th: np.zeros(np.shape(th)))]
    if case == "zero":
        pb.u0, bc, expect = zero, 0, 0.0
    else:
        pb.Er = pb.Et = None
        pb.u0, bc, expect = (lambda r, th: np.ones(np.broadcast(r, th).shape)), 1, 1.0
    say(f"[solve] degenerate '{case}' {m}x{n}, precision={precision}")
    inst = gpu_instance(pb, m, n, 1, 1.3, 1, 1.5, precision=precision, bc=bc)
    stats = inst.solve(pdk.time_desc(0.5, 8, 0.02, pdk.TIME_SINE, 1.5, tol=1e-13))
    got = inst.solution(layout=1)
    say(f"  iters {[s['iters'] for s in stats]}, max |x - {expect}| {np.max(np.abs(got - expect)):.2e}")
    assert np.all(np.isfinite(got))
    assert all(s["status"] == 0 and s["iters"] == 0 for s in stats)
    if case == "zero":
        assert np.all(got == 0.0)
    else:
        assert np.max(np.abs(got - 1.0)) <= 1e-14
    inst.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_explicit_irregular_mesh_solve(precision):
    """A mesh given node by node (the explicit kind): seeded spacings that
    vary up to 3:1 between neighbours in r and in θ, both sides built from
    the same node arrays."""
    from oracle import assemble, make_mesh
    from paper_2509_15879_amd import polardisk as pdk
    from problems import sample
    m, n, theta = 30, 90, 0.5
    rng = np.random.default_rng(1111)
    hr = rng.uniform(0.5, 1.5, m + 1)
    ht = rng.uniform(0.5, 1.5, n)
    r = np.concatenate([[0.0], np.cumsum(hr)]) / hr.sum()
    th = 2 * np.pi * np.concatenate([[0.0], np.cumsum(ht)]) / ht.sum()
    r[-1], th[-1] = 1.0, 2 * np.pi
    say(f"[solve] continuity {m}x{n} on an explicit irregular mesh, precision={precision}")
    pb = continuity_cfg(1111, m, n)
    me = make_mesh(m, n, 2, 1.0, 2, 1.0, r_explicit=r, th_explicit=th)
    S = assemble(me, sample(pb, *me.sample_points()))
    ref = solve(S, time_levels(0.02, 6, 1, 1.5), theta)
    md = pdk.mesh_desc(m, n, pdk.MESH_EXPLICIT, 1.0, pdk.MESH_EXPLICIT, 1.0, r_explicit=r, th_explicit=th)
    inst = pdk.Instance(md, sample(pb, *pdk.mesh_coords(md)), precision)
    stats = inst.solve(pdk.time_desc(theta, 6, 0.02, pdk.TIME_SINE, 1.5, tol=1e-13))
    got = inst.solution(layout=1)
    say(f"  iters/step {np.mean([s['iters'] for s in stats]):.1f}, "
        f"max-rel {max_rel(got, ref):.2e}, l2-rel {l2_rel(got, ref):.2e}")
    if precision == 0:
        assert max_rel(got, ref) <= FP64_BAR
    else:
        assert l2_rel(got, ref) <= MIXED_BAR
    inst.close()


def test_device_pointer_inputs_and_outputs():
    """Every array of the problem descriptor, λ and tpow included, may be a
    device pointer: an instance created from device copies solves bit for bit
    as the one created from host arrays.  Solutions read and written, an
    operator applied and a right-hand side assembled through device pointers
    equal the host-pointer calls."""
    import ctypes as C

    from paper_2509_15879_amd import polardisk as pdk
    from problems import sample
    m, n, theta = 20, 48, 0.5
    N = m * n + 1
    say(f"[device pointers] continuity {m}x{n}")
    hip = hip_runtime()
    md = pdk.mesh_desc(m, n, 1, 1.3)
    data = sample(continuity_cfg(1112, m, n), *pdk.mesh_coords(md))
    host = pdk.Instance(md, data, pdk.PD_FP64)
    pdd = pdk.problem_desc(data)
    bufs = []
    for field, key in (("b_node", "b"), ("D_rface", "Dr"), ("Er_rface", "Er"), ("D_tface", "Dt"),
                       ("Et_tface", "Et"), ("lam", "lam"), ("tpow", "tpow"), ("g", "g"), ("nb", "nb"),
                       ("u0", "u0")):
        if key in pdd._keep:
            bufs.append(DeviceBuffer(hip, pdd._keep[key]))
            setattr(pdd, field, bufs[-1].p.value)
    assert len(bufs) >= 9
    pdd.device_ptrs = 1
    devinst = pdk.Instance.from_desc(md, pdd, pdk.PD_FP64)
    td = pdk.time_desc(theta, 5, 0.02, pdk.TIME_SINE, 1.5, tol=1e-13)
    host.solve(td)
    devinst.solve(td)
    ref = host.solution(layout=1)
    assert np.array_equal(devinst.solution(layout=1), ref)
    out = DeviceBuffer(hip, np.zeros(N))
    pdk._check(pdk.lib.pd_get_solution(devinst.h, out.p, 1, 1))
    assert np.array_equal(out.read(), ref)
    x = DeviceBuffer(hip, 0.5 * ref + 0.25)
    pdk._check(pdk.lib.pd_set_solution(devinst.h, x.p, 1, 1, C.c_double(0.02)))
    assert np.array_equal(devinst.solution(layout=1), 0.5 * ref + 0.25)
    y = DeviceBuffer(hip, np.zeros(N))
    pdk._check(pdk.lib.pd_apply_operator(devinst.h, C.c_double(1e-3), C.c_double(theta), x.p, y.p, 1, 1, 0))
    assert np.array_equal(y.read(), host.apply(0.5 * ref + 0.25, 1e-3, theta, layout=1))
    host.set_solution(0.5 * ref + 0.25, 0.02, layout=1)
    pdk._check(pdk.lib.pd_assemble_rhs(devinst.h, C.c_double(0.02), C.c_double(1e-3), C.c_double(theta), y.p, 1, 1))
    assert np.array_equal(y.read(), host.rhs(0.02, 1e-3, theta, layout=1))
    say("  device-pointer create, get, set, apply and rhs match the host-pointer calls bit for bit")
    devinst.close()
    host.close()
    for b in bufs + [out, x, y]:
        b.free()
