"""Failure paths, forced from the host (every kernel still exits normally):
a step that hits its iteration cap, a non-finite initial state, a solve
stopped by its wall-clock limit, and a failing request in the serving loop.
In each case the failing instance reports its error and the others of the
same launches stay bit-identical to solving alone."""

import numpy as np
import pytest

from helpers import gpu_instance
from problems import continuity_cfg, parabolic_family

pytestmark = pytest.mark.gpu

PD_EBREAKDOWN, PD_ENOCONV = -3, -4

# (problem, m, n, r_kind, p, theta)
SPECS = [
    (lambda: continuity_cfg(4101, 24, 40), 24, 40, 1, 1.3, 0.5),
    (lambda: parabolic_family(1.0, 0.4), 20, 36, 0, 1.0, 1.0),
    (lambda: continuity_cfg(4102, 32, 48), 32, 48, 1, 1.3, 0.7),
]


def say(*a):
    print(*a, flush=True)


def make(spec, precision=0):
    mk, m, n, rk, p, _ = spec
    return gpu_instance(mk(), m, n, rk, p, precision=precision)


def tdesc(spec, **kw):
    from paper_2509_15879_amd import polardisk as pdk
    return pdk.time_desc(spec[5], 8, 0.02, pdk.TIME_SINE, 1.5, tol=1e-12, **kw)


def alone(spec, precision=0):
    inst = make(spec, precision)
    inst.solve(tdesc(spec))
    x = inst.solution()
    inst.close()
    return x


@pytest.mark.parametrize("precision", [0, 1])
def test_iteration_cap_fails_one_instance_only(precision):
    say(f"[failure] max_iters=1 on one instance of three, precision {precision}")
    from paper_2509_15879_amd import polardisk as pdk
    insts = [make(s, precision) for s in SPECS]
    tds = [tdesc(SPECS[0]), tdesc(SPECS[1], max_iters=1), tdesc(SPECS[2])]
    with pytest.raises(pdk.PolarDiskError) as ei:
        pdk.solve_batch(insts, tds)
    assert ei.value.code == PD_ENOCONV
    for q in (0, 2):
        assert np.array_equal(insts[q].solution(), alone(SPECS[q], precision)), q
    # the capped instance stopped at its first level
    assert insts[1].time == pytest.approx(pdk.time_levels(tds[1])[1], abs=0.0)
    for i in insts:
        i.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_nan_state_breaks_down_one_instance_only(precision):
    say(f"[failure] NaN in the initial state of one instance of three, precision {precision}")
    from paper_2509_15879_amd import polardisk as pdk
    insts = [make(s, precision) for s in SPECS]
    x0 = insts[1].solution()
    x0[7] = np.nan
    insts[1].set_solution(x0, 0.0)
    tds = [tdesc(s) for s in SPECS]
    with pytest.raises(pdk.PolarDiskError) as ei:
        pdk.solve_batch(insts, tds)
    assert ei.value.code == PD_EBREAKDOWN
    for q in (0, 2):
        assert np.array_equal(insts[q].solution(), alone(SPECS[q], precision)), q
    for i in insts:
        i.close()


def test_wall_clock_limit_stops_a_solve_and_the_instance_stays_usable():
    say("[failure] wall-clock limit reached before the first round")
    from paper_2509_15879_amd import polardisk as pdk
    inst = make(SPECS[0])
    with pytest.raises(pdk.PolarDiskError, match="wall-clock") as ei:
        inst.solve(tdesc(SPECS[0], max_seconds=1e-9))
    assert ei.value.code == PD_ENOCONV
    assert inst.time == 0.0
    inst.solve(tdesc(SPECS[0]))
    assert np.array_equal(inst.solution(), alone(SPECS[0]))
    inst.close()


def test_failing_request_leaves_the_served_batch_unaffected():
    say("[failure] serving: a request capped at one iteration among good ones; a NaN request refused")
    from paper_2509_15879_amd import polardisk as pdk
    from problems import sample
    B = pdk.Batch(4 << 30, 8)
    tickets = []
    for q, spec in enumerate(SPECS):
        mk, m, n, rk, p, _ = spec
        md = pdk.mesh_desc(m, n, rk, p)
        data = sample(mk(), *pdk.mesh_coords(md))
        if q == 1:
            bad = dict(data)
            grid = np.array(data["u0_grid"], dtype=float, copy=True)
            grid.reshape(-1)[5] = np.nan
            bad["u0_grid"] = grid
            with pytest.raises(pdk.PolarDiskError, match="non-finite"):
                B.submit(md, bad, tdesc(spec), pdk.PD_FP64)
        td = tdesc(spec, max_iters=1) if q == 1 else tdesc(spec)
        tickets.append(B.submit(md, data, td, pdk.PD_FP64))
    results = {}
    for q, t in enumerate(tickets):
        try:
            results[q] = B.wait(t)
        except pdk.PolarDiskError as e:
            results[q] = e
    B.close()
    assert isinstance(results[1], pdk.PolarDiskError) and results[1].code == PD_ENOCONV
    for q in (0, 2):
        x, sm = results[q]
        assert sm["status"] == 0
        assert np.array_equal(x, alone(SPECS[q])), q
