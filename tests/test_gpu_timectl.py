"""Adaptive time stepping on the GPU: the accepted time levels it logs,
replayed by the oracle, give the same state (≤ 1e-10); its step sequence
follows the oracle's own controller (same rules, exact solves); and the
controller's invariants hold (landing on T, bounds, growth, accepted
errors).  Decisions come from error estimates that the solve's rounding
perturbs slightly, so the sequences are compared with a tolerance and
parity is taken on the GPU's own sequence (the decisions are logged and
replayed)."""

import numpy as np
import pytest

from helpers import gpu_instance, max_rel, oracle_system
from oracle.timectl import solve_adaptive, solve_levels
from problems import continuity_cfg

pytestmark = pytest.mark.gpu

T, DT_MIN, DT_MAX = 0.05, 1e-5, 1e-3


def say(*a):
    print(*a, flush=True)


# (θ, tolerance, first step): the last two start too large and are rejected
@pytest.mark.parametrize("theta,tol_time,dt0", [(0.5, 1e-8, 1e-5), (1.0, 1e-6, 1e-5), (0.7, 1e-6, 1e-5),
                                                (0.5, 1e-8, 1e-3), (1.0, 1e-6, 1e-3)])
def test_adaptive_steps_match_the_oracle(theta, tol_time, dt0):
    from paper_2509_15879_amd import polardisk as pdk
    m, n = 24, 48
    pb = continuity_cfg(4201, m, n, theta, 1.3)
    inst = gpu_instance(pb, m, n, 1, 1.3)
    say(f"[timectl] theta {theta}, tol_time {tol_time}, dt0 {dt0}")
    st = pdk.taken(inst.solve(pdk.adaptive_time_desc(theta, T, dt0, tol_time, DT_MIN, DT_MAX, tol=1e-14)))
    x = inst.solution(pdk.LAYOUT_PAPER)
    lv = np.array([0.0] + [s["t"] for s in st])
    dts = np.diff(lv)
    rej = sum(s["rejected"] for s in st)
    say(f"  GPU: {len(st)} steps, {rej} rejected, dt {dts.min():.2e}..{dts.max():.2e}")
    # invariants
    assert all(s["status"] == 0 for s in st)
    assert lv[-1] == T and np.all(dts > 0) and inst.time == T
    assert np.all(dts <= DT_MAX * (1 + 1e-12))
    assert np.all(dts[1:-2] / dts[:-3] <= 2.0 * (1 + 1e-12))
    assert all(s["err_time"] <= 2 * tol_time for s in st[1:] if s["dt"] > DT_MIN)
    # the oracle replays the logged levels
    S, _ = oracle_system(pb, m, n, 1, 1.3)
    ref = solve_levels(S, lv, theta, adaptive_start=True)
    say(f"  replay max-rel {max_rel(x, ref):.2e}")
    assert max_rel(x, ref) <= 1e-10
    # the oracle's own controller
    xo, lvo, steps, rejo = solve_adaptive(S, theta, T, dt0, tol_time, DT_MIN, DT_MAX)
    say(f"  oracle: {len(steps)} steps, {rejo} rejected")
    assert abs(len(steps) - len(st)) <= max(1, len(st) // 20) and rejo == rej
    k = min(len(lvo), len(lv)) - 1
    rel = np.max(np.abs(np.diff(lvo[:k]) - dts[:k - 1]) / dts[:k - 1])
    say(f"  dt sequences: largest relative difference over {k - 1} steps {rel:.2e}")
    assert rel <= 1e-4
    inst.close()


def test_adaptive_batch_equals_alone():
    """Instances stepping adaptively with different θ in one batch take the
    same steps and reach the same states as alone."""
    from paper_2509_15879_amd import polardisk as pdk
    specs = [(0.5, 4202, 20, 40), (1.0, 4203, 16, 64)]
    alone = []
    for th, seed, m, n in specs:
        inst = gpu_instance(continuity_cfg(seed, m, n, th, 1.3), m, n, 1, 1.3)
        st = pdk.taken(inst.solve(pdk.adaptive_time_desc(th, T, 1e-5, 1e-6, DT_MIN, DT_MAX)))
        alone.append((inst.solution(), [s["t"] for s in st]))
        inst.close()
    insts = [gpu_instance(continuity_cfg(seed, m, n, th, 1.3), m, n, 1, 1.3) for th, seed, m, n in specs]
    sts = pdk.solve_batch(insts, [pdk.adaptive_time_desc(th, T, 1e-5, 1e-6, DT_MIN, DT_MAX) for th, *_ in specs])
    for inst, st, (xa, ta) in zip(insts, sts, alone):
        assert [s["t"] for s in pdk.taken(st)] == ta
        assert np.array_equal(inst.solution(), xa)
        inst.close()
