"""GPU batching: instances of different sizes, PDE types and precisions
advanced together in the same launches give exactly the results they give
alone (an instance's reductions depend only on its own tiling), and the
full-size continuity workload matches the oracle step by step."""

import numpy as np
import pytest

from helpers import gpu_instance, l2_rel, max_rel, oracle_system
from oracle import solve, time_levels
from oracle.stepper import step as oracle_step
from problems import continuity_cfg, parabolic_family

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def make_set(precisions=(0, 0, 0)):
    from paper_2509_15879_amd import polardisk as pdk
    specs = [
        (continuity_cfg(1501, 40, 100), (40, 100, 1, 1.3, 1, 1.9), 0, 0.5, 12),
        (parabolic_family(1.0, 0.5), (33, 64, 0, 1.0, 0, 1.0), 0, 1.0, 7),
        (continuity_cfg(1502, 17, 130), (17, 130, 3, 0.6, 1, 2.5), 1, 0.7, 9),
    ]
    out = []
    for (pb, mesh, flux, theta, K), prec in zip(specs, precisions):
        inst = gpu_instance(pb, *mesh, precision=prec, flux=flux)
        td = pdk.time_desc(theta, K, 0.02, pdk.TIME_SINE, 1.5, tol=1e-12)
        out.append((inst, td))
    return out


@pytest.mark.parametrize("precisions", [(0, 0, 0), (1, 1, 1), (0, 1, 0)])
def test_alone_equals_batched(precisions):
    say(f"[batch] alone vs batched, precisions {precisions}")
    from paper_2509_15879_amd import polardisk as pdk
    alone = []
    for inst, td in make_set(precisions):
        inst.solve(td)
        alone.append(inst.solution())
        inst.close()
    pairs = make_set(precisions)
    stats = pdk.solve_batch([p[0] for p in pairs], [p[1] for p in pairs])
    for (inst, td), ref, st in zip(pairs, alone, stats):
        got = inst.solution()
        assert len(st) == td.K and all(s["status"] == 0 for s in st)
        assert np.array_equal(got, ref), max_rel(got, ref)
        inst.close()


def test_batch_of_uneven_lengths_finishes_each_instance():
    say("[batch] instances with 12, 7 and 9 levels")
    from paper_2509_15879_amd import polardisk as pdk
    pairs = make_set()
    stats = pdk.solve_batch([p[0] for p in pairs], [p[1] for p in pairs])
    for (inst, td), st in zip(pairs, stats):
        assert abs(st[-1]["t"] - 0.02) < 1e-15
        inst.close()


def test_cfg2_full_size_step_parity():
    """256 x 512 graded continuity mesh, the launch configuration of the
    benchmark: after 30 GPU levels, the next GPU level equals the oracle's
    step from the same state."""
    say("[batch] cfg2 full size: 30 GPU levels, then one level vs the oracle")
    from paper_2509_15879_amd import polardisk as pdk
    pb = continuity_cfg(1200, 256, 512, 0.5, 1.3)
    t = time_levels(0.05, 100, 1, 1.5)
    inst = gpu_instance(pb, 256, 512, 1, 1.3)
    inst.solve(pdk.time_desc(0.5, 30, table=t[:31], tol=1e-14))
    x30 = inst.solution(pdk.LAYOUT_PAPER)
    st = inst.solve(pdk.time_desc(0.5, 1, table=t[30:32], tol=1e-14))
    got = inst.solution(pdk.LAYOUT_PAPER)
    S, me = oracle_system(pb, 256, 512, 1, 1.3)
    ref = oracle_step(S, x30, t[30], t[31], 0.5)
    say(f"  iters {st[0]['iters']}, max-rel {max_rel(got, ref):.2e}")
    assert max_rel(got, ref) <= 1e-10
    inst.close()


def test_mixed_matches_fp64_on_cfg2_shape():
    """Mixed precision (FP32 inner, FP64 refinement) against the FP64 path on
    a quarter-size graded continuity problem over the whole time table."""
    say("[batch] mixed vs fp64, 128x256 graded, 50 levels")
    from paper_2509_15879_amd import polardisk as pdk
    pb = continuity_cfg(1203, 128, 256, 1.0, 1.3)
    a = gpu_instance(pb, 128, 256, 1, 1.3, precision=0)
    b = gpu_instance(pb, 128, 256, 1, 1.3, precision=1)
    td = pdk.time_desc(1.0, 50, 0.05, pdk.TIME_SINE, 1.5, tol=1e-13)
    pdk.solve_batch([a, b], [td, td])
    xa, xb = a.solution(), b.solution()
    say(f"  l2-rel mixed vs fp64 {l2_rel(xb, xa):.2e}")
    assert l2_rel(xb, xa) <= 1e-9
    a.close()
    b.close()


def test_graph_replay_equals_plain_launches(monkeypatch):
    """The captured cycle graph, replayed many times per level with eager
    launches and synchronisations in between, gives exactly the results of
    plain launches."""
    say("[batch] graph replay vs plain launches")
    from paper_2509_15879_amd import polardisk as pdk
    res = {}
    for mode in ("graph", "plain"):
        if mode == "plain":
            monkeypatch.setenv("PD_NO_GRAPH", "1")
        else:
            monkeypatch.delenv("PD_NO_GRAPH", raising=False)
        pairs = make_set((0, 1, 0))
        pdk.solve_batch([p[0] for p in pairs], [p[1] for p in pairs])
        res[mode] = [p[0].solution() for p in pairs]
        for p in pairs:
            p[0].close()
    for a, b in zip(res["graph"], res["plain"]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("schedule", [(2, 2), (3, 1), (2, 4)])
def test_stream_groups_give_identical_results(schedule):
    """A batch split over several streams (and any cycles per graph) gives
    exactly the results of one stream."""
    say(f"[batch] schedule {schedule} vs (1, 2)")
    from paper_2509_15879_amd import polardisk as pdk
    res = {}
    try:
        for sch in ((1, 2), schedule):
            pdk.set_schedule(*sch)
            pairs = make_set((0, 1, 0))
            pdk.solve_batch([p[0] for p in pairs], [p[1] for p in pairs])
            res[sch] = [p[0].solution() for p in pairs]
            for p in pairs:
                p[0].close()
    finally:
        pdk.set_schedule(1, 2)
    for a, b in zip(res[(1, 2)], res[schedule]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("precisions,bar", [((1, 1, 0), 1e-8), ((0, 0, 0), 1e-10)])
def test_deep_stencil_tiles(precisions, bar):
    """Instances under 8-ring stencil tiles: alone equals batched bit for bit
    under that schedule, and the results stay within the precision's bar
    (L2) of the FP64 solves under 4-ring tiles."""
    say(f"[batch] stencil tiles of 8 rings, precisions {precisions}")
    from paper_2509_15879_amd import polardisk as pdk
    ref = make_set((0, 0, 0))
    pdk.solve_batch([p[0] for p in ref], [p[1] for p in ref])
    xr = [p[0].solution() for p in ref]
    for p in ref:
        p[0].close()
    try:
        pdk.set_schedule(2, 2, 8)
        alone = []
        for inst, td in make_set(precisions):
            inst.solve(td)
            alone.append(inst.solution())
            inst.close()
        pairs = make_set(precisions)
        pdk.solve_batch([p[0] for p in pairs], [p[1] for p in pairs])
        batched = [p[0].solution() for p in pairs]
        for p in pairs:
            p[0].close()
    finally:
        pdk.set_schedule(1, 2)
    for a, b, r in zip(alone, batched, xr):
        assert np.array_equal(a, b)
        assert np.linalg.norm(b - r) / np.linalg.norm(r) <= bar


def test_autotune_leaves_the_state_and_picks_a_timed_candidate():
    say("[batch] autotuner")
    from paper_2509_15879_amd import autotune
    from paper_2509_15879_amd import polardisk as pdk
    pairs = make_set()
    insts, tds = [p[0] for p in pairs], [p[1] for p in pairs]
    before = [i.solution() for i in insts]
    try:
        out = autotune.tune(insts, tds, levels=2, candidates=((1, 2), (2, 2), (2, 4)),
                            use_cache=False)
        # every candidate under both stencil depths
        assert tuple(out["best"][:2]) in ((1, 2), (2, 2), (2, 4)) and out["best"][2] in (4, 8)
        assert len(out["ms"]) == 6
        assert pdk.get_schedule() == {"groups": out["best"][0], "cycles_per_graph": out["best"][1],
                                      "stencil_rings": out["best"][2]}
        for i, x in zip(insts, before):
            assert np.array_equal(i.solution(), x) and i.time == 0.0
    finally:
        pdk.set_schedule(1, 2)
        for i in insts:
            i.close()
