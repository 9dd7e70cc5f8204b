"""Pins of the oracle by the parameter sweeps of the paper's figures
(Figs 2.2, 2.5-2.7 and 2.9-2.11 of Ch. 2 §2.3, Figs 3.5-3.8 of Ch. 3 §3.3
and Figs 3.12-3.15 of Ch. 3 §3.4): the stored sweep table (tests/golden/fig_sweeps.json, written by the
oracle) is the oracle's current output, and it shows what the paper reports
of these figures: in Ch. 3 the mean error is smallest at q = 1.9 (Fig 3.6),
l = 1.5 (Fig 3.7) and a = 0.5 (Fig 3.8, after first rising with a), and a
small p is best (Fig 3.5, about 0.1 on the paper's grid); in Ch. 2 the
maximum error has an interior optimum in p (Figs 2.5, 2.6, 2.9, 2.10), the
best a moves up when the step shrinks (Fig 2.7 at Δt = 0.01 against Fig
2.11 at Δt = 0.02, on the finest swept mesh) and every sweep converges as
the mesh is refined, except Ch. 3 experiment 2 (Figs 3.12-3.15), whose
printed data give a mean error near 0.18 at every mesh.  A wrong exponent
in the angular or time stretch moves these optima; the Ch. 2 optima
themselves differ from the stated
ones (p about 0.9 rather than 1.1; a = 0.45 rather than towards 0.5 at
Δt = 0.01 and a = 0 rather than 0.4 at Δt = 0.02; for the stretch (2.13)
of Fig 2.2 the error falls all the way to p~ = 1 rather than having its
optimum near 0.6) and are not pinned."""

import json
import os

import numpy as np
import pytest

from helpers import oracle_fig_run
from problems.workloads import FIG_SWEEPS, fig_sweep_runs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fig_sweeps.json")


def golden():
    with open(GOLDEN) as f:
        return json.load(f)["figures"]


def test_golden_table_is_the_oracle():
    g = golden()
    for fig, m, n, prm in fig_sweep_runs((19,)):
        k = list(FIG_SWEEPS[fig]["values"]).index(prm[FIG_SWEEPS[fig]["vary"]])
        _, (mean, mx) = oracle_fig_run(fig, m, n, prm)
        e = g[fig]["m"]["19"]
        assert mean == pytest.approx(e["mean"][k], rel=1e-9) and mx == pytest.approx(e["max"][k], rel=1e-9)


@pytest.mark.parametrize("fig,best", [("fig_3_6", 1.9), ("fig_3_7", 1.5), ("fig_3_8", 0.5)])
def test_ch3_optima_are_the_papers(fig, best):
    f = golden()[fig]
    for m, e in f["m"].items():
        assert e["argmin"] == best, (fig, m)
        err = e[f["error"]]
        k = f["values"].index(best)
        # a clear optimum: its neighbours are worse by a margin above rounding
        for j in (k - 1, k + 1):
            if 0 <= j < len(err):
                assert err[j] > err[k] * (1 + 1e-4)


def test_ch3_error_first_rises_then_falls_with_a():
    f = golden()["fig_3_8"]
    v = f["values"]
    for m, e in f["m"].items():
        err = e["mean"]
        assert err[v.index(0.3)] > err[v.index(0.0)] and err[v.index(0.5)] < err[v.index(0.3)], m


def test_ch3_small_p_is_best():
    """Fig 3.5: on the paper's grid of p (from 0.1 up) the best is 0.1, and
    the mean error grows with p up to 0.4."""
    f = golden()["fig_3_5"]
    v = f["values"]
    for m, e in f["m"].items():
        err = e["mean"]
        on_grid = [k for k, p in enumerate(v) if p >= 0.1]
        assert v[min(on_grid, key=lambda k: err[k])] == 0.1
        assert err[v.index(0.1)] < err[v.index(0.2)] < err[v.index(0.4)]


def test_ch2_best_a_moves_up_as_the_step_shrinks():
    """Figs 2.7 (Δt = 0.01) and 2.11 (Δt = 0.02), p = 1.1: on the finest
    swept mesh the smaller step's best a is larger, and there its error at
    a = 0.45 is below the one at a = 0; at Δt = 0.02 the error only grows
    with a."""
    g = golden()
    f7, f11 = g["fig_2_7"], g["fig_2_11"]
    e7, e11 = f7["m"]["59"], f11["m"]["59"]
    assert e7["argmin"] > e11["argmin"]
    v = f7["values"]
    assert e7["max"][v.index(0.45)] < e7["max"][v.index(0.0)]
    assert all(a < b for a, b in zip(e11["max"], e11["max"][1:]))


@pytest.mark.parametrize("fig", ["fig_2_5", "fig_2_6", "fig_2_9", "fig_2_10"])
def test_ch2_interior_optimum_in_p(fig):
    f = golden()[fig]
    for m, e in f["m"].items():
        k = int(np.argmin(e["max"]))
        assert 0 < k < len(f["values"]) - 1, (fig, m)


def test_sweeps_converge_as_the_mesh_is_refined():
    """Every swept value's error falls from m = 19 to 39 to 59, except the
    printed stencil's runs at p >= 0.2 of Fig 3.5 (q = l = 1), whose mean
    error stays between 0.13 and 0.16 at every m, and Ch. 3 experiment 2
    (Figs 3.12-3.15, below)."""
    for fig, f in golden().items():
        if fig in CH3_EX2:
            continue
        for k, val in enumerate(f["values"]):
            if fig == "fig_3_5" and val >= 0.2:
                continue
            es = [f["m"][m][f["error"]][k] for m in ("19", "39", "59")]
            assert es[0] > es[1] > es[2], (fig, val, es)


CH3_EX2 = ("fig_3_12", "fig_3_13", "fig_3_14", "fig_3_15")


def test_ch3_experiment_2_does_not_converge_with_its_printed_data():
    """Figs 3.12-3.15 (Ch. 3 §3.4) with the printed stencil and source: the
    mean error sits between 0.10 and 0.20 at every swept value and changes
    by less than a fifth from m = 19 to 59, so the printed data of this
    experiment do not define a discretisation that converges to its
    printed solution (the paper's own Table 3.2 has mean errors of 0.20 to
    0.33 at m = 99); the optima the text states (p 0.5, q 5, l 5, a 0.1)
    are not pinned, and the sweeps serve as a batched workload with parity
    against the oracle only."""
    g = golden()
    for fig in CH3_EX2:
        f = g[fig]
        for k in range(len(f["values"])):
            es = [f["m"][m]["mean"][k] for m in ("19", "39", "59")]
            assert all(0.10 <= e <= 0.20 for e in es), (fig, es)
            assert abs(es[2] / es[0] - 1) < 0.2, (fig, es)


def test_table_3_2_first_column_within_six_percent():
    """A soft pin of experiment 2 against the paper: Table 3.2's first
    column (m = 99; p = 0.5, q = 5, l = 5, a = 0.1, Δt = 0.01 with the time
    stretch) prints a mean error of 1.97999984e-01; the oracle gives 0.1883
    (-4.9%).  Its other columns are not reproduced (up to a factor 2)."""
    m = 99
    _, (mean, _) = oracle_fig_run("fig_3_15", m, int(np.floor(2 * np.pi * m)), dict(p=0.5, q=5.0, l=5.0, a=0.1))
    assert abs(mean / 1.97999984e-01 - 1) < 0.06, mean
