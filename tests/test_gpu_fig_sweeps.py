"""The parameter sweeps of the paper's Figs 2.2, 2.5-2.7, 2.9-2.11 (Ch. 2
§2.3) and Figs 3.5-3.8 (Ch. 3 §3.3, printed stencil) on the GPU: every run
of the eleven sweeps at m = 19 and 39 (164 instances of uneven size, both
examples, both radial stretches, θ from 0.5 to 1) is solved as one batch,
each run's state is held against the oracle element by element, its
errors against the oracle's stored sweep table, and each sweep's optimum
against the table's."""

import json
import os

import numpy as np
import pytest

from helpers import fig_errors, fig_problem, max_rel, oracle_fig_run
from problems import sample
from problems.workloads import FIG_EXAMPLES, FIG_SWEEPS, fig_sweep_runs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fig_sweeps.json")


def say(*a):
    print(*a, flush=True)


def gpu_run(pdk, fig, m, n, prm):
    ex = FIG_EXAMPLES[FIG_SWEEPS[fig]["example"]]
    md = pdk.mesh_desc(m, n, ex["r_kind"], prm["p"], ex["th_kind"], prm["q"])
    coords = pdk.mesh_coords(md)
    flux = pdk.FLUX_LITERAL if ex["literal"] else pdk.FLUX_CENTRAL
    inst = pdk.Instance(md, sample(fig_problem(FIG_SWEEPS[fig]["example"]), *coords), pdk.PD_FP64, flux=flux)
    td = pdk.time_desc(1.0 - prm["a"], ex["K"], ex["T"], pdk.TIME_SINE if ex["t_kind"] else pdk.TIME_UNIFORM,
                       prm["l"], tol=1e-14)
    return inst, td, coords


def test_sweeps_batched_match_the_oracle():
    from paper_2509_15879_amd import polardisk as pdk
    with open(GOLDEN) as f:
        g = json.load(f)["figures"]
    runs = fig_sweep_runs((19, 39))
    built = [gpu_run(pdk, *r) for r in runs]
    say(f"[fig sweeps] {len(built)} instances batched, cells {sum(b[0].N for b in built)}")
    st = pdk.solve_batch([b[0] for b in built], [b[1] for b in built])
    assert all(s["status"] == 0 for x in st for s in x)
    got = {}
    worst_state = worst_err = 0.0
    for (fig, m, n, prm), (inst, td, coords) in zip(runs, built):
        x = inst.solution(pdk.LAYOUT_PAPER)
        inst.close()
        ex = FIG_EXAMPLES[FIG_SWEEPS[fig]["example"]]
        mean, mx = fig_errors(x, fig_problem(FIG_SWEEPS[fig]["example"]), ex["T"], coords[0], coords[2])
        ref, _ = oracle_fig_run(fig, m, n, prm)
        d = max_rel(x, ref)
        k = list(FIG_SWEEPS[fig]["values"]).index(prm[FIG_SWEEPS[fig]["vary"]])
        e = g[fig]["m"][str(m)]
        de = max(abs(mean / e["mean"][k] - 1), abs(mx / e["max"][k] - 1))
        worst_state, worst_err = max(worst_state, d), max(worst_err, de)
        assert d <= 1e-10, (fig, m, prm, d)
        assert de <= 1e-8, (fig, m, prm, de)
        got.setdefault((fig, m), []).append(mean if ex["error"] == "mean" else mx)
    say(f"  largest state max-rel vs oracle {worst_state:.2e}, largest error deviation {worst_err:.2e}")
    for (fig, m), errs in got.items():
        best = FIG_SWEEPS[fig]["values"][int(np.argmin(errs))]
        say(f"  {fig} m={m}: best {FIG_SWEEPS[fig]['vary']} = {best}")
        assert best == g[fig]["m"][str(m)]["argmin"]
