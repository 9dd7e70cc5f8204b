"""Writes fig_sweeps.json: the FP64 oracle's errors over the parameter
sweeps of the paper's Figs 2.2, 2.5-2.7 and 2.9-2.11 (Ch. 2 §2.3, numerical
experiment 1), Figs 3.5-3.8 (Ch. 3 §3.3, numerical experiment 1) and Figs
3.12-3.15 (Ch. 3 §3.4, numerical experiment 2; printed stencil of §3.2.1 and
origin row of §3.2.2 for both), for m = 19, 39 and 59 rings.

The sweeps (swept parameter, fixed ones, levels) are those of
problems.workloads.FIG_SWEEPS; each run is solved by the oracle alone
(SuperLU per level) and its mean error over the ring unknowns and maximum
error over all unknowns at T are stored, with the swept value of the
smallest figure error per (figure, m).  About five minutes on one core.

    python tests/golden/make_fig_sweeps.py
"""

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
for p in (ROOT, os.path.dirname(HERE)):
    if p not in sys.path:
        sys.path.insert(0, p)

OUT = os.path.join(HERE, "fig_sweeps.json")
MS = (19, 39, 59)


def main():
    from helpers import oracle_fig_run
    from problems.workloads import FIG_EXAMPLES, FIG_SWEEPS, fig_sweep_runs
    out = {"source": ("arXiv:2509.15879, Figs 2.2, 2.5-2.7, 2.9-2.11 (Ch. 2 §2.3), Figs 3.5-3.8 (Ch. 3 §3.3) and "
                      "3.12-3.15 (Ch. 3 §3.4): "
                      "oracle errors over the swept parameter, written by tests/golden/make_fig_sweeps.py"),
           "figures": {}}
    for fig, m, n, prm in fig_sweep_runs(MS):
        _, (mean, mx) = oracle_fig_run(fig, m, n, prm)
        s = FIG_SWEEPS[fig]
        f = out["figures"].setdefault(fig, {"vary": s["vary"], "values": list(s["values"]),
                                            "error": FIG_EXAMPLES[s["example"]]["error"], "m": {}})
        f["m"].setdefault(str(m), {"mean": [], "max": []})
        f["m"][str(m)]["mean"].append(mean)
        f["m"][str(m)]["max"].append(mx)
        print(f"{fig} m={m} {s['vary']}={prm[s['vary']]}: mean {mean:.6e} max {mx:.6e}", flush=True)
    for fig, f in out["figures"].items():
        for m, e in f["m"].items():
            e["argmin"] = f["values"][int(np.argmin(e[f["error"]]))]
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
