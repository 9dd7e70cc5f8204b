#!/usr/bin/env python
"""Throughput benchmark of the polar-disk θ-scheme solver on one MI355X.

Headline workload (one "step" = one pass of the whole hot path): the
drift-diffusion continuity problem on a 1024 x 2048 polar mesh graded
towards r = 0 and r = 1 (radial stretch (2.4), p = 1.3; 2,097,153
unknowns), seeded diffusivity D = 1 + ½ sin(kθ) r² and Fourier-Bessel drift
E = -∇ψ, manufactured exact solution, Crank-Nicolson (θ = 0.5), fixed
Δt = 2.5e-4, 200 levels to T = 0.05, all in FP64.  Metric: cell-updates/s =
unknowns x levels / wall time, valid when the result is within 1e-8
(L2-relative) of the FP64 oracle's solution of the same 200 levels, whose
samples are stored by tests/golden/make_cfg3_reference.py.  The oracle
(FP64 sparse LU on the host) is timed on a bounded sample of the same
workload in a child process beside the GPU legs.  Variants (not the
headline): the same workload in mixed precision, the ten-instance 256 x 512
batch, adaptive time steps, the runs of Table 2.1, the 512-instance uneven
sweep and the serving loop under a Poisson request stream.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from problems.workloads import CFG2, CFG2_SEEDS as SEEDS, CFG2_THETAS as THETAS, cfg2_batch  # noqa: E402

M, N_TH, P_STRETCH, T_END, K_LEVELS, L_TIME = (CFG2[k] for k in ("m", "n", "p", "T", "K", "l"))
HBM_PEAK_GBS = 8000.0
TUNE_LEVELS = 10         # levels the schedule autotuner times each candidate on (the
                         # benchmark batch itself is tuned on whole solves)
ADAPTIVE_CPG = (2, 4, 6)  # cycles per graph tried for the adaptive-step variant
# One instance is one stream group whatever the schedule says, so its
# candidates are the round lengths and stencil depths alone, timed on whole
# solves: the first levels (cold, with little history to extrapolate from)
# ranked the mixed-precision schedules differently from the whole run
# (12 cycles and 4-ring tiles first: 261 ms; 7 cycles and 8-ring tiles: 239).
SINGLE_CANDIDATES = tuple((1, c) for c in (6, 7, 8, 12))

# Algorithmic bytes per unknown of one launch (w: storage bytes of the
# Krylov data; the sweeps' factors are FP32): what the kernel must read and
# write once.
KERNEL_NAMES = {
    "sten_v": "k_sten<T, SM_V>", "sten_t": "k_sten<T, SM_T>", "rad_p": "k_rad<T, RM_P, BM>",
    "rad_s": "k_rad<T, RM_S, BM>", "ang_p": "k_ang<T, AM_P, BM>", "ang_s": "k_ang<T, AM_S, BM>",
    "update": "k_elem_x<T>",
}


# HBM bytes per active unknown that each kernel moved on the headline
# workload (FETCH_SIZE and WRITE_SIZE counters, calibrated on a copy of known
# size), valid for the sources with this SHA-1 only (kernel_source_sha1);
# any other source reports traffic null.
TRAFFIC = {
    "cfg3_fp64": {
        "sha1": "6bc4b8abe6894ef49f1ea3b4c1e356097a1a2160",
        "w": 8,
        "stencil_rings": 8,
        "b_per_cell": {"rad_p": 52.95, "ang_p": 32.23, "sten_v": 65.13, "rad_s": 44.16, "ang_s": 32.23,
                       "sten_t": 64.88, "update": 64.34},
    },
    # the FP32 inner cycle of the same instance in mixed precision
    "cfg3_mixed": {
        "sha1": "6bc4b8abe6894ef49f1ea3b4c1e356097a1a2160",
        "w": 4,
        "stencil_rings": 8,
        "b_per_cell": {"rad_p": 32.24, "ang_p": 24.22, "sten_v": 37.96, "rad_s": 28.14, "ang_s": 24.22,
                       "sten_t": 37.92, "update": 32.26},
    },
}


def code_digest(texts):
    """SHA-1 of C++/HIP sources with comments and blank lines removed."""
    import hashlib
    import re
    h = hashlib.sha1()
    for src in texts:
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        src = re.sub(r"//[^\n]*", "", src)
        code = "\n".join(line.rstrip() for line in src.splitlines() if line.strip())
        h.update(code.encode("utf-8"))
    return h.hexdigest()


def kernel_source_sha1():
    """Digest of the kernels' source and of the host runtime that lays out
    their launches (the block maps decide which tiles share an L2), without
    comments and blank lines: an edit of the comments leaves the measured
    traffic valid, any change of the code voids it."""
    texts = []
    for name in ("pd_kernels.hip", "pd_host.cpp"):
        with open(os.path.join(ROOT, "paper_2509_15879_amd", "csrc", name), encoding="utf-8") as f:
            texts.append(f.read())
    return code_digest(texts)


def bytes_per_cell(family, w):
    return {
        # p̂ or ŝ, 4 face coefficients, r̂ or s in; v or t out; FP32 also reads
        # its 1/diag copy (FP64 forms 1/diag from the faces)
        "sten_v": 7 * w + (4 if w == 4 else 0),
        "sten_t": 7 * w + (4 if w == 4 else 0),
        "rad_p": 5 * w + 12,        # r, p, v in; p, w out; f, g, pivot (FP32) in
        "rad_s": 4 * w + 12,        # r, v in; s, w out; f, g, pivot (FP32) in
        "ang_p": 2 * w + 16,        # w in; p̂ out; f, g, z, pivot (FP32) in
        "ang_s": 2 * w + 16,        # w in; ŝ out; f, g, z, pivot (FP32) in
        "update": 8 * w,            # p̂, ŝ, x, s, t, r̂ in; x, r out
    }[family]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_instances(pdk, precision, stream):
    from problems import sample
    insts, tds, u0s = [], [], []
    for seed, th, pb in cfg2_batch():
        md = pdk.mesh_desc(M, N_TH, pdk.MESH_SINE, P_STRETCH)
        data = sample(pb, *pdk.mesh_coords(md))
        inst = pdk.Instance(md, data, precision, stream=stream)
        insts.append(inst)
        u0s.append(pdk.ring_vector(data["u0_origin"], data["u0_grid"]))
        tds.append((th, pb))
    return insts, tds, u0s


def time_descs(pdk, tds, tol):
    return [pdk.time_desc(th, K_LEVELS, T_END, pdk.TIME_SINE, L_TIME, tol=tol) for th, _ in tds]


def reset(insts, u0s):
    for inst, u0 in zip(insts, u0s):
        inst.set_solution(u0, 0.0)


def mixed_cfg3_variant(pdk, stream, tol, ref):
    """The headline workload in mixed precision (FP32 inner iterations, FP64
    refinement), under its own tuned schedule, against the oracle's stored
    samples."""
    import torch
    from paper_2509_15879_amd import autotune
    from problems.workloads import CFG3
    c = CFG3
    cells = c["m"] * c["n"] + 1
    inst, u0 = cfg3_instance(pdk, pdk.PD_MIXED, stream)
    desc = cfg3_desc(pdk, tol)
    inst.set_solution(u0, 0.0)
    tuned = autotune.tune([inst], [desc], levels=c["K"], candidates=SINGLE_CANDIDATES, repeats=1,
                          sync=torch.cuda.synchronize)
    best, st = float("inf"), None
    for rep in range(2):
        inst.set_solution(u0, 0.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = inst.solve(desc)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    x = inst.solution(pdk.LAYOUT_PAPER)
    inner = int(sum(s["iters"] for s in st))

    def run_step():
        inst.set_solution(u0, 0.0)
        inst.solve(desc)

    # the FP32 inner cycle's dominant kernel, on one more, event-stamped run
    roof = roofline_of(pdk, run_step, 4, cells * inner, TRAFFIC.get("cfg3_mixed"), instance_iters=inner,
                       stencil_rings=tuned["best"][2])
    inst.close()
    return {"value": round(cells * c["K"] / best, 1), "ms": round(1e3 * best, 1), "tol_per_step": tol,
            "schedule": list(tuned["best"]), "autotune_ms_whole_solves": tuned["ms"],
            "roofline": roof,
            "vs_oracle": vs_oracle_samples(x, ref, c["K"]),
            "inner_iters_per_level": round(float(np.mean([s["iters"] for s in st])), 2),
            "refinements_per_level": round(float(np.mean([s["refinements"] for s in st])), 2)}


def uneven_variant(pdk, stream, tol, sample_alone=32):
    """512 uneven instances (m log-uniform in [32, 512], n in [64, 1024], half
    parabolic, half drift-diffusion, θ in [0.5, 1], fixed Δt = 5e-4, 100
    levels): the mixed-precision batch under the autotuned schedule against
    a converged FP64 batch, and FP64 one instance at a time on a sample."""
    import torch
    from paper_2509_15879_amd import autotune
    from problems import sample
    from problems.workloads import CFG4, cfg4_batch
    c = CFG4
    specs = cfg4_batch()
    datas, mds, tds = [], [], []
    for q, m, n, theta, pb in specs:
        md = pdk.mesh_desc(m, n, pdk.MESH_SINE, c["p"])
        mds.append(md)
        datas.append(sample(pb, *pdk.mesh_coords(md)))
        tds.append(pdk.time_desc(theta, c["K"], c["dt"] * c["K"], pdk.TIME_UNIFORM, tol=tol))
    cells = sum(m * n + 1 for _, m, n, _, _ in specs)

    def make(prec):
        return [pdk.Instance(md, d, prec, stream=stream) for md, d in zip(mds, datas)]

    ref_insts = make(pdk.PD_FP64)
    ref_tds = [pdk.time_desc(td.theta, td.K, td.T, pdk.TIME_UNIFORM, tol=1e-13) for td in tds]
    pdk.solve_batch(ref_insts, ref_tds)
    refs = [i.solution() for i in ref_insts]
    # FP64, one instance at a time, on the first `sample_alone` instances
    alone_cells, t_alone = 0, 0.0
    for k, (inst, d, td) in enumerate(zip(ref_insts[:sample_alone], datas, tds)):
        inst.set_solution(pdk.ring_vector(d["u0_origin"], d["u0_grid"]), 0.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        inst.solve(td)
        torch.cuda.synchronize()
        t_alone += time.perf_counter() - t0
        alone_cells += inst.N
    for i in ref_insts:
        i.close()
    insts = make(pdk.PD_MIXED)
    u0s = [pdk.ring_vector(d["u0_origin"], d["u0_grid"]) for d in datas]
    tuned = autotune.tune(insts, tds, levels=TUNE_LEVELS, sync=torch.cuda.synchronize)
    for inst, u0 in zip(insts, u0s):
        inst.set_solution(u0, 0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = pdk.solve_batch(insts, tds)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    errs = [float(np.linalg.norm(i.solution() - r) / np.linalg.norm(r)) for i, r in zip(insts, refs)]
    for i in insts:
        i.close()
    return {
        "workload": ("512 instances, m log-uniform [32,512], n log-uniform [64,1024], half parabolic / "
                     "half drift-diffusion, theta U[0.5,1], dt=5e-4 fixed, 100 levels"),
        "cells": cells,
        "mixed_batched": {"value": round(cells * c["K"] / el, 1), "ms": round(1e3 * el, 1),
                          "schedule": list(tuned["best"]), "autotune_ms_first_levels": tuned["ms"],
                          "l2_rel_vs_fp64_converged_max": max(errs),
                          "inner_iters_per_level_mean": round(float(np.mean(
                              [np.mean([s["iters"] for s in x]) for x in st])), 2)},
        "fp64_one_instance_at_a_time": {"value": round(alone_cells * c["K"] / t_alone, 1),
                                        "sample": f"first {sample_alone} instances"},
    }


def adaptive_variant(pdk, stream, tol, tol_time=1e-6):
    """The benchmark batch advanced to T with a-posteriori step control
    (dt in [1e-5, 1e-3], first step 1e-5, local error tolerance tol_time),
    FP64: steps taken, wall time, and the error against a converged FP64
    solve of the same (logged) time levels."""
    import torch
    insts, tds, u0s = build_instances(pdk, pdk.PD_FP64, stream)
    cells = [i.N for i in insts]
    descs = [pdk.adaptive_time_desc(th, T_END, 1e-5, tol_time, 1e-5, 1e-3, tol=tol) for th, _ in tds]
    # schedule: adaptive steps take few iterations, and a level can only
    # start at a round head, so the round length is chosen on whole solves
    # (the first of each pair warms the plans and graphs up)
    groups = pdk.get_schedule()["groups"]
    tried = {}
    for cpg in ADAPTIVE_CPG:
        pdk.set_schedule(groups, cpg)
        for rep in range(2):
            reset(insts, u0s)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pdk.solve_batch(insts, descs)
            torch.cuda.synchronize()
        tried[cpg] = time.perf_counter() - t0
    best = min(tried, key=tried.get)
    pdk.set_schedule(groups, best)
    reset(insts, u0s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sts = pdk.solve_batch(insts, descs)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    steps = [pdk.taken(st) for st in sts]
    xs = [i.solution() for i in insts]
    # converged FP64 replay of each instance's own levels
    errs = []
    for inst, u0, (th, _), st, x in zip(insts, u0s, tds, steps, xs):
        inst.set_solution(u0, 0.0)
        lv = [0.0] + [s["t"] for s in st]
        # an adaptive Crank-Nicolson solve takes its first two steps with backward Euler
        k0 = 2 if th == 0.5 else 0
        if k0:
            inst.solve(pdk.time_desc(1.0, k0, table=lv[:k0 + 1], tol=1e-13))
        inst.solve(pdk.time_desc(th, len(st) - k0, table=lv[k0:], tol=1e-13))
        r = inst.solution()
        errs.append(float(np.linalg.norm(x - r) / np.linalg.norm(r)))
    for i in insts:
        i.close()
    upd = sum(c * len(st) for c, st in zip(cells, steps))
    return {"workload": "benchmark batch, adaptive dt in [1e-5, 1e-3] from 1e-5, local error tol "
                        f"{tol_time:g}, FP64, T=0.05",
            "schedule": [groups, best], "round_length_ms": {str(k): round(1e3 * v, 1) for k, v in tried.items()},
            "steps_per_instance": [len(st) for st in steps],
            "rejected": sum(s["rejected"] for st in steps for s in st),
            "ms": round(1e3 * el, 1), "value": round(upd / el, 1),
            "iters_per_step_mean": round(float(np.mean([s["iters"] for st in steps for s in st])), 2),
            "l2_rel_vs_fp64_converged_same_levels_max": max(errs)}


def paper_table_variant(pdk, stream):
    """Ch. 2 numerical experiment 1 as one batch of the fifteen runs of its
    error table (m = 19..99, n = floor(2 pi m); the stretch (2.4) with
    p = 1, uniform r, the stretch (2.13) with p~ = 0.6; theta = 0.6,
    dt = 0.01 to T = 0.1): wall time of the batched FP64 solve and each run's
    maximum error against the value the paper prints."""
    import torch
    from problems import paper_parabolic_ex1, sample
    from problems.manufactured import exact_at
    with open(os.path.join(ROOT, "tests", "golden", "table_2_1.json")) as f:
        rows = json.load(f)["rows"]
    pb = paper_parabolic_ex1()
    cols = [(pdk.MESH_SINE, 1.0), (pdk.MESH_UNIFORM, 1.0), (pdk.MESH_POLY, 0.6)]
    insts, tds, runs = [], [], []
    for m_s in sorted(rows, key=int):
        m = int(m_s)
        n = int(np.floor(2 * np.pi * m))
        for c, (rk, p) in enumerate(cols):
            md = pdk.mesh_desc(m, n, rk, p)
            coords = pdk.mesh_coords(md)
            insts.append(pdk.Instance(md, sample(pb, *coords), pdk.PD_FP64, stream=stream))
            tds.append(pdk.time_desc(0.6, 10, 0.1, pdk.TIME_UNIFORM, tol=1e-13))
            runs.append((m, c, coords))
    u0 = [i.solution() for i in insts]
    pdk.solve_batch(insts, tds)                       # warm-up (plans, graphs)
    for i, x in zip(insts, u0):
        i.set_solution(x, 0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pdk.solve_batch(insts, tds)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    dev = {0: 0.0, 1: 0.0, 2: 0.0}
    for inst, (m, c, coords) in zip(insts, runs):
        e0, eg = exact_at(pb, 0.1, coords[0], coords[2])
        err = float(np.max(np.abs(inst.solution() - pdk.ring_vector(e0, eg))))
        dev[c] = max(dev[c], abs(err / rows[str(m)][c] - 1))
    cells = sum(i.N for i in insts)
    for i in insts:
        i.close()
    return {"workload": "Table 2.1 runs batched: 15 instances, m 19..99, n floor(2 pi m), "
                        "theta 0.6, dt 0.01, 10 levels",
            "cells": cells, "ms": round(1e3 * el, 2), "value": round(cells * 10 / el, 1),
            "max_rel_deviation_from_printed": {"stretch_2_4": round(dev[0], 4),
                                               "uniform_r": round(dev[1], 4),
                                               "stretch_2_13": round(dev[2], 4)}}


def fig_sweeps_variant(pdk, stream):
    """The seven parameter sweeps of Figs 2.9-2.11 (Ch. 2 example 1) and
    Figs 3.5-3.8 (Ch. 3 example 1, printed stencil) at m = 19..99: all 250
    runs as one uneven FP64 batch.  Wall time of the batched solve, the
    swept value of the smallest error per figure and m, and the largest
    relative deviation of the runs' errors from the oracle's stored sweep
    table (m = 19, 39, 59)."""
    import torch
    from problems import paper_continuity_ex1, paper_continuity_ex2, paper_parabolic_ex1, sample
    from problems.manufactured import exact_at
    from problems.workloads import FIG_EXAMPLES, FIG_SWEEPS, fig_sweep_runs
    with open(os.path.join(ROOT, "tests", "golden", "fig_sweeps.json")) as f:
        golden = json.load(f)["figures"]
    by_problem = {"ch2": paper_parabolic_ex1(), "ch3": paper_continuity_ex1(), "ch3_2": paper_continuity_ex2()}
    pbs = {k: by_problem[e["problem"]] for k, e in FIG_EXAMPLES.items()}
    runs = fig_sweep_runs()
    insts, tds, coords = [], [], []
    for fig, m, n, prm in runs:
        ex = FIG_EXAMPLES[FIG_SWEEPS[fig]["example"]]
        md = pdk.mesh_desc(m, n, ex["r_kind"], prm["p"], ex["th_kind"], prm["q"])
        c = pdk.mesh_coords(md)
        flux = pdk.FLUX_LITERAL if ex["literal"] else pdk.FLUX_CENTRAL
        insts.append(pdk.Instance(md, sample(pbs[FIG_SWEEPS[fig]["example"]], *c), pdk.PD_FP64, stream=stream,
                                  flux=flux))
        tds.append(pdk.time_desc(1.0 - prm["a"], ex["K"], ex["T"],
                                 pdk.TIME_SINE if ex["t_kind"] else pdk.TIME_UNIFORM, prm["l"], tol=1e-13))
        coords.append(c)
    u0 = [i.solution() for i in insts]
    pdk.solve_batch(insts, tds)                       # warm-up (plans, graphs)
    for i, x in zip(insts, u0):
        i.set_solution(x, 0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pdk.solve_batch(insts, tds)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    best, errs, dev = {}, {}, 0.0
    for inst, (fig, m, n, prm), c in zip(insts, runs, coords):
        ex = FIG_EXAMPLES[FIG_SWEEPS[fig]["example"]]
        e0, eg = exact_at(pbs[FIG_SWEEPS[fig]["example"]], ex["T"], c[0], c[2])
        d = np.abs(inst.solution() - pdk.ring_vector(e0, eg))
        err = float(np.max(d)) if ex["error"] == "max" else float(np.mean(d[1:]))   # origin first
        errs.setdefault((fig, m), []).append(err)
        if str(m) in golden[fig]["m"]:
            k = list(FIG_SWEEPS[fig]["values"]).index(prm[FIG_SWEEPS[fig]["vary"]])
            dev = max(dev, abs(err / golden[fig]["m"][str(m)][ex["error"]][k] - 1))
    for (fig, m), e in errs.items():
        best.setdefault(fig, {})[str(m)] = FIG_SWEEPS[fig]["values"][int(np.argmin(e))]
    cell_updates = sum(i.N * FIG_EXAMPLES[FIG_SWEEPS[r[0]]["example"]]["K"] for i, r in zip(insts, runs))
    cells = sum(i.N for i in insts)
    for i in insts:
        i.close()
    return {"workload": (f"Figs 2.2, 2.5-2.7, 2.9-2.11, 3.5-3.8 and 3.12-3.15 parameter sweeps: {len(runs)} runs, "
                         "m 19..99, n floor(2 pi m), Ch. 2 example 1 (5 or 10 levels; stretch (2.4) or (2.13)) and "
                         "Ch. 3 examples 1 and 2 with the printed stencil (10 levels), theta 0.5..1"),
            "instances": len(runs), "cells": cells, "ms": round(1e3 * el, 2),
            "value": round(cell_updates / el, 1),
            "best_value_per_figure": {f: {"vary": FIG_SWEEPS[f]["vary"], "by_m": b} for f, b in best.items()},
            "paper_states": {"fig_2_2": "p~ ~ 0.6 (stretch (2.13))", "fig_2_5": "p ~ 1.1", "fig_2_6": "p ~ 1.1",
                             "fig_2_7": "a towards 0.5 (smaller dt)",
                             "fig_2_9": "p ~ 1.1", "fig_2_10": "p ~ 1.1", "fig_2_11": "a ~ 0.4 (dt 0.02)",
                             "fig_3_5": "p ~ 0.1", "fig_3_6": "q ~ 1.9", "fig_3_7": "l ~ 1.5",
                             "fig_3_8": "a ~ 0.5", "fig_3_12": "p ~ 0.5", "fig_3_13": "q ~ 5",
                             "fig_3_14": "l ~ 5", "fig_3_15": "a ~ 0.1"},
            "max_rel_error_deviation_vs_oracle_table": dev}


def gummel_variant(pdk, stream, m=256, n=512, K=20, dt=1e-3, theta=0.5):
    """The coupled two-carrier system (electrons and holes through a polar
    Poisson problem, Gummel's iteration to a relative potential change of
    1e-10 per level) on a 256 x 512 graded mesh (p = 1.3), K levels of
    Crank-Nicolson, with the line sweeps for all three fields, with the
    multigrid V-cycle for the potential only, and with it for all three:
    wall time, Gummel and Krylov iterations per level, and the largest
    difference from the line-sweep run."""
    import torch
    from problems import sample, two_carrier
    out = {"workload": (f"two carriers + polar Poisson (Gummel), {m}x{n} graded p=1.3, {K} levels of "
                        f"theta {theta}, dt {dt}, FP64"),
           "unit_note": "cell-updates/s counts the three fields per level"}
    psi_pb, n_pb, p_pb = two_carrier(3200)
    md = pdk.mesh_desc(m, n, pdk.MESH_SINE, 1.3)
    coords = pdk.mesh_coords(md)
    gd = [sample(pb, *coords) for pb in (psi_pb, n_pb, p_pb)]
    finals = {}
    L, MG = pdk.PRECOND_LINE, pdk.PRECOND_MG
    for name, kinds in (("line", (L, L, L)), ("multigrid_potential", (MG, L, L)), ("multigrid", (MG, MG, MG))):
        psi = pdk.Instance(md, gd[0], pdk.PD_FP64, stream=stream)
        car = [pdk.Instance(md, gd[k], pdk.PD_FP64, stream=stream) for k in (1, 2)]
        for inst, d, sign in zip(car, gd[1:], (-1.0, 1.0)):
            pdk.set_mobility(inst, d["D_r"], d["D_t"], sign)
        for inst, kind in zip([psi] + car, kinds):
            pdk.set_preconditioner(inst, kind)
        pdk.gummel_step(psi, car[0], car[1], 0.0, dt, theta, tol=1e-12)     # warm-up (plans, levels)
        u = [ring_u0(d) for d in gd]
        for i, x in zip([psi] + car, u):
            i.set_solution(x, 0.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sts = [pdk.gummel_step(psi, car[0], car[1], k * dt, dt, theta, tol=1e-12, gummel_tol=1e-10, max_gummel=40)
               for k in range(K)]
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        cells = 3 * (m * n + 1)
        out[name] = {"ms": round(1e3 * el, 1), "value": round(cells * K / el, 1),
                     "gummel_iters_per_level": round(float(np.mean([s["gummel_iters"] for s in sts])), 2),
                     "krylov_iters_per_level": round(float(np.mean([s["krylov_iters"] for s in sts])), 1),
                     "last_change": max(s["change"] for s in sts)}
        finals[name] = [i.solution() for i in [psi] + car]
        for i in [psi] + car:
            i.close()
    for name in ("multigrid_potential", "multigrid"):
        out[name]["max_rel_vs_line"] = max(float(np.max(np.abs(a - b)) / np.max(np.abs(a)))
                                           for a, b in zip(finals["line"], finals[name]))
    best = min(("line", "multigrid_potential", "multigrid"), key=lambda k: out[k]["ms"])
    out["best"] = best
    out["value"] = out[best]["value"]
    out["ms"] = out[best]["ms"]
    return out


def multigrid_variant(pdk, stream, sizes=((256, 512), (1024, 2048))):
    """Line sweeps against the multigrid V-cycle where iterations are many:
    the steady potential of the coupled system (a Poisson problem with the
    doping as its source, solved from zero to a scaled tolerance of 1e-10)
    and one cold continuity level of the headline problem (Crank-Nicolson,
    dt = 2.5e-4, from the initial state with no earlier levels to guess
    from, tolerance 3e-12): iterations, wall time of the solve (plans and
    levels built by an untimed first solve) and the largest difference
    between the two solutions."""
    import torch
    from problems import sample, two_carrier
    from problems.workloads import cfg3_problem
    out = {}

    def run(inst, u0, td, kind):
        pdk.set_preconditioner(inst, kind)
        inst.set_solution(u0, 0.0)
        inst.solve(td)                       # untimed: plans, graphs, multigrid levels
        inst.set_solution(u0, 0.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = inst.solve(td)
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0), sum(s["iters"] for s in st), inst.solution()

    for m, n in sizes:
        md = pdk.mesh_desc(m, n, pdk.MESH_SINE, 1.3)
        coords = pdk.mesh_coords(md)
        cases = [("poisson", sample(two_carrier(3200)[0], *coords),
                  pdk.time_desc(1.0, 1, table=[0.0, 1e30], tol=1e-10))]
        if (m, n) == (1024, 2048):
            cases.append(("cold_level", sample(cfg3_problem(), *coords),
                          pdk.time_desc(0.5, 1, 2.5e-4, pdk.TIME_UNIFORM, tol=3e-12)))
        for name, data, td in cases:
            inst = pdk.Instance(md, data, pdk.PD_FP64, stream=stream)
            u0 = ring_u0(data)
            rl = run(inst, u0, td, pdk.PRECOND_LINE)
            rm = run(inst, u0, td, pdk.PRECOND_MG)
            inst.close()
            out[f"{name}_{m}x{n}"] = {
                "line": {"ms": round(rl[0], 2), "iters": rl[1]},
                "multigrid": {"ms": round(rm[0], 2), "iters": rm[1]},
                "speedup": round(rl[0] / rm[0], 2),
                "max_rel_difference": float(np.max(np.abs(rl[2] - rm[2])) / np.max(np.abs(rl[2])))}
    return out


def ring_u0(d):
    from paper_2509_15879_amd import polardisk as pdk
    return pdk.ring_vector(d["u0_origin"], d["u0_grid"])


def serving_variant(pdk, duration=8.0, check=6):
    """The serving loop under a Poisson request stream (200 requests/s for
    `duration` seconds, mixed precision): latency percentiles, aggregate
    throughput and utilisation; `check` requests are compared with the same
    solve alone in FP64 at a tight tolerance."""
    from problems import sample
    from problems.workloads import CFG5, cfg5_arrivals, cfg5_templates
    c = CFG5
    temps = []
    for m, n, pb in cfg5_templates():
        md = pdk.mesh_desc(m, n, pdk.MESH_SINE, c["p"])
        temps.append((md, sample(pb, *pdk.mesh_coords(md)), m * n + 1))
    arr = cfg5_arrivals(duration)
    B = pdk.Batch(200 << 30, 4096)
    tickets, sub_t = [], []
    t_start = time.perf_counter()
    for (ta, k, theta, tol, K) in arr:
        now = time.perf_counter() - t_start
        if ta > now:
            time.sleep(ta - now)
        md, data, N = temps[k]
        td = pdk.time_desc(theta, K, K * c["dt"], pdk.TIME_UNIFORM, tol=tol)
        tickets.append(B.submit(md, data, td, pdk.PD_MIXED))
    results = {}
    while len(results) < len(tickets):
        for tk in tickets:
            if tk not in results:
                r = B.poll(tk)
                if r is not None:
                    results[tk] = r
        time.sleep(2e-4)
    t_end = time.perf_counter()
    info = B.stats()
    B.close()
    lat = np.array([results[tk][1]["latency_s"] for tk in tickets])
    work = sum(temps[k][2] * K for (_, k, _, _, K) in arr)
    wall = t_end - t_start
    # accuracy of a few served results against FP64 alone at a tight tolerance
    errs = {}
    for idx in np.linspace(0, len(arr) - 1, check).astype(int):
        ta, k, theta, tol, K = arr[idx]
        md, data, N = temps[k]
        inst = pdk.Instance(md, data, pdk.PD_FP64)
        inst.solve(pdk.time_desc(theta, K, K * c["dt"], pdk.TIME_UNIFORM, tol=1e-13))
        ref = inst.solution()
        inst.close()
        x = results[tickets[idx]][0]
        errs.setdefault(f"tol {tol:g}", []).append(float(np.linalg.norm(x - ref) / np.linalg.norm(ref)))
    return {
        "workload": (f"Poisson arrivals {c['rate']:g}/s for {duration:g} s, {len(arr)} requests from "
                     f"{len(temps)} templates (m log-U[32,1024], n log-U[64,2048], PDE 50/50), "
                     "theta U[0.5,1], tol 1e-6 or 1e-8, T log-U[5e-3,5e-2] at dt=1e-3, mixed precision"),
        "requests": len(arr),
        "p50_ms": round(1e3 * float(np.percentile(lat, 50)), 2),
        "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 2),
        "value": round(work / wall, 1), "unit": "cell-updates/s",
        "offered_cell_updates_per_s": round(work / duration, 1),
        "utilisation": round((work / duration) / (work / wall), 3),
        "wall_s": round(wall, 2),
        "peak_active": info["peak_active"], "plans_built": info["plans_built"],
        "worker_s": {k: round(info[k], 3) for k in ("build_s", "admit_s", "retire_s", "run_s")},
        "l2_rel_vs_fp64_alone_sample": {k: max(v) for k, v in errs.items()},
    }


def cpu_info():
    """CPU model (from /proc/cpuinfo) and os.cpu_count() of the host."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "cpu_count": os.cpu_count()}


def cpu_baseline_worker(levels, out_path):
    """The oracle on a bounded sample of the headline workload, one thread:
    mesh, sampling, assembly, one SuperLU factorisation (fixed Δt) and the
    first `levels` levels.  Writes its timings and state to out_path (npz).
    Runs in a child process started before anything touches the GPU; it
    waits for a line on stdin (sent once the timed GPU steps are over, so
    that its host work does not overlap them)."""
    from threadpoolctl import threadpool_limits
    from oracle import assemble, make_mesh
    from oracle.stepper import step
    from problems import sample
    from problems.workloads import CFG3, cfg3_problem
    c = CFG3
    sys.stdin.readline()
    with threadpool_limits(1):
        t0 = time.perf_counter()
        me = make_mesh(c["m"], c["n"], 1, c["p"])
        S = assemble(me, sample(cfg3_problem(), *me.sample_points()))
        x = S.initial()
        t_setup = time.perf_counter() - t0
        marks = []
        for k in range(levels):
            x = step(S, x, k * c["dt"], (k + 1) * c["dt"], c["theta"])
            marks.append(time.perf_counter() - t0)
    np.savez(out_path, x=x, t_setup=t_setup, marks=np.array(marks))


def start_cpu_baseline(levels):
    import subprocess
    import tempfile
    fd, path = tempfile.mkstemp(suffix=".npz", prefix="pd_oracle_")
    os.close(fd)
    proc = subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-baseline-worker",
                             str(levels), path], stdin=subprocess.PIPE, stdout=subprocess.DEVNULL,
                            stderr=subprocess.PIPE)
    return proc, path, time.perf_counter()


def release_cpu_baseline(job):
    """Lets the oracle sample start (the worker waits for this line)."""
    if job is not None:
        job[0].stdin.write(b"go\n")
        job[0].stdin.flush()


def finish_cpu_baseline(job, levels, gpu_state):
    """Waits for the oracle sample; its rate and its difference from the GPU
    state after the same levels (full vectors, paper order)."""
    proc, path, t_launch = job
    _, err = proc.communicate()
    if proc.returncode != 0:
        return {"error": err.decode(errors="replace")[-2000:]}
    from problems.workloads import CFG3
    c = CFG3
    d = np.load(path)
    os.unlink(path)
    x, t_setup, marks = d["x"], float(d["t_setup"]), d["marks"]
    N = c["m"] * c["n"] + 1
    el = float(marks[-1])
    t_fact = float(marks[0]) - t_setup                 # first level: factorisation + solve
    t_level = (el - float(marks[0])) / max(1, levels - 1)
    full = t_setup + t_fact + (c["K"] - 1) * t_level
    out = {
        "value": N * levels / el, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
        "sample": (f"the headline workload's first {levels} of {c['K']} levels on one thread: mesh, "
                   f"sampling, assembly ({t_setup:.1f} s), one SuperLU factorisation with the first "
                   f"level ({t_fact:.1f} s), then {t_level:.1f} s per level (LU solve + one refinement "
                   f"step); {el:.1f} s in all, run in a child process beside the GPU legs that "
                   f"follow the timed headline steps"),
        "full_run_estimate_cell_updates_per_s": N * c["K"] / full,
        "full_run_estimate_s": round(full, 1),
        **cpu_info(),
    }
    if gpu_state is not None:
        out["gpu_vs_oracle_same_levels"] = {
            "max_rel": float(np.max(np.abs(gpu_state - x)) / np.max(np.abs(x))),
            "l2_rel": float(np.linalg.norm(gpu_state - x) / np.linalg.norm(x)),
            "levels": levels}
    return out


def oracle_samples():
    """The oracle's stored trajectory of the headline workload (levels 20
    and 200, sampled; written by tests/golden/make_cfg3_reference.py)."""
    path = os.path.join(ROOT, "tests", "golden", "cfg3_oracle_samples.npz")
    return np.load(path)


def vs_oracle_samples(x_paper, ref, level):
    """Max-rel (normwise, by the full state's max norm) and L2-rel over the
    stored samples of the oracle's state at `level`."""
    idx = ref["indices"]
    xr = ref[f"x_{level}"]
    d = x_paper[idx] - xr
    return {"max_rel": float(np.max(np.abs(d)) / float(ref[f"maxabs_{level}"])),
            "l2_rel_samples": float(np.linalg.norm(d) / np.linalg.norm(xr)),
            "samples": int(len(idx))}


def cfg3_instance(pdk, prec, stream):
    from problems import sample
    from problems.workloads import CFG3, cfg3_problem
    c = CFG3
    md = pdk.mesh_desc(c["m"], c["n"], pdk.MESH_SINE, c["p"])
    data = sample(cfg3_problem(), *pdk.mesh_coords(md))
    inst = pdk.Instance(md, data, prec, stream=stream)
    return inst, pdk.ring_vector(data["u0_origin"], data["u0_grid"])


def cfg3_desc(pdk, tol, K=None):
    from problems.workloads import CFG3
    c = CFG3
    K = c["K"] if K is None else K
    return pdk.time_desc(c["theta"], K, c["dt"] * K, pdk.TIME_UNIFORM, tol=tol, max_seconds=120.0)


def roofline_of(pdk, run_step, w, cells_iters, traffic_table, instance_iters=None, stencil_rings=None,
                repeats=2):
    """Event-stamped extra steps: per-family launch times; the dominant
    kernel's algorithmic bytes per launch over its average launch time.
    Of `repeats` such steps the one with the least total cycle-kernel time
    is kept (a step that something else on the machine slowed down would
    otherwise stand for the kernels).  instance_iters (one instance): the
    share of the p-sweep launches that found the instance iterating (the
    rest wait for the next round head).  The counter-measured traffic
    applies only to the sources it was taken on, and a stencil's only to
    the tile depth it was taken at."""
    best = None
    for _ in range(max(1, repeats)):
        pdk.kernel_timing(True, reset=True)
        t0 = time.perf_counter()
        run_step()
        ms = 1e3 * (time.perf_counter() - t0)
        km, kc = pdk.kernel_timing(False, reset=True)
        tot = sum(km[f] for f in KERNEL_NAMES)
        if best is None or tot < best[0]:
            best = (tot, ms, km, kc)
    _, prof_ms, kms, kcnt = best
    fam_bytes = {f: cells_iters * bytes_per_cell(f, w) for f in KERNEL_NAMES}
    dom = max(fam_bytes, key=lambda f: kms[f])
    achieved = fam_bytes[dom] / (kms[dom] / 1e3) / 1e9
    traffic = None
    if (traffic_table is not None and kernel_source_sha1() == traffic_table["sha1"]
            and (not dom.startswith("sten") or stencil_rings == traffic_table["stencil_rings"])):
        traffic = round(traffic_table["b_per_cell"][dom] * cells_iters / max(1, kcnt[dom]))
    return {
        "bound": "hbm", "kernel": KERNEL_NAMES[dom], "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "launches": int(kcnt[dom]), "avg_launch_us": round(1e3 * kms[dom] / max(1, kcnt[dom]), 2),
        "bytes_per_launch": round(fam_bytes[dom] / max(1, kcnt[dom])),
        "kernel_gbs": {f: round(fam_bytes[f] / (kms[f] / 1e3) / 1e9, 1) for f in fam_bytes if kms[f] > 0},
        "kernel_avg_us": {f: round(1e3 * kms[f] / kcnt[f], 2) for f in kms if kcnt[f] > 0},
        "kernel_launches": {f: int(kcnt[f]) for f in kms if kcnt[f] > 0},
        "kernel_ms": {k: round(v, 2) for k, v in kms.items()},
        "profiled_step_ms": round(prof_ms, 1),
        "measured_on": (f"the faster of {max(1, repeats)} extra steps (total cycle-kernel time), each launch "
                        "stamped by its own start/stop events"),
        **({"active_launch_fraction": round(instance_iters / max(1, kcnt["rad_p"]), 4)}
           if instance_iters is not None else {}),
    }


def batch_variant(pdk, stream, tol):
    """The ten-instance 256 x 512 batch (five seeds x θ in {0.5, 1}, 100
    sine-stretched levels): FP64 batched, FP64 one instance at a time and
    mixed batched, each against a converged FP64 solve."""
    import torch
    from paper_2509_15879_amd import autotune
    insts, tds, u0s = build_instances(pdk, pdk.PD_FP64, stream)
    cells = sum(i.N for i in insts)
    reset(insts, u0s)
    pdk.solve_batch(insts, time_descs(pdk, tds, 1e-13))
    refs = [i.solution() for i in insts]
    descs = time_descs(pdk, tds, tol)
    out = {"workload": ("continuity drift-diffusion, 256x512 graded (p=1.3), 100 sine-stretched levels to "
                        "T=0.05, 5 seeds x theta {0.5,1} = 10 instances"), "tol_per_step": tol}

    def timed(instances, ds):
        reset(instances, u0s)
        pdk.solve_batch(instances, ds)
        reset(instances, u0s)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = pdk.solve_batch(instances, ds)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, st

    reset(insts, u0s)
    tuned = autotune.tune(insts, descs, levels=K_LEVELS, repeats=1, sync=torch.cuda.synchronize)
    el, st = timed(insts, descs)
    errs = [float(np.linalg.norm(i.solution() - r) / np.linalg.norm(r)) for i, r in zip(insts, refs)]
    out["fp64_batched"] = {"value": round(cells * K_LEVELS / el, 1), "ms": round(1e3 * el, 1),
                           "schedule": list(tuned["best"]), "l2_rel_vs_fp64_converged_max": max(errs),
                           "iters_per_level": round(float(np.mean([sum(s["iters"] for s in x) for x in st]))
                                                    / K_LEVELS, 2)}
    t_alone = 0.0
    for inst, u0, d in zip(insts, u0s, descs):
        inst.set_solution(u0, 0.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        inst.solve(d)
        torch.cuda.synchronize()
        t_alone += time.perf_counter() - t0
    out["fp64_one_instance_at_a_time"] = {"value": round(cells * K_LEVELS / t_alone, 1),
                                          "ms": round(1e3 * t_alone, 1)}
    mix, _, _ = build_instances(pdk, pdk.PD_MIXED, stream)
    reset(mix, u0s)
    mtuned = autotune.tune(mix, descs, levels=K_LEVELS, repeats=1, sync=torch.cuda.synchronize)
    el, mst = timed(mix, descs)
    me = max(float(np.linalg.norm(i.solution() - r) / np.linalg.norm(r)) for i, r in zip(mix, refs))
    out["mixed_batched"] = {"value": round(cells * K_LEVELS / el, 1), "ms": round(1e3 * el, 1),
                            "schedule": list(mtuned["best"]), "l2_rel_vs_fp64_converged_max": me,
                            "inner_iters_per_level": round(float(np.mean(
                                [sum(s["iters"] for s in x) for x in mst])) / K_LEVELS, 2),
                            "refinements_per_level": round(float(np.mean(
                                [sum(s["refinements"] for s in x) for x in mst])) / K_LEVELS, 2)}
    for i in insts + mix:
        i.close()
    return out


def arg_parser():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--tol", type=float, default=3e-12,
                    help="per-step scaled-residual tolerance of the headline solve")
    ap.add_argument("--oracle-levels", type=int, default=2)
    ap.add_argument("--serving-seconds", type=float, default=60.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--schedule", default=None,
                    help="groups,cycles_per_graph,stencil_rings: use this schedule instead of tuning "
                         "(e.g. to profile the schedule an un-profiled run chose)")
    ap.add_argument("--cpu-baseline-worker", nargs=2, default=None, help=argparse.SUPPRESS)
    return ap


def main():
    args = arg_parser().parse_args()
    if args.cpu_baseline_worker:
        cpu_baseline_worker(int(args.cpu_baseline_worker[0]), args.cpu_baseline_worker[1])
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: --gpus {args.gpus} is not supported "
              "(instances are independent; a multi-GPU run would shard them by footprint)",
              file=sys.stderr)
        sys.exit(2)

    # the oracle's sample runs in a child process beside the GPU legs after
    # the timed steps; it is started before anything touches the GPU
    job = None if args.no_cpu_baseline else start_cpu_baseline(args.oracle_levels)

    import torch
    from paper_2509_15879_amd import autotune
    from paper_2509_15879_amd import polardisk as pdk
    from problems.workloads import CFG3
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream
    c = CFG3
    cells = c["m"] * c["n"] + 1

    log("headline: 1024x2048 instance ...")
    inst, u0 = cfg3_instance(pdk, pdk.PD_FP64, stream)
    desc = cfg3_desc(pdk, args.tol)

    def run_step():
        inst.set_solution(u0, 0.0)
        return inst.solve(desc)

    inst.set_solution(u0, 0.0)
    if args.schedule:
        fixed = tuple(int(v) for v in args.schedule.split(","))
        pdk.set_schedule(*fixed)
        tuned = {"best": fixed, "ms": {}}
    else:
        tuned = autotune.tune([inst], [desc], levels=c["K"], candidates=SINGLE_CANDIDATES, repeats=1,
                              sync=torch.cuda.synchronize)
    log(f"schedule {tuned['best']} from {tuned['ms']}")
    for w in range(args.warmup):
        run_step()
    torch.cuda.synchronize()
    lat, stats = [], None
    for s in range(args.steps):
        inst.set_solution(u0, 0.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats = inst.solve(desc)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
        log(f"step {s}: {lat[-1] * 1e3:.1f} ms")
    release_cpu_baseline(job)
    ms_per_step = 1e3 * float(np.mean(lat))
    value = cells * c["K"] / (ms_per_step / 1e3)
    x = inst.solution(pdk.LAYOUT_PAPER)
    iters = sum(s["iters"] for s in stats)

    # accuracy: the oracle's stored trajectory (sampled) and a converged GPU FP64 solve
    ref = oracle_samples()
    acc = vs_oracle_samples(x, ref, c["K"])
    conv_inst, _ = cfg3_instance(pdk, pdk.PD_FP64, stream)
    conv_inst.solve(cfg3_desc(pdk, 1e-13))
    xc = conv_inst.solution(pdk.LAYOUT_PAPER)
    conv_inst.close()
    acc["l2_rel_vs_gpu_fp64_tol_1e-13"] = float(np.linalg.norm(x - xc) / np.linalg.norm(xc))
    acc["valid"] = acc["l2_rel_samples"] <= 1e-8
    acc["bar"] = "L2-relative <= 1e-8 against the FP64 oracle (levels 200, stored samples)"

    # roofline of the dominant kernel on one more, event-stamped step
    roof = roofline_of(pdk, run_step, 8, cells * iters, TRAFFIC.get("cfg3_fp64"), instance_iters=iters,
                        stencil_rings=tuned["best"][2])
    # the GPU state after the oracle sample's levels, for the live comparison
    early = None
    if job is not None:
        inst.set_solution(u0, 0.0)
        inst.solve(cfg3_desc(pdk, args.tol, K=args.oracle_levels))
        early = inst.solution(pdk.LAYOUT_PAPER)
    inst.close()

    out = {
        "metric": "cell-updates/s (cells×steps/s) at 1e-8 rel err vs FP64; p50/p99 solve latency",
        "value": round(value, 1), "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded manufactured continuity problem)",
        "config": {
            "workload": ("continuity drift-diffusion on a 1024x2048 polar mesh graded towards r=0 and r=1 "
                         "(radial stretch (2.4), p=1.3; 2,097,153 unknowns), seed 1300, theta=0.5 "
                         "(Crank-Nicolson), fixed dt=2.5e-4, 200 levels to T=0.05"),
            "m": c["m"], "n": c["n"], "unknowns": cells, "levels": c["K"], "tol_per_step": args.tol,
            "precision": "fp64", "parallelism": "single GPU, one instance",
            "schedule": {"groups": tuned["best"][0], "cycles_per_graph": tuned["best"][1],
                         "stencil_rings": tuned["best"][2], "autotune_ms_whole_solves": tuned["ms"]},
        },
        "p50_ms": round(1e3 * float(np.percentile(lat, 50)), 3),
        "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 3),
        "accuracy": acc,
        "iters_per_level_mean": round(iters / c["K"], 2),
        "roofline": roof,
    }

    if not args.no_variants:
        var = {}
        log("mixed precision, same workload ...")
        var["mixed_1024x2048"] = mixed_cfg3_variant(pdk, stream, args.tol, ref)
        log("ten-instance 256x512 batch ...")
        var["batch_10x256x512"] = batch_variant(pdk, stream, 4e-12)
        log("adaptive time steps ...")
        var["adaptive_dt"] = adaptive_variant(pdk, stream, 4e-12)
        log("Table 2.1 runs batched ...")
        var["paper_table_2_1"] = paper_table_variant(pdk, stream)
        log("figure sweeps (250 runs) ...")
        var["fig_sweeps"] = fig_sweeps_variant(pdk, stream)
        log("two carriers with Gummel coupling ...")
        var["gummel_2carrier"] = gummel_variant(pdk, stream)
        log("multigrid against the line sweeps ...")
        var["multigrid"] = multigrid_variant(pdk, stream)
        log("uneven batch of 512 ...")
        var["uneven_512"] = uneven_variant(pdk, stream, 4e-12)
        log(f"serving stream ({args.serving_seconds:g} s) ...")
        var["serving"] = serving_variant(pdk, duration=args.serving_seconds)
        out["variants"] = var

    if job is not None:
        log("oracle sample ...")
        out["cpu_baseline"] = finish_cpu_baseline(job, args.oracle_levels, early)

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
