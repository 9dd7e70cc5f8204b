"""A short run of a benchmark workload for hardware-counter profiling.

    python -m paper_2509_15879_amd.profile_workload [--workload W] [--levels L] [--copy-mib M]

Advances the workload (cfg3: the 1024 x 2048 continuity instance of the
headline; cfg2: the ten 256 x 512 continuity instances; poisson: the steady
potential of the coupled system on the 1024 x 2048 mesh, one level from
zero) through its first L time levels with plain kernel launches (no captured graphs, so every
dispatch is counted on its own), then copies an M MiB device buffer, filled
and then pushed out of the caches, once with torch: a kernel that reads and
writes exactly M MiB, against which the profiler's byte counters are
calibrated.  Under rocprofv3 --pmc each pass takes seconds.
"""

import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def arg_parser():
    ap = argparse.ArgumentParser()
    ap.add_argument("--levels", type=int, default=2)
    ap.add_argument("--copy-mib", type=int, default=256)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--workload", choices=["cfg3", "cfg2", "poisson"], default="cfg3")
    ap.add_argument("--precond", choices=["line", "mg"], default="line")
    ap.add_argument("--tol", type=float, default=None)
    ap.add_argument("--schedule", default=None,
                    help="groups,cycles_per_graph,stencil_rings of the run (e.g. the one bench.py tuned)")
    return ap


def main():
    args = arg_parser().parse_args()
    os.environ["PD_NO_GRAPH"] = "1"

    import torch
    from problems import sample
    from problems.workloads import CFG2, CFG3, cfg2_batch, cfg3_problem
    from paper_2509_15879_amd import polardisk as pdk

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream
    if args.schedule:
        pdk.set_schedule(*(int(v) for v in args.schedule.split(",")))
    prec = pdk.PD_MIXED if args.precision == "mixed" else pdk.PD_FP64
    insts, descs = [], []
    if args.workload == "poisson":
        from problems import two_carrier
        c = CFG3
        tol = args.tol or 1e-10
        md = pdk.mesh_desc(c["m"], c["n"], pdk.MESH_SINE, c["p"])
        insts.append(pdk.Instance(md, sample(two_carrier(3200)[0], *pdk.mesh_coords(md)), pdk.PD_FP64,
                                  stream=stream))
        descs.append(pdk.time_desc(1.0, 1, table=[0.0, 1e30], tol=tol))
    elif args.workload == "cfg2":
        c = CFG2
        tol = args.tol or 4e-12
        for seed, th, pb in cfg2_batch():
            md = pdk.mesh_desc(c["m"], c["n"], pdk.MESH_SINE, c["p"])
            insts.append(pdk.Instance(md, sample(pb, *pdk.mesh_coords(md)), prec, stream=stream))
            descs.append(pdk.time_desc(th, c["K"], c["T"], pdk.TIME_SINE, c["l"], tol=tol))
    else:
        c = CFG3
        tol = args.tol or 3e-12
        md = pdk.mesh_desc(c["m"], c["n"], pdk.MESH_SINE, c["p"])
        insts.append(pdk.Instance(md, sample(cfg3_problem(), *pdk.mesh_coords(md)), prec, stream=stream))
        descs.append(pdk.time_desc(c["theta"], c["K"], c["dt"] * c["K"], pdk.TIME_UNIFORM, tol=tol))
    for i in insts:
        pdk.set_preconditioner(i, pdk.PRECOND_MG if args.precond == "mg" else pdk.PRECOND_LINE)
    print(f"[profile] {args.workload}: {len(insts)} instances, {args.levels} levels, {args.precond}", flush=True)
    if args.workload != "poisson":
        t = pdk.time_levels(descs[0])[:args.levels + 1]
        descs = [pdk.time_desc(d.theta, args.levels, table=t, tol=tol) for d in descs]
    stats = pdk.solve_batch(insts, descs)
    torch.cuda.synchronize()
    print("[profile] iterations per level:", [[s["iters"] for s in st] for st in stats], flush=True)
    # calibration: fill a source, push it out of every cache by filling a
    # buffer four times the size, then copy it once
    n = args.copy_mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    evict = torch.full((4 * n,), 2.0, dtype=torch.float32, device="cuda")
    del evict
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(f"[profile] copied {args.copy_mib} MiB (last dispatch)", flush=True)
    for i in insts:
        i.close()


if __name__ == "__main__":
    main()
