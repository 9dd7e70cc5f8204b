"""Seeded workloads: which problems, meshes and time schedules make up a
measured run.  Only parameters and problem objects live here; meshes,
discretisation and solves belong to the solvers."""

from .manufactured import continuity_cfg

# 256 x 512 graded continuity problems (radial stretch p = 1.3), 100
# sine-stretched levels (l = 1.5) to T = 0.05, five coefficient seeds, each
# with θ = 0.5 and θ = 1: ten instances advanced together.
CFG2 = dict(m=256, n=512, p=1.3, T=0.05, K=100, l=1.5)
CFG2_SEEDS = (1200, 1201, 1202, 1203, 1204)
CFG2_THETAS = (0.5, 1.0)


def cfg2_batch():
    """[(seed, theta, Problem)] of the ten-instance continuity workload."""
    c = CFG2
    return [(s, th, continuity_cfg(s, c["m"], c["n"], th, c["p"], c["T"], c["K"], c["l"]))
            for s in CFG2_SEEDS for th in CFG2_THETAS]
