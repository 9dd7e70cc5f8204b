"""Seeded workloads: which problems, meshes and time schedules make up a
measured run.  Only parameters and problem objects live here; meshes,
discretisation and solves belong to the solvers."""

import numpy as np

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


# 1024 x 2048 graded continuity problem (2,097,153 unknowns), θ = 0.5, fixed
# Δt = 2.5e-4, 200 levels: the precision comparison (FP64 against FP32 inner
# iterations with FP64 refinement).
CFG3 = dict(m=1024, n=2048, p=1.3, theta=0.5, dt=2.5e-4, K=200, seed=1300)


def cfg3_problem():
    c = CFG3
    return continuity_cfg(c["seed"], c["m"], c["n"], c["theta"], c["p"], c["dt"] * c["K"], c["K"], 1.0, 0)


# 512 independent instances of uneven size, a parameter-sensitivity sweep:
# m log-uniform in [32, 512], n log-uniform in [64, 1024]; even indices are
# parabolic (seeded decay rate λ in [0.5, 2], tilt β in [0, 0.9] and phase),
# odd ones drift-diffusion (seeded coefficients); θ uniform in [0.5, 1]; the
# radial stretch (2.4) with p = 1.3; fixed Δt = 5e-4, 100 levels.
CFG4 = dict(count=512, m=(32, 512), n=(64, 1024), p=1.3, dt=5e-4, K=100, seed=1400)


def cfg4_batch(count=None):
    """[(index, m, n, theta, Problem)] of the uneven batch (the first `count`)."""
    from .manufactured import parabolic_family
    c = CFG4
    rng = np.random.default_rng(c["seed"])
    out = []
    for q in range(c["count"] if count is None else count):
        m = int(round(np.exp(rng.uniform(np.log(c["m"][0]), np.log(c["m"][1])))))
        n = int(round(np.exp(rng.uniform(np.log(c["n"][0]), np.log(c["n"][1])))))
        theta = float(rng.uniform(0.5, 1.0))
        if q % 2 == 0:
            pb = parabolic_family(float(rng.uniform(0.5, 2.0)), float(rng.uniform(0.0, 0.9)),
                                  float(rng.uniform(0.0, 2 * np.pi)), name=f"cfg4_{q}")
        else:
            pb = continuity_cfg(c["seed"] + q, m, n, theta, c["p"], c["dt"] * c["K"], c["K"], 1.0, 0,
                                name=f"cfg4_{q}")
        out.append((q, m, n, theta, pb))
    return out
