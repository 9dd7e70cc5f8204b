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


# Request stream of the serving loop: Poisson arrivals (rate per second) for
# a bounded duration; each request draws a template (mesh m log-uniform in
# [32, 1024], n in [64, 2048], PDE alternating), its own θ in [0.5, 1],
# tolerance 1e-6 or 1e-8, and end time T log-uniform in [5e-3, 5e-2] at a
# fixed Δt = 1e-3 (5 to 50 levels).
CFG5 = dict(rate=200.0, m=(32, 1024), n=(64, 2048), dt=1e-3, T=(5e-3, 5e-2), tols=(1e-6, 1e-8),
            p=1.3, templates=24, seed=1500)


def cfg5_templates(count=None):
    """[(m, n, Problem)] request templates."""
    from .manufactured import parabolic_family
    c = CFG5
    rng = np.random.default_rng(c["seed"])
    out = []
    for k in range(c["templates"] if count is None else count):
        m = int(round(np.exp(rng.uniform(np.log(c["m"][0]), np.log(c["m"][1])))))
        n = int(round(np.exp(rng.uniform(np.log(c["n"][0]), np.log(c["n"][1])))))
        if k % 2 == 0:
            pb = parabolic_family(float(rng.uniform(0.5, 2.0)), float(rng.uniform(0.0, 0.9)),
                                  float(rng.uniform(0.0, 2 * np.pi)), name=f"cfg5_{k}")
        else:
            pb = continuity_cfg(c["seed"] + k, m, n, 0.5, c["p"], name=f"cfg5_{k}")
        out.append((m, n, pb))
    return out


def cfg5_arrivals(duration, rate=None, seed=None):
    """[(arrival time s, template index, θ, tol, K)] of a Poisson stream."""
    c = CFG5
    rng = np.random.default_rng(c["seed"] + 1 if seed is None else seed)
    rate = c["rate"] if rate is None else rate
    t, out = 0.0, []
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= duration:
            return out
        k = int(rng.integers(0, c["templates"]))
        theta = float(rng.uniform(0.5, 1.0))
        tol = float(c["tols"][int(rng.integers(0, 2))])
        T = float(np.exp(rng.uniform(np.log(c["T"][0]), np.log(c["T"][1]))))
        out.append((t, k, theta, tol, max(1, int(round(T / c["dt"])))))


# Parameter sweeps of the paper's figures, each run of a sweep one instance
# of an uneven batch; m = 19..99 rings with n = floor(2 pi m) (h = 1/(m+1)).
#  Ch. 2 example 1 (Figs 2.9-2.11): stretch (2.4) in r, uniform θ, the
#  θ-scheme with a = 1 - θ, Δt = 0.02 to T = 0.1 (five uniform levels);
#  the maximum error over all unknowns at T.
#  Ch. 3 example 1 (Figs 3.5-3.8): the printed stencil, stretch (2.4) in r
#  with p and the angular stretch with q, ten levels of the time stretch
#  with l to T = 0.1; the mean error over the ring unknowns at T.
# `vary` names the swept parameter, `fixed` the others (p, q, l, a).
FIG_SWEEP_M = (19, 39, 59, 79, 99)
_P2 = (0.6, 0.8, 0.9, 1.0, 1.1, 1.2, 1.3, 1.5, 1.8)
FIG_SWEEPS = {
    # Ch. 2: Fig 2.2 sweeps the parameter p~ of the stretch (2.13) (a = 0.4,
    # Δt = 0.01, as Table 2.1); Figs 2.5-2.7 (their captions lost the
    # parameters) are read as the Δt = 0.01 counterparts of Figs 2.9-2.11
    "fig_2_2": dict(example="ch2_ex1_213", vary="p", values=(0.2, 0.4, 0.5, 0.6, 0.7, 0.8, 1.0),
                    fixed=dict(q=1.0, l=1.0, a=0.4)),
    "fig_2_5": dict(example="ch2_ex1_dt01", vary="p", values=_P2, fixed=dict(q=1.0, l=1.0, a=0.4)),
    "fig_2_6": dict(example="ch2_ex1_dt01", vary="p", values=_P2, fixed=dict(q=1.0, l=1.0, a=0.5)),
    "fig_2_7": dict(example="ch2_ex1_dt01", vary="a", values=(0.0, 0.1, 0.2, 0.3, 0.4, 0.45, 0.5),
                    fixed=dict(p=1.1, q=1.0, l=1.0)),
    "fig_2_9": dict(example="ch2_ex1", vary="p", values=_P2, fixed=dict(q=1.0, l=1.0, a=0.4)),
    "fig_2_10": dict(example="ch2_ex1", vary="p", values=_P2, fixed=dict(q=1.0, l=1.0, a=0.5)),
    "fig_2_11": dict(example="ch2_ex1", vary="a", values=(0.0, 0.1, 0.2, 0.3, 0.4, 0.45, 0.5),
                     fixed=dict(p=1.1, q=1.0, l=1.0)),
    "fig_3_5": dict(example="ch3_ex1", vary="p", values=(0.05, 0.1, 0.2, 0.4, 0.7, 1.0, 1.3),
                    fixed=dict(q=1.0, l=1.0, a=0.5)),
    "fig_3_6": dict(example="ch3_ex1", vary="q", values=(1.0, 1.3, 1.6, 1.9, 2.2, 2.5),
                    fixed=dict(p=0.1, l=1.0, a=0.5)),
    "fig_3_7": dict(example="ch3_ex1", vary="l", values=(1.0, 1.25, 1.5, 1.75, 2.0, 2.5),
                    fixed=dict(p=0.1, q=1.9, a=0.5)),
    "fig_3_8": dict(example="ch3_ex1", vary="a", values=(0.0, 0.1, 0.2, 0.3, 0.4, 0.5),
                    fixed=dict(p=0.1, q=1.9, l=1.5)),
    # Ch. 3, numerical experiment 2 (§3.4), printed stencil; the text's
    # fixed parameters per figure
    "fig_3_12": dict(example="ch3_ex2", vary="p", values=(0.1, 0.2, 0.3, 0.5, 0.7, 1.0, 1.3),
                     fixed=dict(q=1.0, l=1.0, a=0.5)),
    "fig_3_13": dict(example="ch3_ex2", vary="q", values=(1.0, 2.0, 3.0, 4.0, 5.0),
                     fixed=dict(p=0.5, l=1.0, a=0.5)),
    "fig_3_14": dict(example="ch3_ex2", vary="l", values=(1.0, 2.0, 3.0, 4.0, 5.0, 6.0),
                     fixed=dict(p=0.5, q=5.0, a=0.5)),
    "fig_3_15": dict(example="ch3_ex2", vary="a", values=(0.0, 0.1, 0.2, 0.3, 0.4, 0.5),
                     fixed=dict(p=0.5, q=5.0, l=5.0)),
}
FIG_EXAMPLES = {
    # problem (the paper's numerical experiment 1 of Ch. 2, 1 or 2 of Ch. 3),
    # radial kind (1: the stretch (2.4) with p; 3: the stretch (2.13) with
    # p~), angular kind (1: stretched with q), time kind (1: stretched with
    # l), levels, T
    "ch2_ex1": dict(problem="ch2", r_kind=1, th_kind=0, t_kind=0, K=5, T=0.1, error="max", literal=False),
    "ch2_ex1_dt01": dict(problem="ch2", r_kind=1, th_kind=0, t_kind=0, K=10, T=0.1, error="max", literal=False),
    "ch2_ex1_213": dict(problem="ch2", r_kind=3, th_kind=0, t_kind=0, K=10, T=0.1, error="max", literal=False),
    "ch3_ex1": dict(problem="ch3", r_kind=1, th_kind=1, t_kind=1, K=10, T=0.1, error="mean", literal=True),
    "ch3_ex2": dict(problem="ch3_2", r_kind=1, th_kind=1, t_kind=1, K=10, T=0.1, error="mean", literal=True),
}


def fig_sweep_runs(ms=FIG_SWEEP_M, figs=None):
    """[(figure, m, n, params)] of the sweeps: every (figure, m, swept value),
    params = dict(p, q, l, a) with the swept one set."""
    runs = []
    for fig, s in FIG_SWEEPS.items():
        if figs is not None and fig not in figs:
            continue
        for m in ms:
            n = int(np.floor(2 * np.pi * m))
            for v in s["values"]:
                prm = dict(s["fixed"])
                prm[s["vary"]] = v
                runs.append((fig, m, n, prm))
    return runs
