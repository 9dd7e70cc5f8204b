"""Writes cfg3_oracle_samples.npz: the FP64 oracle's trajectory of the
1024 x 2048 graded continuity problem (seed 1300, θ = 0.5, fixed
Δt = 2.5e-4, 200 levels to T = 0.05), sampled.

The oracle assembles the face-flux operator of §3.2 and solves each level's
system (2.11)/(2.12) with one SuperLU factorisation (fixed Δt) plus one
refinement step per solve.  Storing the whole state (16.8 MB per level) is
not sensible, so the file keeps, at levels 20 and 200:

* the origin, four whole rings (1, 2, 512 and m) and two whole radial lines
  (j = 0 and j = n/2), which cover the origin closure, the graded inner and
  outer rings and the periodic seam;
* 16384 further unknowns drawn with default_rng(1300) (without replacement);
* the full state's max norm and 2-norm, which normalise the parity metrics.

Indices are in the paper's unknown order (2.12): the origin first, then
radial line j = 0..n-1 listing rings i = 1..m (index 1 + j*m + i - 1).

Only the oracle and the problem generator run here.  About 15 minutes and
7 GB of memory on one core.

    python tests/golden/make_cfg3_reference.py
"""

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "cfg3_oracle_samples.npz")
KEEP_LEVELS = (20, 200)
RANDOM_SAMPLES = 16384


def sample_indices(m, n, seed):
    """Sorted unique paper-order indices of the stored unknowns."""
    def ring(i):
        return 1 + np.arange(n) * m + (i - 1)

    def line(j):
        return 1 + j * m + np.arange(m)

    fixed = np.concatenate([[0], ring(1), ring(2), ring(m // 2), ring(m), line(0), line(n // 2)])
    rng = np.random.default_rng(seed)
    rand = rng.choice(m * n + 1, size=RANDOM_SAMPLES, replace=False)
    return np.unique(np.concatenate([fixed, rand])).astype(np.int64)


def main():
    from threadpoolctl import threadpool_limits
    from oracle import assemble, make_mesh
    from oracle.stepper import step
    from problems import sample
    from problems.workloads import CFG3, cfg3_problem

    c = CFG3
    m, n, K, dt, theta = c["m"], c["n"], c["K"], c["dt"], c["theta"]
    idx = sample_indices(m, n, c["seed"])
    t0 = time.perf_counter()
    with threadpool_limits(1):
        me = make_mesh(m, n, 1, c["p"])
        S = assemble(me, sample(cfg3_problem(), *me.sample_points()))
        print(f"assembled {S.N} unknowns in {time.perf_counter() - t0:.1f} s", flush=True)
        x = S.initial()
        out = {"indices": idx, "levels": np.array(KEEP_LEVELS, np.int64)}
        for k in range(K):
            x = step(S, x, k * dt, (k + 1) * dt, theta)
            if k == 0:
                print(f"level 1 (factorisation + solve) at {time.perf_counter() - t0:.1f} s", flush=True)
            if (k + 1) in KEEP_LEVELS:
                out[f"x_{k + 1}"] = x[idx]
                out[f"maxabs_{k + 1}"] = np.array(np.max(np.abs(x)))
                out[f"norm2_{k + 1}"] = np.array(np.linalg.norm(x))
                print(f"level {k + 1} kept at {time.perf_counter() - t0:.1f} s", flush=True)
    np.savez_compressed(OUT, **out)
    print(f"wrote {OUT} ({len(idx)} samples) in {time.perf_counter() - t0:.1f} s", flush=True)


if __name__ == "__main__":
    main()
