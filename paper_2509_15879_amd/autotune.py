"""Autotuner of the launch schedule of a batch.

A batch's best schedule (how many stream groups it is split into, how many
Krylov cycles one captured graph holds) and stencil tile (rings per wave)
depend on its instance sizes, precisions and convergence behaviour.  `tune` times the first levels of the
batch's own solve under every candidate schedule, starting each time from
the batch's current state (saved and restored, so tuning leaves no trace),
then sets the fastest as the library's default and returns the table.
Results are cached per batch signature (instance sizes and precisions).
"""

from __future__ import annotations

import time
from typing import Dict, List, Sequence, Tuple

from . import polardisk as pdk

# (stream groups, cycles per graph).  Longer rounds pay for their idle
# cycles (an instance that converges waits for the next round head) by
# running the round head, which costs about one cycle, less often; 6 and 7
# fit warm levels of about six iterations.  4 and 5 groups ran the
# ten-instance 256 x 512 batch 45-53% slower than 3, and more hardware
# queues per process made them slower still: from the fourth stream on the
# groups stop overlapping (same iterations, same results).
DEFAULT_CANDIDATES: Tuple[Tuple[int, int], ...] = tuple((g, c) for g in (1, 2, 3) for c in (4, 6, 7, 8, 12))
STENCIL_RINGS: Tuple[int, ...] = (4, 8)

_cache: Dict[tuple, dict] = {}


def signature(insts: Sequence["pdk.Instance"]) -> tuple:
    return tuple(sorted((i.m, i.n, int(i.precision)) for i in insts))


def _first_levels(td: "pdk.TimeDesc", t0: float, levels: int) -> "pdk.TimeDesc":
    t = pdk.time_levels(td, t0)[:levels + 1]
    return pdk.time_desc(td.theta, len(t) - 1, table=t, tol=td.tol, max_iters=td.max_iters)


def tune(insts: Sequence["pdk.Instance"], tds: Sequence["pdk.TimeDesc"], levels: int = 3,
         candidates: Sequence[Tuple[int, int]] = DEFAULT_CANDIDATES, repeats: int = 2,
         sync=None, use_cache: bool = True) -> dict:
    """Chooses and sets the fastest schedule for advancing `insts` through
    `tds`; returns {"best": (groups, cycles_per_graph, stencil_rings),
    "ms": {...}}.  Every candidate is timed under both stencil depths.

    sync: callable that waits for the device (e.g. torch.cuda.synchronize);
    the library's own calls already return after the work is done."""
    key = signature(insts)
    if use_cache and key in _cache:
        best = _cache[key]["best"]
        pdk.set_schedule(*best)
        return _cache[key]
    saved = [(i.solution(), i.time) for i in insts]
    short = [_first_levels(td, t, levels) for td, (_, t) in zip(tds, saved)]
    full = [(g, c, r) for g, c in candidates for r in STENCIL_RINGS]
    ms: Dict[Tuple[int, int, int], float] = {}
    try:
        for cand in full:
            pdk.set_schedule(*cand)
            best_t = float("inf")
            for rep in range(repeats + 1):                # first run warms the plan up
                for inst, (x, t) in zip(insts, saved):
                    inst.set_solution(x, t)
                if sync:
                    sync()
                t0 = time.perf_counter()
                pdk.solve_batch(insts, short)
                if sync:
                    sync()
                if rep:
                    best_t = min(best_t, time.perf_counter() - t0)
            ms[cand] = 1e3 * best_t
    finally:
        for inst, (x, t) in zip(insts, saved):
            inst.set_solution(x, t)
    best = min(ms, key=ms.get)
    pdk.set_schedule(*best)
    out = {"best": best, "ms": {f"{g}x{c}x{r}": round(v, 3) for (g, c, r), v in ms.items()},
           "levels": levels}
    _cache[key] = out
    return out


def tuned_schedules() -> List[dict]:
    return [dict(signature=k, **v) for k, v in _cache.items()]
