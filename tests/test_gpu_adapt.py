"""GPU error indicator and state transfer against the oracle's, and an
adaptive run (solve, choose a stretch, transfer, solve on) replayed by the
oracle with the GPU's logged choice."""

import numpy as np
import pytest

from helpers import gpu_instance, max_rel, oracle_system
from oracle import solve as oracle_solve
from oracle import time_levels
from oracle.adapt import choose_stretch, indicator, transfer
from oracle.operator import from_vec, to_vec
from problems import continuity_cfg, zero_flux_random

pytestmark = pytest.mark.gpu

CANDS = [0.6, 0.8, 1.0, 1.3, 1.6, 2.0]


def say(*a):
    print(*a, flush=True)


def advanced(pb, m, n, rk, p, K, theta=0.5, bc=0, tk=0, q=1.0):
    """GPU instance after K sine-stretched levels to T = 0.01, and the oracle system."""
    from paper_2509_15879_amd import polardisk as pdk
    inst = gpu_instance(pb, m, n, rk, p, tk, q, bc=bc)
    t = time_levels(0.01, 12, 1, 1.5)
    inst.solve(pdk.time_desc(theta, K, table=t[:K + 1], tol=1e-14))
    S, me = oracle_system(pb, m, n, rk, p, tk, q, bc=bc)
    return inst, S, me, t


@pytest.mark.parametrize("bc", [0, 1])
def test_indicator_matches_oracle(bc):
    say(f"[adapt] indicator vs oracle, bc={bc}")
    from paper_2509_15879_amd import polardisk as pdk
    pb = continuity_cfg(3101, 40, 64) if bc == 0 else zero_flux_random(3102)
    inst, S, me, t = advanced(pb, 40, 64, 1, 1.0, 5, bc=bc)
    res = pdk.error_indicator(inst, 1.0, CANDS, want_eta=True)
    x = inst.solution(pdk.LAYOUT_PAPER)
    nb = S.boundary(t[5]) if bc == 0 else None
    eta, kappa = indicator(me, x, nb)
    scale = eta.max()
    say(f"  eta_max {res['eta_max']:.3e}, p_best {res['p_best']}, recommend {res['recommend']}")
    assert np.max(np.abs(res["eta"] - eta)) <= 1e-10 * scale
    assert np.max(np.abs(res["kappa"] - kappa)) <= 1e-10 * kappa.max()
    assert abs(res["eta_max"] - scale) <= 1e-10 * scale
    assert abs(res["eta_sum"] - eta.sum()) <= 1e-10 * eta.sum()
    p_best, pb_, pc, rec = choose_stretch(me, kappa, 1.0, CANDS)
    assert res["p_best"] == p_best and bool(res["recommend"]) == rec
    assert abs(res["pred_best"] - pb_) <= 1e-10 * pb_ and abs(res["pred_current"] - pc) <= 1e-10 * pc
    inst.close()


@pytest.mark.parametrize("bc", [0, 1])
def test_transfer_matches_oracle(bc):
    say(f"[adapt] transfer vs oracle, bc={bc}")
    from paper_2509_15879_amd import polardisk as pdk
    pb = continuity_cfg(3103, 30, 48) if bc == 0 else zero_flux_random(3104)
    src, S, me, t = advanced(pb, 30, 48, 1, 1.0, 4, bc=bc)
    dst = gpu_instance(pb, 37, 52, 1, 1.6, 1, 1.2, bc=bc)      # other radii and angles
    pdk.remesh_transfer(src, dst)
    got = dst.solution(pdk.LAYOUT_PAPER)
    x = src.solution(pdk.LAYOUT_PAPER)
    _, me2 = oracle_system(pb, 37, 52, 1, 1.6, 1, 1.2, bc=bc)
    ref = transfer(me, x, me2, S.boundary(t[4]) if bc == 0 else None)
    say(f"  max-rel {max_rel(got, ref):.2e}")
    assert max_rel(got, ref) <= 1e-12
    src.close()
    dst.close()


def test_adaptive_run_replayed_by_oracle():
    """Layer at the origin: 4 levels on p = 1, the GPU's choice of stretch,
    transfer, 6 more levels; the oracle replays the same decision."""
    say("[adapt] adaptive run vs oracle replay")
    from paper_2509_15879_amd import polardisk as pdk
    pb = continuity_cfg(3105, 32, 48)
    src, S, me, t = advanced(pb, 32, 48, 1, 1.0, 4)
    res = pdk.error_indicator(src, 1.0, CANDS)
    p_new = res["p_best"] if res["p_best"] != 1.0 else 1.3        # always exercise a transfer
    say(f"  decision: p_best {res['p_best']} (recommend {res['recommend']}), remesh to {p_new}")
    dst = gpu_instance(pb, 32, 48, 1, p_new)
    pdk.remesh_transfer(src, dst)
    dst.solve(pdk.time_desc(0.5, 6, table=t[4:11], tol=1e-14))
    got = dst.solution(pdk.LAYOUT_PAPER)
    # oracle: its own first levels, its own transfer, then the new system
    x4 = oracle_solve(S, t[:5], 0.5)
    S2, me2 = oracle_system(pb, 32, 48, 1, p_new)
    y = transfer(me, x4, me2, S.boundary(t[4]))
    ref = oracle_solve(S2, t[4:11], 0.5, x0=y)
    say(f"  max-rel {max_rel(got, ref):.2e}")
    assert max_rel(got, ref) <= 1e-10
    src.close()
    dst.close()
