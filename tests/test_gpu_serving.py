"""Serving loop (continuous batching): requests of different mesh sizes, PDE
types and precisions submitted while others are running are admitted at
time-level boundaries, share launches, and give exactly the result each
gives alone; admission respects the slot count and the memory pool."""

import time

import numpy as np
import pytest

from helpers import max_rel, oracle_system
from oracle import solve as oracle_solve
from problems import continuity_cfg, parabolic_family, sample

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


# (problem, mesh (m, n, r_kind, p), flux, theta, K, precision); one mesh has
# m > 256, so both radial-sweep classes run in the same launches
SPECS = [
    (lambda: continuity_cfg(2101, 48, 96), (48, 96, 1, 1.3), 0, 0.5, 24, 0),
    (lambda: parabolic_family(1.0, 0.5), (33, 64, 0, 1.0), 0, 1.0, 20, 0),
    (lambda: continuity_cfg(2102, 300, 64), (300, 64, 1, 1.3), 1, 0.7, 16, 0),
    (lambda: continuity_cfg(2103, 40, 130), (40, 130, 1, 1.3), 0, 1.0, 8, 1),
    (lambda: parabolic_family(0.7, 0.3, 0.4), (20, 70, 0, 1.0), 0, 0.5, 12, 1),
    (lambda: continuity_cfg(2104, 64, 64), (64, 64, 1, 1.3), 1, 0.6, 7, 0),
]


def request(spec):
    from paper_2509_15879_amd import polardisk as pdk
    mk, (m, n, rk, p), flux, theta, K, prec = spec
    md = pdk.mesh_desc(m, n, rk, p)
    data = sample(mk(), *pdk.mesh_coords(md))
    td = pdk.time_desc(theta, K, 0.02, pdk.TIME_SINE, 1.5, tol=1e-12)
    return md, data, td, flux, prec


def alone(spec):
    from paper_2509_15879_amd import polardisk as pdk
    md, data, td, flux, prec = request(spec)
    inst = pdk.Instance(md, data, prec, flux=flux)
    inst.solve(td)
    x = inst.solution()
    inst.close()
    return x


def submit(B, spec, req=None):
    md, data, td, flux, prec = req or request(spec)
    return B.submit(md, data, td, prec, flux=flux)


def test_requests_joining_a_running_batch_match_alone():
    say("[serve] 3 requests, then 3 more while they run; results vs alone")
    from paper_2509_15879_amd import polardisk as pdk
    reqs = [request(s) for s in SPECS]             # inputs sampled before any submit
    B = pdk.Batch(8 << 30, 16)
    first = [submit(B, s, r) for s, r in zip(SPECS[:3], reqs[:3])]
    t_end = time.monotonic() + 60
    while B.stats()["slices_run"] < 2:
        assert time.monotonic() < t_end, "the loop did not start"
        time.sleep(1e-4)
    later = [submit(B, s, r) for s, r in zip(SPECS[3:], reqs[3:])]
    got = [B.wait(t) for t in first + later]
    info = B.stats()
    B.close()
    say(f"  loop: {info}")
    assert info["completed"] == len(SPECS) and info["pending"] == 0 and info["active"] == 0
    assert info["peak_active"] >= 4            # the late requests overlapped the early ones
    assert info["plans_built"] >= 2
    for spec, (x, sm) in zip(SPECS, got):
        ref = alone(spec)
        assert sm["status"] == 0 and sm["levels"] == spec[4]
        assert abs(sm["t"] - 0.02) < 1e-15
        assert sm["latency_s"] >= sm["queue_s"] >= 0.0
        assert np.array_equal(x, ref), max_rel(x, ref)


def test_admission_respects_pool_and_slots():
    say("[serve] pool for two requests, five submitted")
    from paper_2509_15879_amd import polardisk as pdk
    specs = [SPECS[0]] * 4 + [SPECS[5]]          # equal footprints, then a smaller one
    fps = []
    for s in specs:
        md, data, td, flux, prec = request(s)
        fps.append(pdk.footprint(md, len(data["lam"]), prec) + (9 * max(td.K, 16) + 1) * 8)
    pool = max(fps) * 2 + max(fps) // 2          # at most two requests fit at once
    B = pdk.Batch(pool, 8)
    tickets = [submit(B, s) for s in specs]
    got = [B.wait(t) for t in tickets]
    info = B.stats()
    B.close()
    say(f"  loop: {info}")
    assert info["peak_bytes"] <= pool and info["peak_active"] <= 2
    assert info["completed"] == len(specs)
    for s, (x, sm) in zip(specs, got):
        assert sm["status"] == 0
        assert np.array_equal(x, alone(s))
    B1 = pdk.Batch(1 << 34, 1)                    # one slot: strictly one after another
    tickets = [submit(B1, s) for s in specs[:3]]
    res = [B1.wait(t) for t in tickets]
    info1 = B1.stats()
    B1.close()
    assert info1["peak_active"] == 1 and all(sm["status"] == 0 for _, sm in res)


def test_served_result_matches_oracle():
    say("[serve] one continuity request vs the oracle")
    from paper_2509_15879_amd import polardisk as pdk
    pb = continuity_cfg(2105, 24, 40)
    md = pdk.mesh_desc(24, 40, 1, 1.3)
    data = sample(pb, *pdk.mesh_coords(md))
    td = pdk.time_desc(0.5, 6, 0.01, pdk.TIME_SINE, 1.5, tol=1e-13)
    B = pdk.Batch(1 << 30, 4)
    x, sm = B.wait(B.submit(md, data, td, pdk.PD_FP64, flux=0))
    B.close()
    S, me = oracle_system(pb, 24, 40, 1, 1.3)
    ref = oracle_solve(S, pdk.time_levels(td), 0.5)
    got = np.asarray(x)
    from oracle.operator import to_vec
    assert sm["status"] == 0
    assert max_rel(to_vec(got[0], got[1:].reshape(24, 40)), ref) <= 1e-10


def test_serving_errors():
    say("[serve] error paths")
    from paper_2509_15879_amd import polardisk as pdk
    B = pdk.Batch(1 << 20, 2)                      # 1 MiB: too small for the large mesh
    md, data, td, flux, prec = request(SPECS[2])
    with pytest.raises(pdk.PolarDiskError, match="pool"):
        B.submit(md, data, td, prec)
    md, data, td, flux, prec = request(SPECS[1])
    bad = pdk.time_desc(1.5, 4, 0.01)
    with pytest.raises(pdk.PolarDiskError, match="theta"):
        B.submit(md, data, bad, prec)
    with pytest.raises(pdk.PolarDiskError, match="ticket"):
        pdk._check(pdk.lib.pd_batch_poll(B.h, 12345, None, None))
    B.close()
