"""Host logic of bench.py that its measurement relies on (no GPU)."""

import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import bench  # noqa: E402

SRC = """// header comment
#include <x.h>
/* a block
   comment */
__global__ void k(double *a) {   // trailing
  a[0] = 1.0;

}
"""


def test_digest_ignores_comments_and_blank_lines():
    edited = SRC.replace("// header comment", "// another header").replace("a block", "other words")
    edited = edited.replace("   // trailing", "") + "\n\n"
    assert bench.code_digest([SRC]) == bench.code_digest([edited])


def test_digest_sees_every_code_change():
    assert bench.code_digest([SRC]) != bench.code_digest([SRC.replace("1.0", "2.0")])
    assert bench.code_digest([SRC]) != bench.code_digest([SRC.replace("a[0]", "a[1]")])
    # file order matters (the kernels, then the host runtime)
    assert bench.code_digest([SRC, "int x;"]) != bench.code_digest(["int x;", SRC])


def test_traffic_table_covers_every_cycle_kernel():
    for name, tab in bench.TRAFFIC.items():
        if tab is None:
            continue
        assert set(tab["b_per_cell"]) == set(bench.KERNEL_NAMES), name
        assert len(tab["sha1"]) == 40
        for fam, b in tab["b_per_cell"].items():
            # measured bytes are at least the algorithmic ones, and not wildly above
            alg = bench.bytes_per_cell(fam, tab["w"])
            assert alg <= b <= 1.25 * alg, (name, fam, b, alg)


def test_oracle_samples_fixture_covers_the_headline():
    ref = bench.oracle_samples()
    idx = ref["indices"]
    m, n = 1024, 2048
    assert idx[0] == 0 and idx[-1] <= m * n and len(set(idx.tolist())) == len(idx)
    assert list(ref["levels"]) == [20, 200]
    for lv in (20, 200):
        x = ref[f"x_{lv}"]
        assert x.shape == idx.shape and np.all(np.isfinite(x))
        assert float(ref[f"maxabs_{lv}"]) >= np.max(np.abs(x))
    # the stored samples are the discrete solution, so they lie within the
    # discretisation error of the manufactured exact solution (measured
    # 1.5e-6 at level 20, 6.4e-6 at level 200); a level or index mix-up
    # would not (level 20 against the exact solution at level 200: 4.6e-2)
    from oracle import make_mesh
    from problems.manufactured import exact_at
    from problems.workloads import CFG3, cfg3_problem
    me = make_mesh(m, n, 1, CFG3["p"])
    i, j = (idx[1:] - 1) % m, (idx[1:] - 1) // m
    for lv, other in ((20, 200), (200, 20)):
        e0, eg = exact_at(cfg3_problem(), lv * CFG3["dt"], me.r, me.th)
        ex = np.concatenate([[e0], eg[i, j]])
        scale = np.max(np.abs(ex))
        assert np.max(np.abs(ref[f"x_{lv}"] - ex)) <= 1e-4 * scale
        assert np.max(np.abs(ref[f"x_{other}"] - ex)) >= 1e-2 * scale
    # a state equal to the samples scores zero
    full = np.zeros(m * n + 1)
    full[idx] = ref["x_200"]
    d = bench.vs_oracle_samples(full, ref, 200)
    assert d["max_rel"] == 0.0 and d["l2_rel_samples"] == 0.0


def test_cpu_info_names_the_host():
    info = bench.cpu_info()
    assert info["cpu_count"] == os.cpu_count()


def test_algorithmic_bytes_of_one_iteration():
    # FP64: two radial sweeps, two ring sweeps, two stencils and the update
    fams = ["rad_p", "ang_p", "sten_v", "rad_s", "ang_s", "sten_t", "update"]
    assert sum(bench.bytes_per_cell(f, 8) for f in fams) == 336
    # FP32 inner iteration (the stencils also read their FP32 1/diag copy)
    assert sum(bench.bytes_per_cell(f, 4) for f in fams) == 204


class _FakeTiming:
    """Stands in for the binding's kernel timing: each extra step reports
    the per-family times given, in turn."""

    FAMS = ("begin", "factor", "rad_p", "ang_p", "sten_v", "rad_s", "ang_s", "sten_t", "update",
            "refine", "control", "level_end", "multigrid")

    def __init__(self, runs):
        self.runs = list(runs)
        self.k = -1

    def kernel_timing(self, enable, reset=False):
        if enable:
            self.k += 1
            return {}, {}
        ms = {f: self.runs[self.k].get(f, 0.0) for f in self.FAMS}
        cnt = {f: (100 if ms[f] > 0 else 0) for f in self.FAMS}
        return ms, cnt


def test_roofline_keeps_the_faster_extra_step():
    fast = {f: 1.0 for f in bench.KERNEL_NAMES}
    fast["rad_p"] = 2.0
    slow = dict(fast, rad_p=3.0)
    for runs in ([slow, fast], [fast, slow]):
        fake = _FakeTiming(runs)
        r = bench.roofline_of(fake, lambda: None, 8, 1000000, None, repeats=2)
        assert r["kernel"] == bench.KERNEL_NAMES["rad_p"]
        assert r["kernel_ms"]["rad_p"] == 2.0
        # 52 B per unknown over 2 ms
        assert abs(r["achieved"] - 52e6 / 2e-3 / 1e9) < 0.1
        assert r["traffic"] is None
