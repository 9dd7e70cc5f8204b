"""Host logic of bench.py that its measurement relies on (no GPU)."""

import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

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
    assert set(bench.TRAFFIC_B_PER_CELL) == set(bench.KERNEL_NAMES)
    for fam, b in bench.TRAFFIC_B_PER_CELL.items():
        # measured bytes are at least the algorithmic ones, and not wildly above
        alg = bench.bytes_per_cell(fam, 8)
        assert alg <= b <= 1.25 * alg, (fam, b, alg)


def test_algorithmic_bytes_of_one_iteration():
    # FP64: two radial sweeps, two ring sweeps, two stencils and the update
    fams = ["rad_p", "ang_p", "sten_v", "rad_s", "ang_s", "sten_t", "update"]
    assert sum(bench.bytes_per_cell(f, 8) for f in fams) == 336
    # FP32 inner iteration (the stencils also read their FP32 1/diag copy)
    assert sum(bench.bytes_per_cell(f, 4) for f in fams) == 204
