"""FP64 CPU oracle for the polar-disk θ-scheme (test infrastructure only).

This package is the slow, plain reference that the GPU library is checked
against.  Only the tests, the smoke check and the CPU-baseline leg of the
benchmark may import it; the library never does, and the two share no code.

What it computes (Ch. 2 §2.1 and Ch. 3 §3.1-§3.2 of the paper):

* the polar mesh with the radial stretch (2.4), the angular stretch and the
  time stretch of §3.1, and the comparison stretch (2.13);
* the discrete spatial operator L_h as a sparse FP64 matrix, either in the
  conservative face-flux form (default) or verbatim from the printed
  stencils (the ℘_h operator of §2.1, the ϖ_h operator of §3.2.1 and the
  origin closure of §3.2.2);
* the θ-weighted scheme (2.5)/(2.11): every step solves
  (I/Δt + θ L_h) n^{k+1} = (I/Δt - (1-θ) L_h) n^k + sources + boundary terms
  with a sparse direct LU (SciPy SuperLU), θ = 1 - a.

The GPU library's own solver parts are stated plainly beside them: the
alternating-line preconditioner (precond.py), the θ-semi-coarsening multigrid
built on it (multigrid.py; the paper's §4.2 names multigrid-type
preconditioners for large grids), the a-posteriori step control
(timectl.py), the error indicator (adapt.py) and the coupled two-carrier
system (gummel.py).

Unknowns are kept in the paper's ordering (2.12): the origin first, then
radial line j = 0..n-1, each listing rings i = 1..m.

Parity pins: every function is pinned by tests against closed forms,
invariants, brute force or printed values; none is "parity unpinned".
"""

from .mesh import Mesh, make_mesh, time_levels  # noqa: F401
from .operator import assemble, assemble_literal, OracleSystem  # noqa: F401
from .stepper import solve, step  # noqa: F401
