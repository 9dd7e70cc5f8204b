"""Seeded synthetic problems for the polar-disk θ-scheme solver.

This package defines *problems*, not the method: PDE coefficients, sources,
boundary and initial data, and exact (manufactured) solutions, as plain
functions of (t, r, θ).  It holds no mesh construction, no discretisation
and no solver arithmetic.  Both the oracle and the GPU path ask it for values
at sample points that each of them computes on its own.
"""

from .manufactured import (  # noqa: F401
    Problem,
    TimeMode,
    sample,
    parabolic_cfg1,
    parabolic_family,
    continuity_cfg,
    closed_form_quadratic,
    paper_parabolic_ex1,
    paper_continuity_ex1,
    paper_continuity_ex2,
    random_positive,
    zero_flux_random,
    two_carrier,
)
