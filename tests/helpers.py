"""Shared set-up for tests: the same seeded problem handed to the oracle
(sampled at the oracle's own mesh) and to the GPU library (sampled at the
library's mesh)."""

import numpy as np

from oracle import assemble, assemble_literal, make_mesh, solve, time_levels  # noqa: F401
from problems import sample


def oracle_system(pb, m, n, r_kind=0, p=1.0, th_kind=0, q=1.0, flux=0, bc=0):
    me = make_mesh(m, n, r_kind, p, th_kind, q)
    return assemble(me, sample(pb, *me.sample_points()), flux=flux, bc=bc), me


def gpu_instance(pb, m, n, r_kind=0, p=1.0, th_kind=0, q=1.0, precision=0, flux=0, bc=0):
    from paper_2509_15879_amd import polardisk as pdk
    md = pdk.mesh_desc(m, n, r_kind, p, th_kind, q)
    data = sample(pb, *pdk.mesh_coords(md))
    return pdk.Instance(md, data, precision, flux=flux, bc=bc)


def max_rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def l2_rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
