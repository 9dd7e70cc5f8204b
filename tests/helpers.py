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


class DeviceBuffer:
    """Device memory from the HIP runtime the library itself is linked
    against (already loaded in this process), filled from a host array."""

    def __init__(self, hip, arr):
        import ctypes as C
        self.hip = hip
        self.a = np.ascontiguousarray(arr)
        self.p = C.c_void_p()
        assert hip.hipMalloc(C.byref(self.p), max(self.a.nbytes, 8)) == 0
        assert hip.hipMemcpy(self.p, self.a.ctypes.data, self.a.nbytes, 1) == 0   # host to device

    def read(self):
        out = np.empty_like(self.a)
        assert self.hip.hipMemcpy(out.ctypes.data, self.p, out.nbytes, 2) == 0   # device to host
        return out

    def free(self):
        if self.p:
            assert self.hip.hipFree(self.p) == 0
            self.p = None


def hip_runtime():
    """The HIP runtime the loaded library resolved (by its soname, so the copy
    already in the process is the one returned)."""
    import ctypes as C
    from paper_2509_15879_amd import polardisk  # noqa: F401  (loads the library first)
    hip = C.CDLL("libamdhip64.so.7")
    hip.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
    hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    hip.hipFree.argtypes = [C.c_void_p]
    return hip


def fig_problem(example):
    from problems import paper_continuity_ex1, paper_continuity_ex2, paper_parabolic_ex1
    from problems.workloads import FIG_EXAMPLES
    make = {"ch2": paper_parabolic_ex1, "ch3": paper_continuity_ex1, "ch3_2": paper_continuity_ex2}
    return make[FIG_EXAMPLES[example]["problem"]]()


def fig_errors(x, pb, T, r_nodes, th_nodes):
    """(mean over the ring unknowns, max over all unknowns) of |x - exact| at
    T; x in the paper's unknown order (2.12)."""
    from oracle.operator import to_vec
    from problems.manufactured import exact_at
    e0, eg = exact_at(pb, T, r_nodes, th_nodes)
    d = np.abs(x - to_vec(e0, eg))
    return float(np.mean(d[1:])), float(np.max(d))


def oracle_fig_run(fig, m, n, prm):
    """One run of a figure's sweep with the oracle: its state at T (paper
    order) and its errors (mean, max)."""
    from problems.workloads import FIG_EXAMPLES, FIG_SWEEPS
    ex = FIG_EXAMPLES[FIG_SWEEPS[fig]["example"]]
    pb = fig_problem(FIG_SWEEPS[fig]["example"])
    me = make_mesh(m, n, ex["r_kind"], prm["p"], ex["th_kind"], prm["q"])
    data = sample(pb, *me.sample_points())
    S = assemble_literal(me, data) if ex["literal"] else assemble(me, data)
    x = solve(S, time_levels(ex["T"], ex["K"], ex["t_kind"], prm["l"]), 1.0 - prm["a"])
    return x, fig_errors(x, pb, ex["T"], me.r, me.th)
