"""ctypes binding of libpolardisk (include/polardisk.h).

Argument marshalling only: every step of the solver runs in the HIP kernels
of the shared library.  The library must have been built
(``python -m paper_2509_15879_amd.build``); importing this module fails
loudly otherwise.
"""

from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpolardisk.so")

PD_OK, PD_PENDING = 0, 1
ERRORS = {-1: "PD_EINVAL", -2: "PD_ENOMEM", -3: "PD_EBREAKDOWN", -4: "PD_ENOCONV",
          -5: "PD_EHIP", -6: "PD_EBUSY"}
PD_FP64, PD_MIXED = 0, 1
MESH_UNIFORM, MESH_SINE, MESH_EXPLICIT, MESH_POLY = 0, 1, 2, 3
LAYOUT_RING, LAYOUT_PAPER = 0, 1
PRECOND_LINE, PRECOND_MG = 0, 1
FLUX_CENTRAL, FLUX_UPWIND, FLUX_LITERAL = 0, 1, 2
TIME_UNIFORM, TIME_SINE, TIME_TABLE, TIME_ADAPTIVE = 0, 1, 2, 3


class PolarDiskError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class MeshDesc(C.Structure):
    _fields_ = [("nr", C.c_int32), ("ntheta", C.c_int32), ("r_kind", C.c_int32), ("p", C.c_double),
                ("th_kind", C.c_int32), ("q", C.c_double), ("r_explicit", C.c_void_p),
                ("th_explicit", C.c_void_p)]


class ProblemDesc(C.Structure):
    _fields_ = [("pde", C.c_int32), ("flux", C.c_int32), ("bc", C.c_int32), ("layout", C.c_int32),
                ("device_ptrs", C.c_int32), ("b_node", C.c_void_p), ("D_rface", C.c_void_p),
                ("Er_rface", C.c_void_p), ("D_tface", C.c_void_p), ("Et_tface", C.c_void_p),
                ("nsrc", C.c_int32), ("lam", C.c_void_p), ("tpow", C.c_void_p), ("g", C.c_void_p),
                ("nb", C.c_void_p), ("u0", C.c_void_p), ("E_node", C.c_void_p), ("D_origin", C.c_double)]


class TimeDesc(C.Structure):
    _fields_ = [("t_kind", C.c_int32), ("K", C.c_int32), ("T", C.c_double), ("l", C.c_double),
                ("t_table", C.c_void_p), ("theta", C.c_double), ("tol", C.c_double),
                ("max_iters", C.c_int32), ("dt0", C.c_double), ("dt_min", C.c_double),
                ("dt_max", C.c_double), ("tol_time", C.c_double), ("max_seconds", C.c_double)]


class StepStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("refinements", C.c_int32), ("status", C.c_int32),
                ("reserved", C.c_int32), ("rel_resid", C.c_double), ("dt", C.c_double),
                ("t", C.c_double), ("err_time", C.c_double), ("rejected", C.c_int32),
                ("pad", C.c_int32)]

    def as_dict(self):
        return {"iters": self.iters, "refinements": self.refinements, "status": self.status,
                "restarts": self.reserved, "rel_resid": self.rel_resid, "dt": self.dt, "t": self.t,
                "err_time": self.err_time, "rejected": self.rejected}


class RequestSummary(C.Structure):
    _fields_ = [("status", C.c_int32), ("levels", C.c_int32), ("iters", C.c_int32),
                ("refinements", C.c_int32), ("max_rel_resid", C.c_double), ("t", C.c_double),
                ("queue_s", C.c_double), ("latency_s", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class BatchInfo(C.Structure):
    _fields_ = [("pending", C.c_int32), ("active", C.c_int32), ("peak_active", C.c_int32),
                ("reserved", C.c_int32), ("submitted", C.c_uint64), ("completed", C.c_uint64),
                ("slices_run", C.c_uint64), ("plans_built", C.c_uint64), ("used_bytes", C.c_size_t),
                ("peak_bytes", C.c_size_t), ("build_s", C.c_double), ("admit_s", C.c_double),
                ("retire_s", C.c_double), ("run_s", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class GummelStats(C.Structure):
    _fields_ = [("gummel_iters", C.c_int32), ("krylov_iters", C.c_int32), ("change", C.c_double)]


class Indicator(C.Structure):
    _fields_ = [("eta_max", C.c_double), ("eta_sum", C.c_double), ("i_max", C.c_int32),
                ("j_max", C.c_int32), ("p_best", C.c_double), ("pred_best", C.c_double),
                ("pred_current", C.c_double), ("recommend", C.c_int32), ("reserved", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


# every entry point declared in include/polardisk.h
EXPORTS = ("pd_mesh_coords", "pd_time_levels", "pd_mesh_create", "pd_scheme_step", "pd_solve_to_T", "pd_solve_batch",
           "pd_get_solution", "pd_set_solution", "pd_apply_operator", "pd_assemble_rhs",
           "pd_apply_preconditioner", "pd_set_preconditioner", "pd_set_mobility", "pd_gummel_step",
           "pd_footprint", "pd_destroy", "pd_batch_create", "pd_batch_submit", "pd_batch_poll",
           "pd_batch_stats", "pd_error_indicator", "pd_error_indicator_noalloc", "pd_remesh_transfer", "pd_set_schedule",
           "pd_get_schedule", "pd_get_time",
           "pd_batch_destroy", "pd_kernel_timing", "pd_last_error")

KERNEL_FAMILIES = ("begin", "factor", "rad_p", "ang_p", "sten_v", "rad_s", "ang_s", "sten_t",
                   "update", "refine", "control", "level_end", "multigrid")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: the HIP library has not been built "
                          "(python -m paper_2509_15879_amd.build)")
    # One HIP runtime per process: torch's is loaded first, so that the
    # library binds to it and shares its device, streams and memory (loaded
    # the other way round, a second runtime comes in beside torch's and
    # finds no device).
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    P, I32, D, U64, SZ = C.c_void_p, C.c_int32, C.c_double, C.c_uint64, C.c_size_t
    sig = {
        "pd_mesh_coords": [C.POINTER(MeshDesc), P, P, P, P],
        "pd_time_levels": [C.POINTER(TimeDesc), D, P],
        "pd_mesh_create": [C.POINTER(MeshDesc), C.POINTER(ProblemDesc), I32, P, C.POINTER(P)],
        "pd_scheme_step": [P, D, D, D, D, C.POINTER(StepStats)],
        "pd_solve_to_T": [P, C.POINTER(TimeDesc), P],
        "pd_solve_batch": [C.POINTER(P), I32, C.POINTER(TimeDesc), P],
        "pd_get_solution": [P, P, I32, I32],
        "pd_set_solution": [P, P, I32, I32, D],
        "pd_apply_operator": [P, D, D, P, P, I32, I32, I32],
        "pd_assemble_rhs": [P, D, D, D, P, I32, I32],
        "pd_apply_preconditioner": [P, D, D, P, P, I32, I32],
        "pd_set_mobility": [P, P, P, D, I32],
        "pd_set_preconditioner": [P, I32],
        "pd_gummel_step": [P, P, P, D, D, D, D, D, I32, C.POINTER(GummelStats)],
        "pd_footprint": [C.POINTER(MeshDesc), I32, I32, C.POINTER(SZ)],
        "pd_destroy": [P],
        "pd_batch_create": [SZ, I32, P, C.POINTER(P)],
        "pd_batch_submit": [P, C.POINTER(MeshDesc), C.POINTER(ProblemDesc), C.POINTER(TimeDesc), I32,
                            C.POINTER(U64)],
        "pd_batch_poll": [P, U64, P, C.POINTER(RequestSummary)],
        "pd_batch_stats": [P, C.POINTER(BatchInfo)],
        "pd_error_indicator": [P, D, P, I32, P, P, C.POINTER(Indicator)],
        "pd_error_indicator_noalloc": [P, D, P, I32, P, P, C.POINTER(Indicator)],
        "pd_remesh_transfer": [P, P],
        "pd_set_schedule": [P],
        "pd_get_time": [P, P],
        "pd_get_schedule": [P],
        "pd_batch_destroy": [P],
        "pd_kernel_timing": [I32, I32, P, P],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_int
    lib.pd_last_error.argtypes = []
    lib.pd_last_error.restype = C.c_char_p
    return lib


lib = _load()


def _check(rc: int):
    if rc < 0:
        raise PolarDiskError(rc, lib.pd_last_error().decode(errors="replace"))
    return rc


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def mesh_desc(m, n, r_kind=0, p=1.0, th_kind=0, q=1.0, r_explicit=None, th_explicit=None):
    md = MeshDesc(int(m), int(n), int(r_kind), float(p), int(th_kind), float(q), None, None)
    keep = []
    if r_explicit is not None:
        a = _f64(r_explicit)
        keep.append(a)
        md.r_explicit = _ptr(a)
    if th_explicit is not None:
        a = _f64(th_explicit)
        keep.append(a)
        md.th_explicit = _ptr(a)
    md._keep = keep
    return md


def mesh_coords(md: MeshDesc):
    """Library mesh: (r_nodes, r_faces, th_nodes, th_faces)."""
    m, n = md.nr, md.ntheta
    r = np.empty(m + 2)
    rf = np.empty(m + 1)
    th = np.empty(n + 1)
    tf = np.empty(n)
    _check(lib.pd_mesh_coords(C.byref(md), _ptr(r), _ptr(rf), _ptr(th), _ptr(tf)))
    return r, rf, th, tf


def ring_vector(origin, grid):
    """(origin, (m, n) grid) -> ring-layout node vector of length m n + 1."""
    return np.concatenate([[float(origin)], np.asarray(grid, np.float64).reshape(-1)])


def time_desc(theta, K, T=None, t_kind=TIME_UNIFORM, l=1.0, table=None, tol=1e-12, max_iters=0,
              max_seconds=0.0):
    td = TimeDesc(int(t_kind), int(K), float(T or 0.0), float(l), None, float(theta), float(tol),
                  int(max_iters), 0.0, 0.0, 0.0, 0.0, float(max_seconds))
    if table is not None:
        a = _f64(table)
        td.t_table = _ptr(a)
        td.t_kind = TIME_TABLE
        td._keep = a
    return td


def adaptive_time_desc(theta, T, dt0, tol_time, dt_min, dt_max, K_max=20000, tol=1e-12, max_iters=0,
                       max_seconds=0.0):
    """A-posteriori step control from the current time to T later: the GPU
    picks every Δt from its local error estimate (statistics past the steps
    taken have dt = 0)."""
    return TimeDesc(TIME_ADAPTIVE, int(K_max), float(T), 1.0, None, float(theta), float(tol),
                    int(max_iters), float(dt0), float(dt_min), float(dt_max), float(tol_time),
                    float(max_seconds))


def taken(stats):
    """The steps an (adaptive) solve took: statistics with dt > 0."""
    return [s for s in stats if s["dt"] > 0.0]


def time_levels(td: TimeDesc, t_start=0.0):
    """The K+1 time levels a solve with `td` advances through from t_start."""
    out = np.empty(td.K + 1)
    _check(lib.pd_time_levels(C.byref(td), float(t_start), _ptr(out)))
    return out


def problem_desc(data: dict, flux=0, bc=0):
    """Builds a ProblemDesc from sampled problem data (origin/grid pieces, ring layout)."""
    m, n = data["m"], data["n"]
    keep = {}

    def put(key, arr):
        a = _f64(arr)
        keep[key] = a
        return _ptr(a)

    ns = int(len(data["lam"]))
    pd_ = ProblemDesc()
    pd_.pde = int(data.get("pde", 1))
    pd_.flux = int(flux)
    pd_.bc = int(bc)
    pd_.layout = LAYOUT_RING
    pd_.device_ptrs = 0
    pd_.b_node = put("b", ring_vector(data["b_origin"], data["b_grid"])) \
        if np.any(np.asarray(data["b_grid"]) != 0) or data["b_origin"] != 0 else None
    pd_.D_rface = put("Dr", np.asarray(data["D_r"]).reshape(m + 1, n))
    pd_.Er_rface = put("Er", np.asarray(data["Er_r"]).reshape(m + 1, n))
    pd_.D_tface = put("Dt", np.asarray(data["D_t"]).reshape(m, n))
    pd_.Et_tface = put("Et", np.asarray(data["Et_t"]).reshape(m, n))
    pd_.nsrc = ns
    pd_.lam = put("lam", data["lam"])
    tp = np.ascontiguousarray(data["tpow"], dtype=np.int32)
    keep["tpow"] = tp
    pd_.tpow = _ptr(tp)
    pd_.g = put("g", np.stack([ring_vector(data["g_origin"][q], data["g_grid"][q]) for q in range(ns)]))
    pd_.nb = put("nb", np.asarray(data["nb"]).reshape(ns, n))
    pd_.u0 = put("u0", ring_vector(data["u0_origin"], data["u0_grid"]))
    if flux == FLUX_LITERAL and "E_grid" in data:
        pd_.E_node = put("E", ring_vector(data["E_origin"], data["E_grid"]))
        pd_.D_origin = float(data["D_origin"])
    pd_._keep = keep
    return pd_


def footprint(md: MeshDesc, nsrc=1, precision=PD_FP64) -> int:
    b = C.c_size_t()
    _check(lib.pd_footprint(C.byref(md), int(nsrc), int(precision), C.byref(b)))
    return int(b.value)


class Instance:
    """One disk problem resident on the GPU."""

    def __init__(self, md: MeshDesc, data: dict, precision=PD_FP64, flux=0, bc=0, stream=None):
        self._create(md, problem_desc(data, flux, bc), precision, stream)

    @classmethod
    def from_desc(cls, md: MeshDesc, pdesc: ProblemDesc, precision=PD_FP64, stream=None):
        """An instance from a problem descriptor built by the caller (for
        instance one whose arrays are device pointers, device_ptrs = 1)."""
        inst = cls.__new__(cls)
        inst._create(md, pdesc, precision, stream)
        return inst

    def _create(self, md, pdesc, precision, stream):
        self.h = None
        self.md = md
        self.m, self.n = md.nr, md.ntheta
        self.N = self.m * self.n + 1
        self.precision = precision
        h = C.c_void_p()
        _check(lib.pd_mesh_create(C.byref(md), C.byref(pdesc), int(precision),
                                  C.c_void_p(stream) if stream else None, C.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            _check(lib.pd_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def step(self, t, dt, theta, tol=1e-12):
        st = StepStats()
        _check(lib.pd_scheme_step(self.h, float(t), float(dt), float(theta), float(tol), C.byref(st)))
        return st.as_dict()

    def solve(self, td: TimeDesc):
        st = (StepStats * td.K)()
        _check(lib.pd_solve_to_T(self.h, C.byref(td), C.cast(st, C.c_void_p)))
        return [s.as_dict() for s in st]

    def solution(self, layout=LAYOUT_RING):
        out = np.empty(self.N)
        _check(lib.pd_get_solution(self.h, _ptr(out), int(layout), 0))
        return out

    @property
    def time(self) -> float:
        t = C.c_double()
        _check(lib.pd_get_time(self.h, C.byref(t)))
        return t.value

    def set_solution(self, x, t, layout=LAYOUT_RING):
        a = _f64(x)
        _check(lib.pd_set_solution(self.h, _ptr(a), int(layout), 0, float(t)))

    def apply(self, x, dt, theta, layout=LAYOUT_RING, precision=0):
        a = _f64(x)
        y = np.empty(self.N)
        _check(lib.pd_apply_operator(self.h, float(dt), float(theta), _ptr(a), _ptr(y), int(layout),
                                     0, int(precision)))
        return y

    def precondition(self, y, dt, theta, layout=LAYOUT_RING):
        """z = M^{-1} y of the preconditioner of the step system at (dt, θ)."""
        a = _f64(y)
        z = np.empty(self.N)
        _check(lib.pd_apply_preconditioner(self.h, float(dt), float(theta), _ptr(a), _ptr(z), int(layout), 0))
        return z

    def rhs(self, t, dt, theta, layout=LAYOUT_RING):
        y = np.empty(self.N)
        _check(lib.pd_assemble_rhs(self.h, float(t), float(dt), float(theta), _ptr(y), int(layout), 0))
        return y


def solve_batch(instances: Sequence[Instance], tds: Sequence[TimeDesc]):
    """Advances all instances together; returns every step's statistics per instance."""
    n = len(instances)
    hs = (C.c_void_p * n)(*[i.h for i in instances])
    arr = (TimeDesc * n)(*tds)
    sts = [(StepStats * td.K)() for td in tds]
    ptrs = (C.c_void_p * n)(*[C.cast(s, C.c_void_p) for s in sts])
    _check(lib.pd_solve_batch(hs, n, arr, ptrs))
    return [[s.as_dict() for s in st] for st in sts]


def error_indicator(inst: "Instance", p_current: float, candidates=(), want_eta=False):
    """Indicator of the instance's current state and the recommended radial stretch."""
    cand = _f64(list(candidates)) if len(candidates) else None
    kappa = np.empty(inst.m)
    eta = np.empty(inst.m * inst.n) if want_eta else None
    res = Indicator()
    _check(lib.pd_error_indicator(inst.h, float(p_current), _ptr(cand) if cand is not None else None,
                                  len(candidates), _ptr(kappa), _ptr(eta) if eta is not None else None,
                                  C.byref(res)))
    out = res.as_dict()
    out["kappa"] = kappa
    out["eta"] = eta.reshape(inst.m, inst.n) if eta is not None else None
    return out


def error_indicator_noalloc(inst: "Instance", p_current: float, candidates=(), eta_device_ptr=None):
    """The same indicator through the allocation-free entry point; the field
    (if wanted) goes to caller-owned device memory at eta_device_ptr (m*n
    doubles, ring-major)."""
    cand = _f64(list(candidates)) if len(candidates) else None
    kappa = np.empty(inst.m)
    res = Indicator()
    _check(lib.pd_error_indicator_noalloc(inst.h, float(p_current), _ptr(cand) if cand is not None else None,
                                          len(candidates), _ptr(kappa),
                                          C.c_void_p(eta_device_ptr) if eta_device_ptr else None,
                                          C.byref(res)))
    out = res.as_dict()
    out["kappa"] = kappa
    return out


def remesh_transfer(src: "Instance", dst: "Instance"):
    """Sets dst's state (another mesh of the same problem) from src's by cubic interpolation."""
    _check(lib.pd_remesh_transfer(src.h, dst.h))


class Batch:
    """Serving loop: requests of any size, PDE and precision are submitted at
    any time and advanced together, level by level, in shared launches."""

    def __init__(self, pool_bytes: int, max_slots: int, stream=None):
        h = C.c_void_p()
        _check(lib.pd_batch_create(C.c_size_t(int(pool_bytes)), int(max_slots),
                                   C.c_void_p(stream) if stream else None, C.byref(h)))
        self.h = h
        self.sizes = {}

    def submit(self, md: MeshDesc, data: dict, td: TimeDesc, precision=PD_FP64, flux=0, bc=0) -> int:
        pdesc = problem_desc(data, flux, bc)
        t = C.c_uint64()
        _check(lib.pd_batch_submit(self.h, C.byref(md), C.byref(pdesc), C.byref(td), int(precision),
                                   C.byref(t)))
        self.sizes[t.value] = md.nr * md.ntheta + 1
        return t.value

    def poll(self, ticket: int):
        """None while pending, else (solution, summary); raises on a failed solve."""
        out = np.empty(self.sizes[ticket])
        sm = RequestSummary()
        rc = lib.pd_batch_poll(self.h, C.c_uint64(ticket), _ptr(out), C.byref(sm))
        if rc == PD_PENDING:
            return None
        del self.sizes[ticket]
        _check(rc)
        return out, sm.as_dict()

    def wait(self, ticket: int, timeout: float = 120.0, interval: float = 1e-3):
        import time as _time
        t_end = _time.monotonic() + timeout
        while True:
            r = self.poll(ticket)
            if r is not None:
                return r
            if _time.monotonic() > t_end:
                raise TimeoutError(f"ticket {ticket} still pending after {timeout} s")
            _time.sleep(interval)

    def stats(self) -> dict:
        info = BatchInfo()
        _check(lib.pd_batch_stats(self.h, C.byref(info)))
        return info.as_dict()

    def close(self):
        if self.h:
            _check(lib.pd_batch_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def set_preconditioner(inst: "Instance", kind: int):
    """Preconditioner of the instance's later solves: PRECOND_LINE (the
    alternating line sweeps) or PRECOND_MG (the θ-semi-coarsening V-cycle
    built on them; FP64 instances solved on their own)."""
    _check(lib.pd_set_preconditioner(inst.h, int(kind)))


def set_mobility(carrier: "Instance", mu_rface, mu_tface, sign: float):
    """Makes `carrier` (FP64, created without drift) a carrier of the coupled
    system with charge sign +1 (holes) or -1 (electrons) and face
    mobilities mu_rface ((m+1, n)) and mu_tface ((m, n))."""
    mr = _f64(np.asarray(mu_rface).reshape(carrier.m + 1, carrier.n))
    mt = _f64(np.asarray(mu_tface).reshape(carrier.m, carrier.n))
    _check(lib.pd_set_mobility(carrier.h, _ptr(mr), _ptr(mt), float(sign), 0))


def gummel_step(psi: "Instance", n_carrier: "Instance", p_carrier: "Instance", t, dt, theta, tol=1e-12,
                gummel_tol=1e-10, max_gummel=30):
    """One time level of the coupled system (potential, electrons, holes) by
    Gummel's iteration; returns its statistics."""
    st = GummelStats()
    _check(lib.pd_gummel_step(psi.h, n_carrier.h, p_carrier.h, float(t), float(dt), float(theta), float(tol),
                              float(gummel_tol), int(max_gummel), C.byref(st)))
    return {"gummel_iters": st.gummel_iters, "krylov_iters": st.krylov_iters, "change": st.change}


class Schedule(C.Structure):
    _fields_ = [("groups", C.c_int32), ("cycles_per_graph", C.c_int32),
                ("stencil_rings", C.c_int32)]


def set_schedule(groups=1, cycles_per_graph=2, stencil_rings=4):
    """Default launch schedule of later solves: stream groups, cycles per
    graph, and the stencil tile depth (rings per wave)."""
    sc = Schedule(int(groups), int(cycles_per_graph), int(stencil_rings))
    _check(lib.pd_set_schedule(C.byref(sc)))


def get_schedule():
    sc = Schedule()
    _check(lib.pd_get_schedule(C.byref(sc)))
    return {"groups": sc.groups, "cycles_per_graph": sc.cycles_per_graph,
            "stencil_rings": sc.stencil_rings}


def kernel_timing(enable: bool, reset: bool = False):
    """Per-family kernel time (ms) and launch counts since the last reset."""
    ms = np.zeros(len(KERNEL_FAMILIES))
    cnt = np.zeros(len(KERNEL_FAMILIES), dtype=np.int64)
    _check(lib.pd_kernel_timing(int(enable), int(reset), _ptr(ms), _ptr(cnt)))
    return dict(zip(KERNEL_FAMILIES, ms)), dict(zip(KERNEL_FAMILIES, cnt))
