"""ctypes binding of libpdfgpu.so (declared in include/pdf.h).

Argument marshalling only: every step of the particle time step runs in the HIP
kernels of the library.  The library must have been built (``__graft_entry__.build()``
or ``python paper_1006_0532_amd/build.py``); loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("PDFGPU_LIB") or os.path.join(HERE, "libpdfgpu.so")

PDF_NSTAT = 13
PDF_STATS_ALL = (1 << PDF_NSTAT) - 1   # stat_mask selecting every statistic
PDF_NCOUNTERS = 8
PDF_NTIMERS = 12
TIMER_NAMES = ["init", "advance", "scan", "scatter", "element_pass", "node_finalize",
               "control_plan", "control_scan", "control_apply", "fill", "count", "other"]
COUNTER_NAMES = ["wall_a", "wall_b", "reflections", "fallbacks", "omega_reflections",
                 "c0_clamps", "walk_steps", "source_hits"]
STATUS = {0: "OK", -1: "INVAL", -2: "NOMEM", -3: "HIP", -4: "MESH", -5: "CAPACITY", -6: "LOST",
          -7: "NONFINITE", -8: "STATE"}

# every symbol include/pdf.h declares
EXPORTS = ["pdf_grid_create", "pdf_grid_destroy", "pdf_particles_init", "pdf_ens_destroy", "pdf_step",
           "pdf_stats", "pdf_control", "pdf_count", "pdf_particles_export", "pdf_particles_import",
           "pdf_counters", "pdf_timing", "pdf_set_feedback", "pdf_cfl_dt", "pdf_cfl_dt_noalloc", "pdf_redistribute", "pdf_elliptic_relaxation",
           "pdf_pressure_projection", "pdf_get_options", "pdf_set_options", "pdf_autotune",
           "pdf_sync",
           "pdf_last_error"]
PDF_FP64, PDF_MIXED = 0, 1


class PdfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class MeshDesc(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("xy", C.POINTER(C.c_double)), ("n_elems", C.c_int64),
                ("tri", C.POINTER(C.c_int32)), ("edge_kind", C.POINTER(C.c_uint8)),
                ("period_x", C.c_double)]


class FieldsDesc(C.Structure):
    _fields_ = [(n, C.POINTER(C.c_double)) for n in ("grad_p", "wp", "mean_u", "mean_omega", "rey")]


class Model(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("nu", "rho", "C3", "C4", "CT", "Cw1", "Cw2", "Cs", "Ct")]


class InitDesc(C.Structure):
    _fields_ = [("ppe", C.c_int32), ("u_sigma", C.c_double), ("omega_shape", C.c_double),
                ("src_x", C.c_double), ("src_y", C.c_double), ("src_r", C.c_double),
                ("src_continuous", C.c_int32), ("bins", C.c_int32 * 3), ("min_per_bin", C.c_int32),
                ("precision", C.c_int32), ("seed", C.c_uint64), ("capacity", C.c_int64),
                ("estimator", C.c_int32), ("conditioning", C.c_int32)]


class EllipticModel(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("C1", "C2", "CL", "Ceta", "Cv", "gamma5")]


class Options(C.Structure):
    _fields_ = [("use_graph", C.c_int32), ("adv_block", C.c_int32), ("ppl", C.c_int32)]


class ControlReport(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("live", "cloned", "merged", "empty", "below", "above")]


_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library (no fallback of any kind)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libpdfgpu.so not built at {path}; run __graft_entry__.build()")
    L = C.CDLL(path)
    vp, dp, ip, u8p, u64p, i64p = (C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32),
                                   C.POINTER(C.c_uint8), C.POINTER(C.c_uint64), C.POINTER(C.c_int64))
    sig = {
        "pdf_grid_create": [C.POINTER(MeshDesc), C.POINTER(FieldsDesc), C.POINTER(Model), vp, C.POINTER(vp)],
        "pdf_grid_destroy": [vp],
        "pdf_particles_init": [C.POINTER(vp), C.POINTER(InitDesc), C.c_int32, vp, C.POINTER(vp)],
        "pdf_ens_destroy": [vp],
        "pdf_step": [vp, dp, C.c_int32, vp],
        "pdf_stats": [vp, C.c_int32, C.c_uint32, vp, C.c_int32, vp],
        "pdf_control": [vp, C.c_int32, C.c_int32, C.POINTER(ControlReport), vp],
        "pdf_count": [vp, C.c_int32, i64p],
        "pdf_particles_export": [vp, C.c_int32, C.c_int64, dp, dp, dp, dp, dp, dp, u64p, ip, i64p, vp],
        "pdf_particles_import": [vp, C.c_int32, C.c_int64, dp, dp, dp, dp, dp, dp, u64p, ip, C.c_int64,
                                 C.c_uint64, vp],
        "pdf_counters": [vp, C.c_int32, i64p],
        "pdf_timing": [vp, C.c_int32, dp, i64p],
        "pdf_set_feedback": [vp, C.c_int32, C.c_double, C.c_int32, vp],
        "pdf_cfl_dt": [vp, C.c_int32, C.c_double, dp, vp],
        "pdf_cfl_dt_noalloc": [vp, C.c_int32, C.c_double, vp, vp],
        "pdf_redistribute": [vp, C.c_int32, C.c_int32, C.POINTER(C.c_int64), vp],
        "pdf_elliptic_relaxation": [vp, C.POINTER(EllipticModel), C.c_double, C.c_int32, C.c_int32, vp, C.c_int32,
                                    C.POINTER(C.c_int32), vp],
        "pdf_pressure_projection": [vp, C.c_double, C.c_double, C.c_double, C.c_int32, vp, C.c_int32,
                                    C.POINTER(C.c_int32), vp],
        "pdf_get_options": [vp, C.POINTER(Options)],
        "pdf_set_options": [vp, C.POINTER(Options)],
        "pdf_autotune": [vp, dp, C.c_int32, vp, C.POINTER(Options), ip, dp],
        "pdf_sync": [vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int32
    L.pdf_last_error.argtypes = []
    L.pdf_last_error.restype = C.c_char_p
    _lib = L
    return L


def _check(st: int):
    if st != 0:
        raise PdfError(st, load().pdf_last_error().decode())


def _ptr(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def current_stream() -> int:
    """Handle of torch's current HIP stream (0 = default stream when torch is absent)."""
    try:
        import torch
        if torch.cuda.is_available():
            return int(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return 0


class Grid:
    def __init__(self, mesh, fields, model: dict, stream: int | None = None):
        L = load()
        self._xy = np.ascontiguousarray(mesh.xy, np.float64)
        self._tri = np.ascontiguousarray(mesh.tri, np.int32)
        self._kind = np.ascontiguousarray(mesh.edge_kind, np.uint8)
        self._f = [np.ascontiguousarray(a, np.float64) for a in fields.as_tuple()]
        md = MeshDesc(mesh.n_nodes, _ptr(self._xy, C.c_double), mesh.n_elems, _ptr(self._tri, C.c_int32),
                      _ptr(self._kind, C.c_uint8), float(mesh.period_x))
        fd = FieldsDesc(*[_ptr(a, C.c_double) for a in self._f])
        mo = Model(**{n: float(model[n]) for n, _ in Model._fields_})
        h = C.c_void_p()
        _check(L.pdf_grid_create(C.byref(md), C.byref(fd), C.byref(mo),
                                 C.c_void_p(current_stream() if stream is None else stream), C.byref(h)))
        self.h = h
        self.nn, self.ne = mesh.n_nodes, mesh.n_elems

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            load().pdf_grid_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_init(d: dict, capacity: int = 0, precision: int = 0) -> InitDesc:
    s = InitDesc()
    s.ppe = int(d["ppe"]); s.u_sigma = float(d["u_sigma"]); s.omega_shape = float(d["omega_shape"])
    s.src_x, s.src_y, s.src_r = float(d["src_x"]), float(d["src_y"]), float(d["src_r"])
    s.src_continuous = int(d["src_continuous"])
    for i in range(3):
        s.bins[i] = int(d["bins"][i])
    s.min_per_bin = int(d["min_per_bin"]); s.precision = int(precision); s.seed = int(d["seed"])
    s.capacity = int(capacity or d.get("capacity", 0))
    s.estimator = int(d.get("estimator", 0))
    s.conditioning = int(d.get("conditioning", 0))
    return s


class Ensemble:
    """Particles of one problem, or of several independent problems advanced together
    (grid and init may be lists of equal length; problem p is numbered p)."""

    def __init__(self, grid, init, capacity: int = 0, precision: int = PDF_FP64, stream: int | None = None):
        L = load()
        grids = list(grid) if isinstance(grid, (list, tuple)) else [grid]
        inits = list(init) if isinstance(init, (list, tuple)) else [init]
        if len(grids) != len(inits):
            raise ValueError("one init descriptor per grid")
        self.grids = grids
        self.grid = grids[0]
        self.n_problems = len(grids)
        self.precision = int(precision)
        if isinstance(capacity, (list, tuple)):
            caps = list(capacity)
        elif self.n_problems == 1 or not capacity:
            caps = [capacity] + [0] * (self.n_problems - 1)
        else:
            raise ValueError("several problems take one capacity per problem")
        descs = (InitDesc * self.n_problems)(*[make_init(d, c, precision) for d, c in zip(inits, caps)])
        self.desc = descs[0]
        self._descs = descs
        hs = (C.c_void_p * self.n_problems)(*[g.h.value for g in grids])
        h = C.c_void_p()
        self.stream = current_stream() if stream is None else stream
        _check(L.pdf_particles_init(hs, descs, self.n_problems, C.c_void_p(self.stream), C.byref(h)))
        self.h = h

    def _dts(self, dt):
        v = list(dt) if isinstance(dt, (list, tuple, np.ndarray)) else [dt] * self.n_problems
        if len(v) != self.n_problems:
            raise ValueError("one time step per problem")
        return (C.c_double * self.n_problems)(*[float(x) for x in v])

    def step(self, dt, n: int = 1):
        _check(load().pdf_step(self.h, self._dts(dt), int(n), C.c_void_p(self.stream)))

    def sync(self):
        _check(load().pdf_sync(self.h))

    def stats(self, problem: int = 0, mask: int = PDF_STATS_ALL) -> np.ndarray:
        """Nodal statistics [n_nodes][k] of the statistics whose bits are set in mask."""
        k = bin(int(mask) & PDF_STATS_ALL).count("1") or 1
        out = np.empty((self.grids[problem].nn, k))
        _check(load().pdf_stats(self.h, int(problem), int(mask), out.ctypes.data_as(C.c_void_p), 0,
                                C.c_void_p(self.stream)))
        return out

    def stats_device(self, ptr: int, problem: int = 0, mask: int = PDF_STATS_ALL):
        _check(load().pdf_stats(self.h, int(problem), int(mask), C.c_void_p(ptr), 1, C.c_void_p(self.stream)))

    # check=False: a sticky device error does not raise; its status is kept in
    # self.last_status and the call's outputs (filled before the error is reported) are
    # returned, so that the state after the error can be inspected
    def _status(self, st: int, check: bool):
        self.last_status = int(st)
        if check:
            _check(st)
        elif st not in (0, -5, -6, -7):
            _check(st)

    def control(self, n_min: int, n_max: int, check: bool = True, report: bool = True):
        """Number control; report=False only enqueues it (no synchronisation) and returns None."""
        if not report:
            self._status(load().pdf_control(self.h, int(n_min), int(n_max), None, C.c_void_p(self.stream)), check)
            return None
        r = ControlReport()
        self._status(load().pdf_control(self.h, int(n_min), int(n_max), C.byref(r), C.c_void_p(self.stream)),
                     check)
        return {n: getattr(r, n) for n, _ in ControlReport._fields_}

    def count(self, problem: int = -1, check: bool = True) -> int:
        v = C.c_int64()
        self._status(load().pdf_count(self.h, int(problem), C.byref(v)), check)
        return int(v.value)

    def export(self, sort_by_pid: bool = True, problem: int = 0, check: bool = True) -> dict:
        n = self.count(problem, check)
        o = dict(x=np.empty(n), y=np.empty(n), u=np.empty((n, 3)), om=np.empty(n), psi=np.empty(n),
                 w=np.empty(n), pid=np.empty(n, np.uint64), elem=np.empty(n, np.int32))
        got = C.c_int64()
        self._status(load().pdf_particles_export(self.h, int(problem), n, *[_ptr(o[k], C.c_double) for k in
                                                                            ("x", "y", "u", "om", "psi", "w")],
                                                 _ptr(o["pid"], C.c_uint64), _ptr(o["elem"], C.c_int32),
                                                 C.byref(got), C.c_void_p(self.stream)), check)
        assert got.value == n
        if sort_by_pid:
            order = np.argsort(o["pid"], kind="stable")
            o = {k: v[order] for k, v in o.items()}
        return o

    def import_state(self, st: dict, step: int, next_pid: int):
        n = len(st["x"])
        arrs = [np.ascontiguousarray(st[k], np.float64) for k in ("x", "y", "u", "om", "psi", "w")]
        pid = np.ascontiguousarray(st["pid"], np.uint64)
        el = np.ascontiguousarray(st["elem"], np.int32)
        _check(load().pdf_particles_import(self.h, 0, n, *[_ptr(a, C.c_double) for a in arrs],
                                           _ptr(pid, C.c_uint64), _ptr(el, C.c_int32), int(step),
                                           int(next_pid), C.c_void_p(self.stream)))

    def counters(self, problem: int = 0) -> dict:
        o = (C.c_int64 * PDF_NCOUNTERS)()
        _check(load().pdf_counters(self.h, int(problem), o))
        return dict(zip(COUNTER_NAMES, o[:]))

    def timing(self, enable: bool):
        ms = (C.c_double * PDF_NTIMERS)()
        cnt = (C.c_int64 * PDF_NTIMERS)()
        _check(load().pdf_timing(self.h, int(enable), ms, cnt))
        return {TIMER_NAMES[i]: (ms[i], cnt[i]) for i in range(PDF_NTIMERS)}

    def set_feedback(self, enable: bool = True, alpha: float = 1.0, feed_rey: bool = False,
                     feed_omega: bool = False):
        """Feed the nodal statistics back into the fields now and after every step."""
        flags = int(bool(feed_rey)) | (2 if feed_omega else 0)
        _check(load().pdf_set_feedback(self.h, int(bool(enable)), float(alpha), flags, C.c_void_p(self.stream)))

    def cfl_dt(self, cfl: float = 0.7, problem: int = 0) -> float:
        """Time step of Eq. (26) from the last statistics."""
        v = C.c_double()
        _check(load().pdf_cfl_dt(self.h, int(problem), float(cfl), C.byref(v), C.c_void_p(self.stream)))
        return float(v.value)

    def cfl_dt_noalloc(self, dt_out_ptr: int, cfl: float = 0.7, problem: int = 0):
        """Eq. (26) into one double of device memory at dt_out_ptr (enqueued, no sync)."""
        _check(load().pdf_cfl_dt_noalloc(self.h, int(problem), float(cfl), C.c_void_p(dt_out_ptr),
                                         C.c_void_p(self.stream)))

    def redistribute(self, n_min: int, problem: int = -1) -> int:
        """Particle redistribution of App. B; returns the number of moves."""
        v = C.c_int64()
        _check(load().pdf_redistribute(self.h, int(problem), int(n_min), C.byref(v), C.c_void_p(self.stream)))
        return int(v.value)

    def elliptic_relaxation(self, consts: dict | None = None, tol: float = 1e-12, max_iter: int = 20000,
                            store: bool = False):
        """Eq. (12) from the current statistics: (wp [nn, 3, 3], CG iterations); store makes
        the solution the ensemble's wp field for the following steps."""
        nn = self.grids[0].nn
        out = np.empty((nn, 3, 3))
        it = C.c_int32()
        m = None if consts is None else C.byref(EllipticModel(**consts))
        _check(load().pdf_elliptic_relaxation(self.h, m, float(tol), int(max_iter), int(bool(store)),
                                              out.ctypes.data_as(C.c_void_p), 0, C.byref(it), C.c_void_p(self.stream)))
        return out, int(it.value)

    def pressure_projection(self, dt: float, cp: float = 1e-3, tol: float = 1e-12, max_iter: int = 50000):
        """Eqs. (30)-(33) and (31) after a step: (dP [nn], CG iterations)."""
        nn = self.grids[0].nn
        out = np.empty(nn)
        it = C.c_int32()
        _check(load().pdf_pressure_projection(self.h, float(dt), float(cp), float(tol), int(max_iter),
                                              out.ctypes.data_as(C.c_void_p), 0, C.byref(it), C.c_void_p(self.stream)))
        return out, int(it.value)

    def options(self) -> dict:
        o = Options()
        _check(load().pdf_get_options(self.h, C.byref(o)))
        return {n: getattr(o, n) for n, _ in Options._fields_}

    def set_options(self, **kw):
        cur = self.options()
        cur.update(kw)
        o = Options(**{n: int(cur[n]) for n, _ in Options._fields_})
        _check(load().pdf_set_options(self.h, C.byref(o)))

    def autotune(self, dt, steps_per_trial: int = 2):
        """Times the candidate launch options on the live ensemble (which advances) and
        keeps the fastest; returns (chosen options, [trial ms])."""
        o = Options()
        n = C.c_int32(16)
        ms = (C.c_double * 16)()
        _check(load().pdf_autotune(self.h, self._dts(dt), int(steps_per_trial), C.c_void_p(self.stream),
                                   C.byref(o), C.byref(n), ms))
        return {k: getattr(o, k) for k, _ in Options._fields_}, list(ms[:n.value])

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            load().pdf_ens_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
