"""ctypes binding of the CPU oracle (``liborc.so``, built from ``orc.c``).

TEST INFRASTRUCTURE ONLY.  The oracle is a plain FP64 CPU restatement of the
particle time step of the non-hybrid PDF method; it checks the GPU library and is
loaded only by the tests, the smoke check and the benchmark's CPU-baseline leg.
It shares no code with the GPU path.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.environ.get("ORC_LIB_OVERRIDE") or os.path.join(HERE, "liborc.so")
SRC = os.path.join(HERE, "orc.c")

NSTAT = 13
STAT_NAMES = ["W", "U1", "U2", "U3", "omega", "psi", "R11", "R22", "R33", "R12", "R13",
              "R23", "psi_var"]
COUNTER_NAMES = ["wall_a", "wall_b", "reflections", "fallbacks", "omega_reflections",
                 "c0_clamps", "walk_steps", "source_hits"]


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall",
           "-ffp-contract=off", "-o", LIB, SRC, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("oracle build failed:\n" + r.stderr)
    if verbose and r.stderr:
        print(r.stderr)
    return LIB


class Model(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("nu", "rho", "C3", "C4", "CT", "Cw1", "Cw2", "Cs", "Ct")]


class InitDesc(C.Structure):
    _fields_ = [("ppe", C.c_int32), ("u_sigma", C.c_double), ("omega_shape", C.c_double),
                ("src_x", C.c_double), ("src_y", C.c_double), ("src_r", C.c_double),
                ("src_continuous", C.c_int32), ("bins", C.c_int32 * 3),
                ("min_per_bin", C.c_int32), ("seed", C.c_uint64), ("problem", C.c_int32),
                ("estimator", C.c_int32), ("conditioning", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if "ORC_LIB_OVERRIDE" not in os.environ and (
            not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC)):
        build()
    L = C.CDLL(LIB)
    P = C.c_void_p
    dp, ip, u8p, u64p, i64p = (C.POINTER(C.c_double), C.POINTER(C.c_int32),
                               C.POINTER(C.c_uint8), C.POINTER(C.c_uint64),
                               C.POINTER(C.c_int64))
    sig = {
        "orc_philox4x32_10": (None, [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]),
        "orc_u01": (C.c_double, [C.c_uint32]),
        "orc_box_muller": (None, [C.c_uint32, C.c_uint32, dp]),
        "orc_normals": (None, [C.c_uint64, C.c_int32, C.c_uint64, C.c_uint32, C.c_uint32, C.c_int64, dp]),
        "orc_gamma": (C.c_double, [C.c_double, C.c_double, C.c_uint64, C.c_int32, C.c_uint64, C.c_uint32, C.c_uint32]),
        "orc_grid_create": (P, [C.c_int64, dp, C.c_int64, ip, u8p, C.c_double, dp, dp, dp, dp, dp,
                                C.POINTER(Model), C.c_char_p, C.c_int32]),
        "orc_grid_destroy": (None, [P]),
        "orc_grid_export": (None, [P, dp, dp, ip, u8p, dp, dp, u8p, dp]),
        "orc_bary": (None, [P, C.c_int32, C.c_double, C.c_double, dp]),
        "orc_locate_brute": (C.c_int32, [P, C.c_double, C.c_double, dp]),
        "orc_init": (P, [P, C.POINTER(InitDesc), C.c_char_p, C.c_int32]),
        "orc_ens_destroy": (None, [P]),
        "orc_step": (C.c_int32, [P, C.c_double]),
        "orc_count": (C.c_int64, [P]),
        "orc_step_index": (C.c_int64, [P]),
        "orc_export": (None, [P, dp, dp, dp, dp, dp, dp, u64p, ip]),
        "orc_import": (C.c_int32, [P, C.c_int64, dp, dp, dp, dp, dp, dp, u64p, ip, C.c_int64, C.c_uint64]),
        "orc_stats": (C.c_int32, [P, dp]),
        "orc_refresh_stats": (C.c_int32, [P]),
        "orc_feedback": (C.c_int32, [P, C.c_double, C.c_int32]),
        "orc_shift_velocities": (C.c_int32, [P, dp, dp]),
        "orc_set_grad_p": (None, [P, dp]),
        "orc_set_wp": (None, [P, dp]),
        "orc_cfl_dt": (C.c_double, [P, C.c_double]),
        "orc_redistribute": (C.c_int64, [P, C.c_int32]),
        "orc_control": (C.c_int32, [P, C.c_int32, C.c_int32, i64p]),
        "orc_counters": (None, [P, i64p]),
        "orc_bin_element": (C.c_int32, [C.c_int32, dp, u64p, ip, C.c_int32, ip, ip]),
        "orc_project_element": (C.c_int32, [C.c_int32, dp, dp, dp, u64p, C.c_int32, C.c_int32, dp, ip, ip, dp]),
        "orc_tm": (C.c_double, [P, C.c_int32]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def _d(a):
    return _p(np.ascontiguousarray(a, dtype=np.float64), C.c_double)


# ------------------------------------------------------------------------ units

def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def u01(w):
    return lib().orc_u01(int(w) & 0xFFFFFFFF)


def box_muller(a, b):
    o = (C.c_double * 2)()
    lib().orc_box_muller(int(a) & 0xFFFFFFFF, int(b) & 0xFFFFFFFF, o)
    return o[0], o[1]


def normals(seed, problem, pid, step, tag, n):
    out = np.empty(n, dtype=np.float64)
    lib().orc_normals(seed, problem, pid, step, tag, n, _p(out, C.c_double))
    return out


def gamma(shape, mean, seed, problem, pid, step, tag):
    return lib().orc_gamma(shape, mean, seed, problem, pid, step, tag)


def bin_element(u, pid, bins, min_per_bin=2):
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1, 3)
    pid = np.ascontiguousarray(pid, dtype=np.uint64)
    n = u.shape[0]
    pos = np.empty(n, dtype=np.int32)
    b = np.empty(n, dtype=np.int32)
    bb = (C.c_int32 * 3)(*bins)
    cp = lib().orc_bin_element(n, _p(u, C.c_double), _p(pid, C.c_uint64), bb, min_per_bin,
                               _p(pos, C.c_int32), _p(b, C.c_int32))
    return cp, pos, b


def project_element(u, psi, w, pid, nc, min_per_bin=2):
    """Fox's projection of one element (Eqs. 64-66): (bins used, key, pos, bin, alpha)."""
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1, 3)
    psi = np.ascontiguousarray(psi, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    pid = np.ascontiguousarray(pid, dtype=np.uint64)
    n = u.shape[0]
    key = np.empty(n)
    pos = np.empty(n, dtype=np.int32)
    b = np.empty(n, dtype=np.int32)
    alpha = np.empty(3)
    cp = lib().orc_project_element(n, _p(u, C.c_double), _p(psi, C.c_double), _p(w, C.c_double),
                                   _p(pid, C.c_uint64), int(nc), int(min_per_bin), _p(key, C.c_double),
                                   _p(pos, C.c_int32), _p(b, C.c_int32), _p(alpha, C.c_double))
    return cp, key, pos, b, alpha


# ------------------------------------------------------------------------ grid / ensemble

class Grid:
    def __init__(self, mesh, fields, model: dict):
        L = lib()
        self.mesh = mesh
        self._keep = [np.ascontiguousarray(mesh.xy, np.float64),
                      np.ascontiguousarray(mesh.tri, np.int32),
                      np.ascontiguousarray(mesh.edge_kind, np.uint8)]
        self._f = [np.ascontiguousarray(a, np.float64) for a in fields.as_tuple()]
        self.model = Model(**{n: float(model[n]) for n, _ in Model._fields_})
        err = C.create_string_buffer(256)
        self.h = L.orc_grid_create(mesh.n_nodes, _p(self._keep[0], C.c_double), mesh.n_elems,
                                   _p(self._keep[1], C.c_int32), _p(self._keep[2], C.c_uint8),
                                   float(mesh.period_x), *[_p(a, C.c_double) for a in self._f],
                                   C.byref(self.model), err, 256)
        if not self.h:
            raise ValueError("oracle grid: " + err.value.decode())
        self.nn, self.ne = mesh.n_nodes, mesh.n_elems

    def export(self):
        ne, nn = self.ne, self.nn
        out = dict(frame=np.empty((ne, 6)), area=np.empty(ne), nbr=np.empty((ne, 3), np.int32),
                   kind=np.empty((ne, 3), np.uint8), gradu=np.empty((ne, 6)),
                   lapu=np.empty((nn, 3)), wall=np.empty(ne, np.uint8), wline=np.empty((ne, 4)))
        lib().orc_grid_export(self.h, _p(out["frame"], C.c_double), _p(out["area"], C.c_double),
                              _p(out["nbr"], C.c_int32), _p(out["kind"], C.c_uint8),
                              _p(out["gradu"], C.c_double), _p(out["lapu"], C.c_double),
                              _p(out["wall"], C.c_uint8), _p(out["wline"], C.c_double))
        return out

    def set_grad_p(self, gp):
        """Replaces the nodal mean pressure gradient field [nn, 2]."""
        gp = np.ascontiguousarray(gp, np.float64)
        lib().orc_set_grad_p(self.h, _p(gp, C.c_double))

    def set_wp(self, wp):
        """Replaces the nodal elliptic-relaxation tensor, wp [nn, 3, 3]."""
        wp = np.ascontiguousarray(wp, np.float64)
        lib().orc_set_wp(self.h, _p(wp, C.c_double))

    def bary(self, e, x, y):
        o = (C.c_double * 3)()
        lib().orc_bary(self.h, int(e), float(x), float(y), o)
        return np.array(o[:])

    def locate_brute(self, x, y):
        xs = C.c_double(0.0)
        e = lib().orc_locate_brute(self.h, float(x), float(y), C.byref(xs))
        return e, xs.value

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().orc_grid_destroy(self.h)
                self.h = None
        except Exception:
            pass


def make_init(d: dict, problem: int = 0) -> InitDesc:
    s = InitDesc()
    s.ppe = int(d["ppe"]); s.u_sigma = float(d["u_sigma"]); s.omega_shape = float(d["omega_shape"])
    s.src_x, s.src_y, s.src_r = float(d["src_x"]), float(d["src_y"]), float(d["src_r"])
    s.src_continuous = int(d["src_continuous"])
    for i in range(3):
        s.bins[i] = int(d["bins"][i])
    s.min_per_bin = int(d["min_per_bin"]); s.seed = int(d["seed"]); s.problem = int(problem)
    s.estimator = int(d.get("estimator", 0))
    s.conditioning = int(d.get("conditioning", 0))
    return s


class Ensemble:
    def __init__(self, grid: Grid, init: dict, problem: int = 0):
        self.grid = grid
        self.desc = make_init(init, problem)
        err = C.create_string_buffer(256)
        self.h = lib().orc_init(grid.h, C.byref(self.desc), err, 256)
        if not self.h:
            raise ValueError("oracle init: " + err.value.decode())

    def step(self, dt: float, n: int = 1):
        for _ in range(n):
            rc = lib().orc_step(self.h, float(dt))
            if rc != 0:
                raise RuntimeError(f"oracle step failed: {rc}")

    def count(self) -> int:
        return int(lib().orc_count(self.h))

    @property
    def step_index(self) -> int:
        return int(lib().orc_step_index(self.h))

    def export(self, sort_by_pid: bool = True) -> dict:
        n = self.count()
        o = dict(x=np.empty(n), y=np.empty(n), u=np.empty((n, 3)), om=np.empty(n),
                 psi=np.empty(n), w=np.empty(n), pid=np.empty(n, np.uint64),
                 elem=np.empty(n, np.int32))
        lib().orc_export(self.h, *[_p(o[k], C.c_double) for k in ("x", "y", "u", "om", "psi", "w")],
                         _p(o["pid"], C.c_uint64), _p(o["elem"], C.c_int32))
        if sort_by_pid:
            order = np.argsort(o["pid"], kind="stable")
            o = {k: v[order] for k, v in o.items()}
        return o

    def import_state(self, st: dict, step: int, next_pid: int):
        n = len(st["x"])
        arrs = [np.ascontiguousarray(st[k], np.float64) for k in ("x", "y", "u", "om", "psi", "w")]
        pid = np.ascontiguousarray(st["pid"], np.uint64)
        el = np.ascontiguousarray(st["elem"], np.int32)
        rc = lib().orc_import(self.h, n, *[_p(a, C.c_double) for a in arrs], _p(pid, C.c_uint64),
                              _p(el, C.c_int32), int(step), int(next_pid))
        if rc != 0:
            raise RuntimeError(f"oracle import failed: {rc}")

    def stats(self) -> np.ndarray:
        out = np.empty((self.grid.nn, NSTAT))
        rc = lib().orc_stats(self.h, _p(out, C.c_double))
        if rc != 0:
            raise RuntimeError(f"oracle stats failed: {rc}")
        return out

    def feedback(self, alpha: float, feed_rey: bool = False, feed_omega: bool = False):
        """Nodal statistics of the last step become the grid's fields (mean velocity scaled
        by alpha, Reynolds stresses when feed_rey, mean frequency when feed_omega);
        gradients and Laplacians are derived again.  The grid is modified."""
        rc = lib().orc_feedback(self.h, float(alpha), int(bool(feed_rey)) | (2 if feed_omega else 0))
        if rc != 0:
            raise RuntimeError(f"orc_feedback: {rc}")

    def shift_velocities(self, de, dn):
        """Eq. (31) applied with per-element particle shifts de [ne, 2] and nodal shifts
        dn [nn, 2] of the mean velocity."""
        de = np.ascontiguousarray(de, np.float64)
        dn = np.ascontiguousarray(dn, np.float64)
        rc = lib().orc_shift_velocities(self.h, _p(de, C.c_double), _p(dn, C.c_double))
        if rc != 0:
            raise RuntimeError(f"orc_shift_velocities: {rc}")

    def redistribute(self, n_min: int) -> int:
        """App. B redistribution; returns the number of moves."""
        rc = lib().orc_redistribute(self.h, int(n_min))
        if rc < 0:
            raise RuntimeError(f"orc_redistribute: {rc}")
        return int(rc)

    def cfl_dt(self, cfl: float = 0.7) -> float:
        """Time step of Eq. (26) from the last statistics."""
        return float(lib().orc_cfl_dt(self.h, float(cfl)))

    def refresh_stats(self):
        lib().orc_refresh_stats(self.h)

    def control(self, n_min: int, n_max: int) -> dict:
        rep = (C.c_int64 * 6)()
        rc = lib().orc_control(self.h, int(n_min), int(n_max), rep)
        if rc != 0:
            raise RuntimeError(f"oracle control failed: {rc}")
        return dict(zip(["live", "cloned", "merged", "empty", "below", "above"], rep[:]))

    def counters(self) -> dict:
        o = (C.c_int64 * 8)()
        lib().orc_counters(self.h, o)
        return dict(zip(COUNTER_NAMES, o[:]))

    def tm(self, e: int) -> float:
        return lib().orc_tm(self.h, int(e))

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().orc_ens_destroy(self.h)
                self.h = None
        except Exception:
            pass
