"""FP64 CPU oracle for the FED-FEM bio-heat step -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this package.  The product (the GPU library and its binding) never imports
it, and it never imports the product.  The arithmetic lives in
`fedfem_oracle.c` (plain C, double precision, Algorithm 1 of the paper); this
module marshals arrays through ctypes and adds the dense brute-force checks
(`dense.py`) and closed forms (`closed_forms.py`).
"""
from __future__ import annotations

import ctypes as C
import os
import time

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

M_FIELDS = ("rho0", "c0", "k0", "drho_dT", "dc_dT", "dk_dT", "T_ref", "T_lo",
            "T_hi", "w_b", "c_b", "T_a", "Q_m")


class _Problem(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("n_tets", C.c_int64),
                ("tets", C.c_void_p), ("A", C.c_void_p), ("Vi", C.c_void_p),
                ("mat", C.c_void_p), ("is_dir", C.c_void_p),
                ("T_dir", C.c_void_p), ("q", C.c_void_p),
                ("csr_off", C.c_void_p), ("csr_ec", C.c_void_p),
                ("dt", C.c_double), ("n_threads", C.c_int), ("tabs", C.c_void_p)]

MAX_TAB = 16
TAB_NAMES = ("k", "rho", "c")


def table_array(tables):
    """Property tables {name: (T, values)} -> the oracle's flat layout
    [3][count, MAX_TAB temperatures, MAX_TAB values] (None if empty)."""
    if not tables:
        return None
    out = np.zeros(3 * (1 + 2 * MAX_TAB))
    for p, name in enumerate(TAB_NAMES):
        if name in tables and tables[name] is not None:
            T, V = (np.asarray(a, dtype=np.float64) for a in tables[name])
            assert 1 <= len(T) == len(V) <= MAX_TAB and np.all(np.diff(T) > 0)
            b = p * (1 + 2 * MAX_TAB)
            out[b] = len(T)
            out[b + 1:b + 1 + len(T)] = T
            out[b + 1 + MAX_TAB:b + 1 + MAX_TAB + len(V)] = V
    return out


def lib():
    global _lib
    if _lib is None:
        path = os.path.join(_HERE, "libfedfem_oracle.so")
        src = os.path.join(_HERE, "fedfem_oracle.c")
        if (not os.path.exists(path)
                or os.path.getmtime(path) < os.path.getmtime(src)):
            _build.build()
        L = C.CDLL(path)
        P = C.c_void_p
        L.oracle_geometry.restype = C.c_int64
        L.oracle_geometry.argtypes = [C.c_int64, P, P, P, P, P, P, C.c_int]
        L.oracle_build_csr.argtypes = [C.c_int64, C.c_int64, P, P, P]
        L.oracle_lumped_volume.argtypes = [C.c_int64, P, P, P, P, C.c_int]
        L.oracle_step.argtypes = [P, P, P, P, P, P]
        L.oracle_run.restype = C.c_int
        L.oracle_run.argtypes = [P, C.c_int64, P]
        L.oracle_source_nodal.argtypes = [C.c_int64, P, P, C.c_int, P, P]
        L.oracle_source_consistent.argtypes = [C.c_int64, P, C.c_int64, P, P,
                                               P, P, C.c_int, P, P, C.c_int]
        L.oracle_quadrature_points.argtypes = [P]
        L.oracle_max_threads.restype = C.c_int
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def max_threads():
    return lib().oracle_max_threads()


def mat_vector(materials):
    """Material object (with the 13 named fields) -> float64[13]."""
    return np.array([float(getattr(materials, f)) for f in M_FIELDS])


class OracleModel:
    """Precomputed FED-FEM model (Algorithm 1, pre-computation block)."""

    def __init__(self, xyz, tets, materials, dir_nodes=(), dir_T=(),
                 n_threads=0, tables=None):
        self.xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        self.tets = np.ascontiguousarray(tets, dtype=np.int32)
        self.N = len(self.xyz)
        self.E = len(self.tets)
        self.n_threads = int(n_threads)
        self.mat = mat_vector(materials)
        self.tables = dict(tables) if tables else None
        self.tabs = table_array(self.tables)
        L = lib()
        self.A = np.empty((self.E, 4, 4))
        self.vol = np.empty(self.E)
        self.detJ = np.empty(self.E)
        self.gradN = np.empty((self.E, 4, 3))
        bad = L.oracle_geometry(self.E, _p(self.xyz), _p(self.tets),
                                _p(self.A), _p(self.vol), _p(self.detJ),
                                _p(self.gradN), self.n_threads)
        if bad >= 0:
            raise ValueError(f"degenerate tetrahedron {bad}")
        self.csr_off = np.empty(self.N + 1, dtype=np.int64)
        self.csr_ec = np.empty(4 * self.E, dtype=np.int64)
        L.oracle_build_csr(self.N, self.E, _p(self.tets), _p(self.csr_off),
                           _p(self.csr_ec))
        self.Vi = np.empty(self.N)
        L.oracle_lumped_volume(self.N, _p(self.vol), _p(self.csr_off),
                               _p(self.csr_ec), _p(self.Vi), self.n_threads)
        self.is_dir = np.zeros(self.N, dtype=np.uint8)
        self.T_dir = np.zeros(self.N)
        dn = np.asarray(dir_nodes, dtype=np.int64)
        self.is_dir[dn] = 1
        self.T_dir[dn] = np.asarray(dir_T, dtype=np.float64)
        self.q = np.zeros(self.N)
        self.dt = 0.0

    # -- sources -----------------------------------------------------------
    def source_nodal(self, sources):
        s = np.ascontiguousarray(sources, dtype=np.float64).reshape(-1, 5)
        q = np.empty(self.N)
        lib().oracle_source_nodal(self.N, _p(self.xyz), _p(self.Vi), len(s),
                                  _p(s), _p(q))
        return q

    def source_consistent(self, sources):
        s = np.ascontiguousarray(sources, dtype=np.float64).reshape(-1, 5)
        q = np.empty(self.N)
        lib().oracle_source_consistent(self.N, _p(self.xyz), self.E,
                                       _p(self.tets), _p(self.vol),
                                       _p(self.csr_off), _p(self.csr_ec),
                                       len(s), _p(s), _p(q), self.n_threads)
        return q

    def source(self, sources, mode):
        return self.source_nodal(sources) if mode == 0 else \
            self.source_consistent(sources)

    # -- stepping ----------------------------------------------------------
    def _problem(self, q):
        self._q_keep = None if q is None else np.ascontiguousarray(
            q, dtype=np.float64)
        return _Problem(self.N, self.E, _p(self.tets).value,
                        _p(self.A).value, _p(self.Vi).value,
                        _p(self.mat).value, _p(self.is_dir).value,
                        _p(self.T_dir).value,
                        None if self._q_keep is None else
                        _p(self._q_keep).value,
                        _p(self.csr_off).value, _p(self.csr_ec).value,
                        float(self.dt), self.n_threads,
                        None if self.tabs is None else _p(self.tabs).value)

    def step(self, T, q=None):
        """One step; returns (T_next, F, C) with F the assembled loads."""
        T = np.ascontiguousarray(T, dtype=np.float64)
        Tn = np.empty(self.N)
        F = np.empty(self.N)
        Cm = np.empty(self.N)
        Fe = np.empty(4 * self.E)
        prob = self._problem(q)
        lib().oracle_step(C.byref(prob), _p(T), _p(Tn), _p(F), _p(Cm), _p(Fe))
        return Tn, F, Cm

    def run(self, T, n_steps, q=None):
        """n_steps explicit steps from T (a copy is returned)."""
        T = np.array(T, dtype=np.float64, copy=True)
        prob = self._problem(q)
        rc = lib().oracle_run(C.byref(prob), int(n_steps), _p(T))
        if rc != 0:
            raise MemoryError("oracle_run failed")
        return T

    def run_schedule(self, T, n_steps, patterns, schedules, q=None, t0=0.0):
        """n_steps steps where step n (starting at t_n = t0 + n dt) uses the
        source q + sum_p a_p(t_n) Q_p (Algorithm 1 applies the external heat
        at every step); a copy of T is returned."""
        T = np.array(T, dtype=np.float64, copy=True)
        base = np.zeros(self.N) if q is None else np.asarray(q, dtype=np.float64)
        pats = [np.asarray(Q, dtype=np.float64) for Q in patterns]
        for n in range(int(n_steps)):
            t = t0 + n * self.dt
            qn = base.copy()
            for Q, (ts, am) in zip(pats, schedules):
                qn += schedule_amplitude(ts, am, t) * Q
            T = self.step(T, qn)[0]
        return T

    def initial(self, T0):
        T = np.full(self.N, float(T0))
        T[self.is_dir.astype(bool)] = self.T_dir[self.is_dir.astype(bool)]
        return T

    # -- critical step -----------------------------------------------------
    def geometry_lambda(self, method="auto"):
        from . import dense
        return dense.geometry_lambda(self, method=method)

    def dt_cr(self, method="auto"):
        from . import dense
        return dense.critical_dt(self, method=method)


def schedule_amplitude(times, amps, t):
    """Piecewise-linear amplitude through the points (times[k], amps[k]):
    amps[0] before the first time, amps[-1] from the last time on, and where
    a time repeats, the last point given at it holds from that time on."""
    if t < times[0]:
        return float(amps[0])
    k = 0
    while k + 1 < len(times) and times[k + 1] <= t:
        k += 1
    if k + 1 == len(times):
        return float(amps[-1])
    w = (t - times[k]) / (times[k + 1] - times[k])
    return float(amps[k] + w * (amps[k + 1] - amps[k]))


def flux_loads(xyz, faces, flux):
    """Nodal loads of a surface heat flux (Eq 4): triangle f with flux q_f
    [W/m^2] gives each of its nodes q_f |f| / 3, |f| = |(b - a) x (c - a)| / 2."""
    xyz = np.asarray(xyz, dtype=np.float64)
    faces = np.asarray(faces, dtype=np.int64).reshape(-1, 3)
    flux = np.asarray(flux, dtype=np.float64).reshape(-1)
    out = np.zeros(len(xyz))
    for f, (a, b, c) in enumerate(faces):
        area = 0.5 * np.linalg.norm(np.cross(xyz[b] - xyz[a], xyz[c] - xyz[a]))
        for v in (a, b, c):
            out[v] += flux[f] * area / 3.0
    return out


def quadrature_points():
    out = np.empty((256, 4))
    lib().oracle_quadrature_points(_p(out))
    return out


def build_model(scn, n_threads=0):
    """OracleModel for a synth Scenario (inputs only)."""
    return OracleModel(scn.xyz, scn.tets, scn.materials, scn.dir_nodes,
                       scn.dir_T, n_threads=n_threads)


def timed_run(model, T, n_steps, q=None):
    t0 = time.perf_counter()
    out = model.run(T, n_steps, q)
    return out, time.perf_counter() - t0
