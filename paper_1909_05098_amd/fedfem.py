"""Thin ctypes binding of libfedfem.so (the gfx950 FED-FEM library).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  The binding raises if the shared library is missing; there is
no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfedfem.so")

FP64 = 0
FP32C = 1
SOURCE_NODAL = 0
SOURCE_CONSISTENT = 1
DOSE_OFF = 0
DOSE_CEM43 = 1
DOSE_ARRHENIUS = 2
TUNE_BATCH = 1

OK = 0
E_INVALID = -1
E_DEGENERATE = -2
E_NOT_PRECOMPUTED = -3
E_UNSTABLE = -4
E_DIVERGED = -5
E_HIP = -6
E_NOMEM = -7
E_STATE = -8
E_TOO_LARGE = -9

MAT_FIELDS = ("rho0", "c0", "k0", "drho_dT", "dc_dT", "dk_dT", "T_ref", "T_lo",
              "T_hi", "w_b", "c_b", "T_a", "Q_m")


class Mesh(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("xyz", C.c_void_p),
                ("n_tets", C.c_int64), ("tets", C.c_void_p)]


class Materials(C.Structure):
    _fields_ = [(f, C.c_double) for f in MAT_FIELDS] + [("precision", C.c_int32)]


class BC(C.Structure):
    _fields_ = [("T0", C.c_double), ("n_dir", C.c_int64),
                ("dir_nodes", C.c_void_p), ("dir_T", C.c_void_p),
                ("dt", C.c_double)]


class Options(C.Structure):
    _fields_ = [("reorder", C.c_int32), ("tile_elems", C.c_int32),
                ("threads", C.c_int32), ("max_tile_nodes", C.c_int32),
                ("xcd", C.c_int32), ("reserved", C.c_int32 * 3)]


class Info(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("n_tets", C.c_int64),
                ("n_dirichlet", C.c_int64), ("n_tiles", C.c_int64),
                ("n_partials", C.c_int64), ("max_tile_nodes", C.c_int64),
                ("precision", C.c_int32), ("tile_elems", C.c_int32),
                ("threads", C.c_int32), ("reorder", C.c_int32),
                ("device_bytes", C.c_int64), ("lambda_geometry", C.c_double),
                ("lanczos_iterations", C.c_int32),
                ("max_tile_valence", C.c_int32), ("fixed_point_shift", C.c_int32),
                ("n_single_tile_nodes", C.c_int32), ("reserved", C.c_int32 * 4)]


class FedFemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


_lib = None

# name -> (restype, argtypes)
_P = C.c_void_p
_SIGS = {
    "fedfem_create": (C.c_int, [_P, _P, _P, _P]),
    "fedfem_create_hex": (C.c_int, [_P, _P, _P, _P]),
    "fedfem_set_options": (C.c_int, [_P, _P]),
    "fedfem_precompute": (C.c_int, [_P]),
    "fedfem_precompute_many": (C.c_int, [_P, C.c_int32, C.c_int32, _P]),
    "fedfem_release_cached_memory": (C.c_size_t, []),
    "fedfem_set_schedule": (C.c_int, [_P, C.c_int32, _P, _P, _P, _P]),
    "fedfem_set_property_tables": (C.c_int, [_P, C.c_int32, _P, _P, C.c_int32, _P, _P,
                                             C.c_int32, _P, _P]),
    "fedfem_flux_loads": (C.c_int, [_P, C.c_int64, _P, _P, _P]),
    "fedfem_flux_loads_quad": (C.c_int, [_P, C.c_int64, _P, _P, _P]),
    "fedfem_set_dose": (C.c_int, [_P, C.c_int32, C.c_double, C.c_double]),
    "fedfem_read_dose": (C.c_int, [_P, _P]),
    "fedfem_step": (C.c_int, [_P, C.c_int64, _P]),
    "fedfem_step_static": (C.c_int, [_P, C.c_int64, _P]),
    "fedfem_prepare": (C.c_int, [_P, C.c_int64]),
    "fedfem_set_source": (C.c_int, [_P, _P]),
    "fedfem_set_gaussian_sources": (C.c_int, [_P, C.c_int32, _P, C.c_int32]),
    "fedfem_read_source": (C.c_int, [_P, _P]),
    "fedfem_read_T": (C.c_int, [_P, _P]),
    "fedfem_read_T_device": (C.c_int, [_P, _P]),
    "fedfem_get_dt": (C.c_int, [_P, _P, _P]),
    "fedfem_get_time": (C.c_int, [_P, _P, _P]),
    "fedfem_set_dt": (C.c_int, [_P, C.c_double]),
    "fedfem_set_stream": (C.c_int, [_P, _P]),
    "fedfem_state_bytes": (C.c_int, [_P, _P]),
    "fedfem_read_state": (C.c_int, [_P, _P, _P, _P]),
    "fedfem_write_state": (C.c_int, [_P, _P, C.c_double, C.c_int64]),
    "fedfem_get_info": (C.c_int, [_P, _P]),
    "fedfem_autotune": (C.c_int, [_P, C.c_char_p, C.c_int32, _P]),
    "fedfem_time_kernels": (C.c_int, [_P, C.c_int64, _P, _P]),
    "fedfem_destroy": (C.c_int, [_P]),
    "fedfem_strerror": (C.c_char_p, [C.c_int]),
    "fedfem_last_error": (C.c_int, [_P, C.c_char_p, C.c_size_t]),
    "fedfem_batch_create": (C.c_int, [_P, C.c_int32, _P]),
    "fedfem_batch_run": (C.c_int, [_P, _P, _P]),
    "fedfem_batch_last_ms": (C.c_int, [_P, _P]),
    "fedfem_batch_destroy": (C.c_int, [_P]),
}


def load(path=LIB_PATH):
    """Load libfedfem.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise FileNotFoundError(
                f"{path} is missing: build it with __graft_entry__.build() "
                "(there is no CPU fallback)")
        L = C.CDLL(path)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return sorted(_SIGS)


def _ptr(a):
    return None if a is None else C.c_void_p(a.ctypes.data)


class Handle:
    """One scenario: mesh (tetrahedra, or eight-node hexahedra when `tets` has
    8 columns), materials, boundary conditions, device state."""

    def __init__(self, xyz, tets, materials, T0=37.0, dir_nodes=(), dir_T=(),
                 dt=-0.9, precision=FP32C, reorder=True, tile_elems=0,
                 threads=0, max_tile_nodes=0, xcd=False):
        L = load()
        self._L = L
        self._h = C.c_void_p()
        self.xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        self.tets = np.ascontiguousarray(tets, dtype=np.int32)
        dn = np.ascontiguousarray(dir_nodes, dtype=np.int32)
        dT = np.ascontiguousarray(np.broadcast_to(np.asarray(dir_T, np.float64),
                                                  dn.shape))
        self.N = len(self.xyz)
        self.E = len(self.tets)
        # (E, 4) tetrahedra or (E, 8) hexahedra (corner order of fedfem_mesh_hex)
        self.hex = self.tets.ndim == 2 and self.tets.shape[1] == 8
        mesh = Mesh(self.N, _ptr(self.xyz), self.E, _ptr(self.tets))
        if isinstance(materials, dict):
            vals = [float(materials[f]) for f in MAT_FIELDS]
        else:
            vals = [float(getattr(materials, f)) for f in MAT_FIELDS]
        mat = Materials(*vals, int(precision))
        bc = BC(float(T0), len(dn), _ptr(dn) if len(dn) else None,
                _ptr(dT) if len(dn) else None, float(dt))
        create = L.fedfem_create_hex if self.hex else L.fedfem_create
        self._check(create(C.byref(mesh), C.byref(mat), C.byref(bc), C.byref(self._h)),
                    "fedfem_create_hex" if self.hex else "fedfem_create")
        self.precision = int(precision)
        opt = Options(1 if reorder else 0, int(tile_elems), int(threads),
                      int(max_tile_nodes), 1 if xcd else 0)
        self._check(L.fedfem_set_options(self._h, C.byref(opt)),
                    "fedfem_set_options")

    # -- errors ---------------------------------------------------------------
    def last_error(self):
        buf = C.create_string_buffer(512)
        if self._h:
            self._L.fedfem_last_error(self._h, buf, 512)
        return buf.value.decode()

    def _check(self, rc, what):
        if rc != OK:
            msg = self._L.fedfem_strerror(rc).decode()
            detail = self.last_error() if self._h else ""
            raise FedFemError(rc, f"{what}: {msg}" + (f": {detail}" if detail else ""))

    # -- lifecycle ------------------------------------------------------------
    def precompute(self):
        self._check(self._L.fedfem_precompute(self._h), "fedfem_precompute")
        return self

    def close(self):
        if self._h:
            self._L.fedfem_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- stepping -------------------------------------------------------------
    def _source(self, source):
        if source is None:
            return None
        src = np.ascontiguousarray(source, np.float64).reshape(-1)
        if len(src) != self.N:
            raise ValueError(f"source has {len(src)} entries, the mesh {self.N} nodes")
        return src

    def step(self, n_steps, source=None):
        src = self._source(source)
        self._check(self._L.fedfem_step(self._h, int(n_steps), _ptr(src)),
                    "fedfem_step")

    def step_static(self, n_steps, source=None):
        """fedfem_step without allocation (the library's fixed scratch)."""
        src = self._source(source)
        self._check(self._L.fedfem_step_static(self._h, int(n_steps), _ptr(src)),
                    "fedfem_step_static")

    def prepare(self, n_steps):
        self._check(self._L.fedfem_prepare(self._h, int(n_steps)), "fedfem_prepare")

    def set_source(self, source):
        src = self._source(source)
        self._check(self._L.fedfem_set_source(self._h, _ptr(src)),
                    "fedfem_set_source")

    def set_gaussian_sources(self, params, mode=SOURCE_CONSISTENT):
        p = np.ascontiguousarray(params, dtype=np.float64).reshape(-1, 5)
        self._check(self._L.fedfem_set_gaussian_sources(self._h, len(p), _ptr(p),
                                                        int(mode)),
                    "fedfem_set_gaussian_sources")

    def set_property_tables(self, tables):
        """Tables {"k" | "rho" | "c": (T, values)} replacing the linear laws
        (before precompute)."""
        args = []
        keep = []
        for name in ("k", "rho", "c"):
            tab = (tables or {}).get(name)
            if tab is None:
                args += [0, None, None]
                continue
            T = np.ascontiguousarray(tab[0], dtype=np.float64)
            V = np.ascontiguousarray(tab[1], dtype=np.float64)
            keep += [T, V]
            args += [len(T), _ptr(T), _ptr(V)]
        self._check(self._L.fedfem_set_property_tables(self._h, *args),
                    "fedfem_set_property_tables")

    def set_schedule(self, patterns, schedules):
        """Scheduled source patterns: patterns [P, N] (W, caller order) and,
        per pattern, (times, amplitudes) of its piecewise-linear amplitude.
        An empty list removes the schedule."""
        P = len(schedules)
        if P == 0:
            self._check(self._L.fedfem_set_schedule(self._h, 0, None, None, None, None),
                        "fedfem_set_schedule")
            return
        pat = np.ascontiguousarray(patterns, dtype=np.float64).reshape(P, -1)
        npts = np.array([len(t) for t, _ in schedules], dtype=np.int32)
        ts = np.ascontiguousarray(np.concatenate([np.asarray(t, float) for t, _ in schedules]))
        am = np.ascontiguousarray(np.concatenate([np.asarray(a, float) for _, a in schedules]))
        self._check(self._L.fedfem_set_schedule(self._h, P, _ptr(pat), _ptr(npts), _ptr(ts),
                                                _ptr(am)), "fedfem_set_schedule")

    def flux_loads(self, faces, flux):
        """Nodal loads [W] of surface flux `flux` [W/m^2] on triangles (3
        columns) or, on a hexahedral mesh, bilinear quadrilaterals (4)."""
        f = np.ascontiguousarray(faces, dtype=np.int32)
        if f.ndim != 2 or f.shape[1] not in (3, 4):
            raise ValueError("faces must be a 2-D array with 3 (triangles) or 4 "
                             f"(quadrilaterals) columns, got shape {f.shape}")
        nv = f.shape[1]
        q = np.ascontiguousarray(flux, dtype=np.float64).reshape(-1)
        if len(q) != len(f):
            raise ValueError(f"flux has {len(q)} entries for {len(f)} faces")
        out = np.empty(len(self.xyz))
        name = "fedfem_flux_loads_quad" if nv == 4 else "fedfem_flux_loads"
        self._check(getattr(self._L, name)(self._h, len(f), _ptr(f), _ptr(q), _ptr(out)), name)
        return out

    def set_dose(self, model, A=0.0, Ea=0.0):
        """Start (from zero) or stop the nodal thermal dose: DOSE_CEM43, or
        DOSE_ARRHENIUS with frequency factor A [1/s] and activation energy
        Ea [J/mol]."""
        self._check(self._L.fedfem_set_dose(self._h, int(model), float(A), float(Ea)),
                    "fedfem_set_dose")

    def read_dose(self):
        out = np.empty(self.N)
        self._check(self._L.fedfem_read_dose(self._h, _ptr(out)), "fedfem_read_dose")
        return out

    def read_source(self):
        out = np.empty(self.N)
        self._check(self._L.fedfem_read_source(self._h, _ptr(out)),
                    "fedfem_read_source")
        return out

    def read_T(self):
        out = np.empty(self.N)
        self._check(self._L.fedfem_read_T(self._h, _ptr(out)), "fedfem_read_T")
        return out

    def read_T_device(self, tensor):
        """Write T into a contiguous float64 device tensor of length N."""
        assert tensor.dtype.itemsize == 8 and tensor.numel() == self.N
        self._check(self._L.fedfem_read_T_device(self._h,
                                                 C.c_void_p(tensor.data_ptr())),
                    "fedfem_read_T_device")

    def dt(self):
        dt = C.c_double()
        dtc = C.c_double()
        self._check(self._L.fedfem_get_dt(self._h, C.byref(dt), C.byref(dtc)),
                    "fedfem_get_dt")
        return dt.value, dtc.value

    def set_dt(self, dt):
        self._check(self._L.fedfem_set_dt(self._h, float(dt)), "fedfem_set_dt")

    def time(self):
        t = C.c_double()
        n = C.c_int64()
        self._check(self._L.fedfem_get_time(self._h, C.byref(t), C.byref(n)),
                    "fedfem_get_time")
        return t.value, n.value

    def set_stream(self, stream_ptr):
        self._check(self._L.fedfem_set_stream(self._h, C.c_void_p(stream_ptr)),
                    "fedfem_set_stream")

    def read_state(self):
        nb = C.c_size_t()
        self._check(self._L.fedfem_state_bytes(self._h, C.byref(nb)),
                    "fedfem_state_bytes")
        buf = np.empty(nb.value, dtype=np.uint8)
        t = C.c_double()
        n = C.c_int64()
        self._check(self._L.fedfem_read_state(self._h, _ptr(buf), C.byref(t),
                                              C.byref(n)), "fedfem_read_state")
        return buf, t.value, n.value

    def write_state(self, buf, t, steps):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        self._check(self._L.fedfem_write_state(self._h, _ptr(buf), float(t),
                                               int(steps)), "fedfem_write_state")

    def autotune(self, cache_path=None, for_batch=False):
        """Let the library time candidate layouts and keep the fastest."""
        o = Options()
        path = None if cache_path is None else os.fsencode(cache_path)
        self._check(self._L.fedfem_autotune(self._h, path, TUNE_BATCH if for_batch else 0,
                                            C.byref(o)), "fedfem_autotune")
        return {f: getattr(o, f) for f, _ in Options._fields_ if f != "reserved"}

    def info(self):
        inf = Info()
        self._check(self._L.fedfem_get_info(self._h, C.byref(inf)),
                    "fedfem_get_info")
        return {f: (getattr(inf, f) if f != "reserved" else None)
                for f, _ in Info._fields_ if f != "reserved"}

    def time_kernels(self, n_steps):
        a = C.c_double()
        b = C.c_double()
        self._check(self._L.fedfem_time_kernels(self._h, int(n_steps), C.byref(a),
                                                C.byref(b)), "fedfem_time_kernels")
        return a.value, b.value


def precompute_many(handles, threads=0):
    """fedfem_precompute on all handles, overlapped on host threads."""
    hs = list(handles)
    if not hs:
        return
    L = load()
    arr = (C.c_void_p * len(hs))(*[h._h.value for h in hs])
    rcs = np.zeros(len(hs), dtype=np.int32)
    rc = L.fedfem_precompute_many(arr, len(hs), int(threads), _ptr(rcs))
    if rc != OK:
        j = int(np.nonzero(rcs)[0][0]) if np.any(rcs) else -1
        msg = hs[j].last_error() if j >= 0 else ""
        raise FedFemError(rc, f"fedfem_precompute_many: handle {j}: {msg}")


def release_cached_memory():
    """Return the library's cached device blocks; gives the bytes released."""
    return int(load().fedfem_release_cached_memory())


class Batch:
    """Many precomputed handles advanced by one captured launch sequence."""

    def __init__(self, handles):
        L = load()
        self._L = L
        self.handles = list(handles)
        arr = (C.c_void_p * len(self.handles))(*[h._h.value for h in self.handles])
        self._b = C.c_void_p()
        rc = L.fedfem_batch_create(arr, len(self.handles), C.byref(self._b))
        if rc != OK:
            raise FedFemError(rc, "fedfem_batch_create: "
                              + L.fedfem_strerror(rc).decode())

    def run(self, n_steps, sources=None):
        """Advance scenario j by n_steps[j]; sources[j] (optional, nodal [W])
        replaces handle j's active source first."""
        n = np.ascontiguousarray(n_steps, dtype=np.int64)
        assert len(n) == len(self.handles)
        arr = None
        if sources is not None:
            assert len(sources) == len(self.handles)
            keep = [None if q is None else np.ascontiguousarray(q, dtype=np.float64)
                    for q in sources]
            arr = (C.c_void_p * len(keep))(*[None if q is None else q.ctypes.data
                                              for q in keep])
        rc = self._L.fedfem_batch_run(self._b, _ptr(n), arr)
        if rc != OK:
            raise FedFemError(rc, "fedfem_batch_run: "
                              + self._L.fedfem_strerror(rc).decode())

    def last_ms(self):
        ms = C.c_double()
        self._L.fedfem_batch_last_ms(self._b, C.byref(ms))
        return ms.value

    def close(self):
        if self._b:
            self._L.fedfem_batch_destroy(self._b)
            self._b = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
