"""Dense and sparse brute force for the FP64 oracle -- TEST INFRASTRUCTURE.

Everything here is derived independently of the C oracle's element routine:
element gradients come from inverting each element's 4x4 vertex matrix
[[1,1,1,1],[x],[y],[z]] (the gradients of the barycentric coordinates are
columns 1..3 of its inverse), volumes from its determinant.  With those the
global conduction matrix K(T) = sum_e k_e V_e grad N grad N^T (Eq 11-12, 15)
is assembled explicitly, which the element-level method avoids.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

M = {f: i for i, f in enumerate(("rho0", "c0", "k0", "drho_dT", "dc_dT",
                                 "dk_dT", "T_ref", "T_lo", "T_hi", "w_b",
                                 "c_b", "T_a", "Q_m"))}


def element_matrices(xyz, tets):
    """(A [E,4,4], vol [E]) from the inverse of each 4x4 vertex matrix."""
    X = xyz[tets]                                   # [E,4,3]
    Mv = np.ones((len(tets), 4, 4))
    Mv[:, 1:, :] = np.transpose(X, (0, 2, 1))       # rows: 1, x, y, z
    det = np.linalg.det(Mv)
    vol = np.abs(det) / 6.0
    inv = np.linalg.inv(Mv)                         # lambda = inv @ [1,x,y,z]
    G = inv[:, :, 1:]                               # [E,4(node),3] gradients
    A = vol[:, None, None] * np.einsum("eai,ebi->eab", G, G)
    return A, vol


def lumped_volume(n_nodes, tets, vol):
    Vi = np.zeros(n_nodes)
    np.add.at(Vi, tets.ravel(), np.repeat(vol / 4.0, 4))
    return Vi


def assemble(n_nodes, tets, Ae, scale=None, dense=True):
    """Global matrix sum_e scale_e A_e (dense ndarray or CSR)."""
    if scale is not None:
        Ae = Ae * scale[:, None, None]
    rows = np.repeat(tets, 4, axis=1).ravel()
    cols = np.tile(tets, (1, 4)).ravel()
    K = sp.coo_matrix((Ae.ravel(), (rows, cols)),
                      shape=(n_nodes, n_nodes)).tocsr()
    return K.toarray() if dense else K


def _clamp(T, m):
    return np.clip(T, m[M["T_lo"]], m[M["T_hi"]])


def k_of(T, m):
    return m[M["k0"]] + m[M["dk_dT"]] * (_clamp(T, m) - m[M["T_ref"]])


def rho_c_of(T, m):
    d = _clamp(T, m) - m[M["T_ref"]]
    return (m[M["rho0"]] + m[M["drho_dT"]] * d) * (m[M["c0"]] + m[M["dc_dT"]] * d)


class DenseModel:
    """Brute-force model: assembled K(T) every step (tiny meshes only)."""

    def __init__(self, xyz, tets, mat_vec, dir_nodes, dir_T, dt):
        self.xyz = np.asarray(xyz, dtype=np.float64)
        self.tets = np.asarray(tets, dtype=np.int64)
        self.m = np.asarray(mat_vec, dtype=np.float64)
        self.N = len(self.xyz)
        self.A, self.vol = element_matrices(self.xyz, self.tets)
        self.Vi = lumped_volume(self.N, self.tets, self.vol)
        self.D = np.zeros(self.N, dtype=bool)
        self.D[np.asarray(dir_nodes, dtype=np.int64)] = True
        self.TD = np.zeros(self.N)
        self.TD[np.asarray(dir_nodes, dtype=np.int64)] = dir_T
        self.dt = float(dt)

    def K_of_T(self, T):
        ke = k_of(T[self.tets], self.m).mean(axis=1)     # Eq 13
        return assemble(self.N, self.tets, self.A, ke)   # Eq 11-12

    def step(self, T, q=None):
        m = self.m
        K = self.K_of_T(T)
        wbcb = m[M["w_b"]] * m[M["c_b"]]
        Cd = rho_c_of(T, m) * self.Vi
        rhs = -(K @ T) - wbcb * self.Vi * T + wbcb * m[M["T_a"]] * self.Vi \
            + m[M["Q_m"]] * self.Vi
        if q is not None:
            rhs = rhs + q
        Tn = T + self.dt / Cd * rhs
        Tn[self.D] = self.TD[self.D]
        return Tn

    def run(self, T, n, q=None):
        T = np.array(T, dtype=np.float64)
        T[self.D] = self.TD[self.D]
        for _ in range(n):
            T = self.step(T, q)
        return T

    def expm_solution(self, T0, t, q=None):
        """Exact semi-discrete solution at time t (constant properties).

        Free nodes obey C_f dT_f/dt = -(K_ff + Kb_f) T_f - K_fD T_D + b_f.
        The affine system is solved with the exponential of an augmented
        matrix [[Ms, c],[0, 0]].
        """
        m = self.m
        K = self.K_of_T(np.full(self.N, m[M["T_ref"]]))
        wbcb = m[M["w_b"]] * m[M["c_b"]]
        Cd = rho_c_of(np.full(self.N, m[M["T_ref"]]), m) * self.Vi
        f = ~self.D
        Kff = K[np.ix_(f, f)] + np.diag(wbcb * self.Vi[f])
        b = wbcb * m[M["T_a"]] * self.Vi[f] + m[M["Q_m"]] * self.Vi[f] \
            - K[np.ix_(f, self.D)] @ self.TD[self.D]
        if q is not None:
            b = b + q[f]
        Ms = -Kff / Cd[f][:, None]
        c = b / Cd[f]
        n = Ms.shape[0]
        Aug = np.zeros((n + 1, n + 1))
        Aug[:n, :n] = Ms
        Aug[:n, n] = c
        E = sla.expm(Aug * t)
        T0 = np.asarray(T0, dtype=np.float64)
        out = np.array(T0, dtype=np.float64)
        out[f] = E[:n, :n] @ T0[f] + E[:n, n]
        out[self.D] = self.TD[self.D]
        return out


def geometry_lambda_from(n_nodes, tets, A, Vi, is_dir, method="auto"):
    """Largest eigenvalue of (sum_e A_e) v = lambda diag(V) v on free nodes."""
    free = ~np.asarray(is_dir, dtype=bool)
    K = assemble(n_nodes, np.asarray(tets, dtype=np.int64), A, dense=False)
    K = K[free][:, free]
    s = 1.0 / np.sqrt(Vi[free])
    B = sp.diags(s) @ K @ sp.diags(s)
    nf = B.shape[0]
    if method == "dense" or (method == "auto" and nf <= 4000):
        return float(np.linalg.eigvalsh(B.toarray())[-1])
    vals = spla.eigsh(B.tocsc(), k=1, which="LA", tol=1e-13,
                      return_eigenvectors=False, maxiter=20000, ncv=64)
    return float(vals[-1])


def table_value(T, table):
    """Linear interpolation in (temperatures, values), constant outside."""
    t, v = (np.asarray(a, dtype=np.float64) for a in table)
    return np.interp(T, t, v)


def prop_value(T, m, tables, name):
    """k, rho or c at T: the table when given, else the clamped linear law."""
    if tables and tables.get(name) is not None:
        return table_value(T, tables[name])
    d = _clamp(np.asarray(T, dtype=np.float64), m) - m[M["T_ref"]]
    p0, dp = {"k": ("k0", "dk_dT"), "rho": ("rho0", "drho_dT"), "c": ("c0", "dc_dT")}[name]
    return m[M[p0]] + m[M[dp]] * d


def material_window(m, tables=None):
    """(k_max, rhoc_min) over all temperatures.  Every property is piecewise
    linear, with breakpoints at its table points or its window ends; k peaks
    at a breakpoint, rho c (quadratic between consecutive breakpoints) at a
    breakpoint or at the vertex of that quadratic."""
    if tables:
        pts = []
        for name in ("k", "rho", "c"):
            if tables.get(name) is not None:
                pts += list(np.asarray(tables[name][0], dtype=np.float64))
            else:
                pts += [m[M["T_lo"]], m[M["T_hi"]]]
        pts = np.unique(np.array(pts))
        cand = list(pts)
        for a, b in zip(pts[:-1], pts[1:]):
            r = prop_value(np.array([a, b]), m, tables, "rho")
            c = prop_value(np.array([a, b]), m, tables, "c")
            sr, scc = (r[1] - r[0]) / (b - a), (c[1] - c[0]) / (b - a)
            if sr * scc != 0.0:
                x = a - (r[0] * scc + c[0] * sr) / (2.0 * sr * scc)
                if a < x < b:
                    cand.append(x)
        cand = np.array(cand)
        k = prop_value(cand, m, tables, "k")
        rc = prop_value(cand, m, tables, "rho") * prop_value(cand, m, tables, "c")
        return float(np.max(k)), float(np.min(rc))
    # clamped linear laws over [T_lo, T_hi]
    lo, hi = m[M["T_lo"]], m[M["T_hi"]]
    ts = [lo, hi]
    # rho(T) c(T) is quadratic in T; its vertex may lie inside the window
    a = m[M["drho_dT"]] * m[M["dc_dT"]]
    if a != 0.0:
        b = m[M["rho0"]] * m[M["dc_dT"]] + m[M["c0"]] * m[M["drho_dT"]]
        tv = m[M["T_ref"]] - b / (2 * a)
        if lo < tv < hi:
            ts.append(tv)
    ts = np.array(ts)
    return float(np.max(k_of(ts, m))), float(np.min(rho_c_of(ts, m)))


def critical_dt_from_lambda(lam_geo, m, tables=None):
    """Eq 9 with lambda_max bounded over the property window."""
    kmax, rcmin = material_window(m, tables)
    lam = lam_geo * kmax / rcmin + m[M["w_b"]] * m[M["c_b"]] / rcmin
    return 2.0 / lam, lam


def geometry_lambda(model, method="auto"):
    A, vol = element_matrices(model.xyz, model.tets.astype(np.int64))
    Vi = lumped_volume(model.N, model.tets.astype(np.int64), vol)
    return geometry_lambda_from(model.N, model.tets, A, Vi, model.is_dir,
                                method)


def critical_dt(model, method="auto"):
    lam = geometry_lambda(model, method)
    return critical_dt_from_lambda(lam, model.mat, getattr(model, "tables", None))[0]
