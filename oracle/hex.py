"""FP64 CPU oracle for FED-FEM on eight-node reduced-integration hexahedra --
TEST INFRASTRUCTURE.

Only the tests may use this module; the product never imports it.  It is
plain NumPy, written from Sec 2.3.3 of the paper:

- Eq 14/16: the element matrix of the eight-node hexahedron with one
  integration point is A_e = 8 det(J) B^T B, with the Jacobian J and the
  temperature-gradient matrix B evaluated at the element centre (the weight
  8 is the volume of the parent cube [-1, 1]^3).  The absolute value of det J
  is used, so that the element's orientation does not matter (as for the
  tetrahedron's volume).
- Eq 13: k_e is the mean of k over the element's eight nodes.
- Eq 17, 11: F_e = k_e A_e T_e, gathered at the nodes in ascending element
  order.
- Lumping (Sec 2.3.4): each node receives an eighth of V_e = 8 |det J|.
- Eq 19 (with the sign reading S1 of the tetrahedral oracle): the explicit
  update with lumped capacity, perfusion and metabolic heat; Dirichlet nodes
  are held.

The paper is silent on hourglass (zero-energy) modes of the one-point rule;
this oracle, like the library, takes Eq 14 literally and adds no hourglass
control (the pins show the zero-energy mode on a regular grid).

Node order of a hexahedron: corners at natural coordinates
(-1,-1,-1), (1,-1,-1), (1,1,-1), (-1,1,-1), (-1,-1,1), (1,-1,1), (1,1,1),
(-1,1,1): the bottom face counter-clockwise, then the top face above it.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .dense import M, k_of, rho_c_of, critical_dt_from_lambda

# natural coordinates of the eight corners, in the node order above
NAT = np.array([[-1, -1, -1], [1, -1, -1], [1, 1, -1], [-1, 1, -1],
                [-1, -1, 1], [1, -1, 1], [1, 1, 1], [-1, 1, 1]], dtype=np.float64)


def element_matrices(xyz, hexes):
    """(A [E,8,8], V [E], grad [E,8,3]) of Eq 14/16 at the element centre.

    The shape functions are N_a = (1 + xi_a xi)(1 + eta_a eta)(1 + zeta_a zeta)/8,
    so at the centre dN_a/d(xi, eta, zeta) = (xi_a, eta_a, zeta_a) / 8.  With
    Jn[j, i] = dx_i / dxi_j = sum_a dN_a/dxi_j x_a,i the chain rule gives
    grad_x N_a = Jn^{-1} grad_xi N_a.
    """
    X = np.asarray(xyz, dtype=np.float64)[np.asarray(hexes, dtype=np.int64)]  # [E,8,3]
    dN = NAT / 8.0                                    # [8(a), 3(j)]
    Jn = np.einsum("aj,eai->eji", dN, X)              # [E, j, i]
    det = np.linalg.det(Jn)
    grad = np.linalg.solve(Jn, np.broadcast_to(dN.T, (len(X), 3, 8)))  # [E, i, a]
    grad = np.transpose(grad, (0, 2, 1))              # [E, a, i]
    V = 8.0 * np.abs(det)
    A = V[:, None, None] * np.einsum("eai,ebi->eab", grad, grad)
    return A, V, grad


def lumped_volume(n_nodes, hexes, V):
    """V_i = sum over the node's elements of V_e / 8 (Sec 2.3.4)."""
    Vi = np.zeros(n_nodes)
    np.add.at(Vi, np.asarray(hexes, dtype=np.int64).ravel(), np.repeat(V / 8.0, 8))
    return Vi


def assemble(n_nodes, hexes, Ae, scale=None):
    """Global sparse matrix sum_e scale_e A_e (only for the brute-force checks)."""
    hexes = np.asarray(hexes, dtype=np.int64)
    if scale is not None:
        Ae = Ae * scale[:, None, None]
    rows = np.repeat(hexes, 8, axis=1).ravel()
    cols = np.tile(hexes, (1, 8)).ravel()
    return sp.coo_matrix((Ae.ravel(), (rows, cols)), shape=(n_nodes, n_nodes)).tocsr()


def flux_loads_quad(xyz, faces, flux):
    """Nodal loads [W] of a surface flux q_f [W/m^2] on bilinear
    quadrilaterals (corners in order around the face): each corner a receives
    the integral of q_f N_a over the face, by the 2 x 2 Gauss-Legendre rule on
    the bilinear map (area element |x_s x x_t|; exact on planar
    parallelograms), summed in ascending face order."""
    X = np.asarray(xyz, dtype=np.float64)[np.asarray(faces, dtype=np.int64)]   # [F, 4, 3]
    st = np.array([[-1, -1], [1, -1], [1, 1], [-1, 1]], dtype=np.float64)
    g, w = np.polynomial.legendre.leggauss(2)
    acc = np.zeros((len(X), 4))
    for s_, ws in zip(g, w):
        for t_, wt in zip(g, w):
            N = (1 + st[:, 0] * s_) * (1 + st[:, 1] * t_) / 4.0
            dNs = st[:, 0] * (1 + st[:, 1] * t_) / 4.0
            dNt = st[:, 1] * (1 + st[:, 0] * s_) / 4.0
            xs = np.einsum("a,fai->fi", dNs, X)
            xt = np.einsum("a,fai->fi", dNt, X)
            dA = np.linalg.norm(np.cross(xs, xt), axis=1)
            acc += (ws * wt) * (np.asarray(flux, dtype=np.float64) * dA)[:, None] * N[None, :]
    out = np.zeros(len(np.asarray(xyz)))
    np.add.at(out, np.asarray(faces, dtype=np.int64).ravel(), acc.ravel())
    return out


class HexModel:
    """Element-level FED-FEM (Algorithm 1) on hexahedra, in FP64."""

    def __init__(self, xyz, hexes, mat_vec, dir_nodes=(), dir_T=(), dt=None):
        self.xyz = np.asarray(xyz, dtype=np.float64)
        self.hexes = np.asarray(hexes, dtype=np.int64)
        self.m = np.asarray(mat_vec, dtype=np.float64)
        self.N = len(self.xyz)
        self.A, self.V, self.grad = element_matrices(self.xyz, self.hexes)
        self.Vi = lumped_volume(self.N, self.hexes, self.V)
        self.is_dir = np.zeros(self.N, dtype=bool)
        self.is_dir[np.asarray(dir_nodes, dtype=np.int64)] = True
        self.T_dir = np.zeros(self.N)
        self.T_dir[np.asarray(dir_nodes, dtype=np.int64)] = np.asarray(dir_T, dtype=np.float64)
        self.dt = None if dt is None else float(dt)

    # -- precompute -------------------------------------------------------
    def geometry_lambda(self, method="auto"):
        """Largest eigenvalue of (sum_e A_e) v = lambda diag(V) v on the free
        nodes (the pencil of Eq 9 with k = rho c = 1, no perfusion)."""
        free = ~self.is_dir
        K = assemble(self.N, self.hexes, self.A)[free][:, free]
        s = 1.0 / np.sqrt(self.Vi[free])
        B = sp.diags(s) @ K @ sp.diags(s)
        if method == "dense" or (method == "auto" and B.shape[0] <= 4000):
            return float(np.linalg.eigvalsh(B.toarray())[-1])
        return float(spla.eigsh(B.tocsc(), k=1, which="LA", tol=1e-13, maxiter=20000,
                                ncv=64, return_eigenvectors=False)[-1])

    def dt_cr(self, method="auto"):
        return critical_dt_from_lambda(self.geometry_lambda(method), self.m)[0]

    def source_nodal(self, sources):
        """Q_i = sum over Gaussian sources of Q0 exp(-r^2 / (2 sigma^2)) V_i,
        sources given as rows (x, y, z, sigma, Q0)."""
        q = np.zeros(self.N)
        for x, y, z, s, Q0 in np.asarray(sources, dtype=np.float64).reshape(-1, 5):
            r2 = np.sum((self.xyz - np.array([x, y, z])) ** 2, axis=1)
            q += Q0 * np.exp(-r2 / (2.0 * s * s)) * self.Vi
        return q

    def source_consistent(self, sources, order=4):
        """Q_i = integral of the Gaussian density against N_i over the mesh,
        by the order^3 tensor Gauss-Legendre rule on each element's
        trilinear map (weights |det J(xi)|), sources given as rows
        (x, y, z, sigma, Q0).  An element is skipped for a source when its
        nearest point can lie no closer than 8 sigma to the centre (as for
        tetrahedra).  Corner loads are gathered in ascending element order."""
        g, w = np.polynomial.legendre.leggauss(order)
        X = self.xyz[self.hexes]                                  # [E, 8, 3]
        cen = X.mean(axis=1)
        rad = np.sqrt(np.max(np.sum((X - cen[:, None, :]) ** 2, axis=2), axis=1))
        acc = np.zeros((len(self.hexes), 8))
        src = np.asarray(sources, dtype=np.float64).reshape(-1, 5)
        for xi, wx in zip(g, w):
            for eta, wy in zip(g, w):
                for zeta, wz in zip(g, w):
                    q = np.array([xi, eta, zeta])
                    N = np.prod(1.0 + NAT * q, axis=1) / 8.0                 # [8]
                    dN = np.empty((8, 3))
                    for j in range(3):
                        other = [k for k in range(3) if k != j]
                        dN[:, j] = NAT[:, j] * np.prod(1.0 + NAT[:, other] * q[other],
                                                       axis=1) / 8.0
                    x = np.einsum("a,eai->ei", N, X)
                    Jn = np.einsum("aj,eai->eji", dN, X)
                    det = np.abs(np.linalg.det(Jn))
                    f = np.zeros(len(X))
                    for sx, sy, sz, sg, Q0 in src:
                        near = np.sqrt(np.sum((cen - [sx, sy, sz]) ** 2, axis=1)) - rad
                        r2 = np.sum((x - [sx, sy, sz]) ** 2, axis=1)
                        f += np.where(near > 8.0 * sg, 0.0, Q0 * np.exp(-r2 / (2.0 * sg * sg)))
                    acc += (wx * wy * wz) * (f * det)[:, None] * N[None, :]
        return np.bincount(self.hexes.ravel(), weights=acc.ravel(), minlength=self.N)

    # -- time steps -------------------------------------------------------
    def initial(self, T0):
        T = np.full(self.N, float(T0))
        T[self.is_dir] = self.T_dir[self.is_dir]
        return T

    def loads(self, T):
        """F_i (Eq 11, 13, 17): element loads gathered in element order."""
        ke = k_of(T[self.hexes], self.m).mean(axis=1)                 # Eq 13
        Fe = ke[:, None] * np.einsum("eab,eb->ea", self.A, T[self.hexes])  # Eq 17
        return np.bincount(self.hexes.ravel(), weights=Fe.ravel(), minlength=self.N)

    def step(self, T, q=None):
        m = self.m
        F = self.loads(T)
        qn = np.zeros(self.N) if q is None else q
        R = (qn - F) + m[M["Q_m"]] * self.Vi \
            + m[M["w_b"]] * m[M["c_b"]] * self.Vi * (m[M["T_a"]] - T)
        Tn = T + self.dt * R / (rho_c_of(T, m) * self.Vi)           # Eq 19
        Tn[self.is_dir] = self.T_dir[self.is_dir]
        return Tn

    def run(self, T, n_steps, q=None):
        T = np.array(T, dtype=np.float64)
        for _ in range(int(n_steps)):
            T = self.step(T, q)
        return T
