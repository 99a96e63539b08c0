"""Closed-form solutions used to pin the oracle -- TEST INFRASTRUCTURE.

All formulas are written from the mathematics of the Pennes equation (Eq 1)
and of the explicit Euler step (Eq 6), not from the oracle's code.
"""
from __future__ import annotations

import numpy as np


def slab_discrete(theta0, src, alpha, m, h, dt, n_steps, rho_c):
    """Explicit-Euler solution of the 7-point / 3-point slab scheme.

    1-D grid x_j = j h, j = 0..M, theta_0 = theta_M = 0, with theta = T - T_a
    (= T - T_Gamma).  Interior nodes obey
        theta_j^{k+1} = theta_j^k + dt [alpha (theta_{j-1} - 2 theta_j
                        + theta_{j+1}) / h^2 - m theta_j + s_j / rho_c]
    The sine vectors sin(n pi j / M) diagonalise it with
        mu_n = 4 alpha / h^2 sin^2(n pi / (2 M)) + m,
    so each mode evolves as g^k b_n + (1 - g^k) s_n / (rho_c mu_n),
    g = 1 - dt mu_n.  theta0 and src hold the M-1 interior values.
    """
    theta0 = np.asarray(theta0, dtype=np.float64)
    src = np.asarray(src, dtype=np.float64)
    Mc = len(theta0) + 1
    j = np.arange(1, Mc)
    n = np.arange(1, Mc)
    S = np.sin(np.pi * np.outer(n, j) / Mc)          # S S^T = (M/2) I
    b = S @ theta0 * (2.0 / Mc)
    s = S @ src * (2.0 / Mc)
    mu = 4.0 * alpha / h**2 * np.sin(n * np.pi / (2 * Mc)) ** 2 + m
    g = 1.0 - dt * mu
    coef = g**n_steps * b + (1.0 - g**n_steps) * s / (rho_c * mu)
    return coef @ S


def slab_series(x, t, L, alpha, m, rho_c, theta0_fn, src_fn, n_terms=400,
                n_quad=4000):
    """Continuous Pennes slab: theta(0)=theta(L)=0, constant properties.

    rho_c theta_t = k theta_xx - w_b c_b theta + Q(x), alpha = k / rho_c,
    m = w_b c_b / rho_c.  With sine coefficients b_n of theta(x,0) and q_n of
    Q(x), lambda_n = alpha (n pi / L)^2 + m:
        theta = sum_n [b_n e^{-lambda_n t}
                       + q_n / (rho_c lambda_n) (1 - e^{-lambda_n t})]
                      sin(n pi x / L)
    Coefficients come from a midpoint rule with n_quad points.
    """
    xq = (np.arange(n_quad) + 0.5) * L / n_quad
    n = np.arange(1, n_terms + 1)
    Sq = np.sin(np.outer(n, xq) * np.pi / L)
    b = Sq @ theta0_fn(xq) * (2.0 / n_quad)
    q = Sq @ src_fn(xq) * (2.0 / n_quad)
    lam = alpha * (n * np.pi / L) ** 2 + m
    e = np.exp(-lam * t)
    coef = b * e + q / (rho_c * lam) * (1.0 - e)
    return np.sin(np.outer(np.asarray(x), n) * np.pi / L) @ coef


def uniform_perfusion(theta0, dt, m, n):
    """Uniform field, no conduction: theta^n = theta0 (1 - dt m)^n."""
    return theta0 * (1.0 - dt * m) ** n


def uniform_metabolic_ti(T0, dt, Qm, rho_c, n):
    """Uniform field, constant properties, metabolic heat only."""
    return T0 + n * dt * Qm / rho_c


def uniform_metabolic_td(T0, dt, Qm, rho_c_fn, n):
    """Scalar explicit recurrence T <- T + dt Qm / (rho(T) c(T))."""
    T = float(T0)
    for _ in range(n):
        T = T + dt * Qm / rho_c_fn(T)
    return T


def kuhn_cube_lambda(n_cubes, h):
    """Largest eigenvalue of -Laplacian (7-point) on an n^3-cube grid with
    Dirichlet boundary: 12 / h^2 sin^2((n-1) pi / (2n))."""
    return 12.0 / h**2 * np.sin((n_cubes - 1) * np.pi / (2 * n_cubes)) ** 2


def kirchhoff_slab(x, L, T_left, T_right, k0, beta, T_r):
    """Steady 1-D conduction with k = k0 (1 + beta (T - T_r)).

    U(T) = k0 [(T - T_r) + beta (T - T_r)^2 / 2] satisfies U'' = 0, so U is
    linear in x between its boundary values; invert the quadratic for T.
    """
    def U(T):
        d = T - T_r
        return k0 * (d + beta * d * d / 2.0)
    u = U(T_left) + (U(T_right) - U(T_left)) * np.asarray(x) / L
    return T_r + (-1.0 + np.sqrt(1.0 + 2.0 * beta * u / k0)) / beta


def gaussian_total_power(Q0, sigma):
    """Integral of Q0 exp(-r^2 / (2 sigma^2)) over R^3."""
    return Q0 * (2.0 * np.pi) ** 1.5 * sigma**3


def kirchhoff_slab_table(x, L, T_left, T_right, Tk, kv):
    """Steady 1-D conduction with k(T) piecewise linear through (Tk, kv),
    constant outside.  U(T) = integral of k from Tk[0] is piecewise
    quadratic; U'' = 0 makes U linear in x between its boundary values, and
    each U is inverted on the piece where it falls."""
    Tk = np.asarray(Tk, dtype=np.float64)
    kv = np.asarray(kv, dtype=np.float64)
    # U at the table points (exact for piecewise-linear k)
    Uk = np.concatenate([[0.0], np.cumsum(0.5 * (kv[1:] + kv[:-1]) * np.diff(Tk))])

    def U(T):
        if T <= Tk[0]:
            return kv[0] * (T - Tk[0])
        if T >= Tk[-1]:
            return Uk[-1] + kv[-1] * (T - Tk[-1])
        j = np.searchsorted(Tk, T, side="right") - 1
        s = (kv[j + 1] - kv[j]) / (Tk[j + 1] - Tk[j])
        d = T - Tk[j]
        return Uk[j] + kv[j] * d + 0.5 * s * d * d

    def U_inv(u):
        if u <= 0.0:
            return Tk[0] + u / kv[0]
        if u >= Uk[-1]:
            return Tk[-1] + (u - Uk[-1]) / kv[-1]
        j = np.searchsorted(Uk, u, side="right") - 1
        s = (kv[j + 1] - kv[j]) / (Tk[j + 1] - Tk[j])
        r = u - Uk[j]
        if s == 0.0:
            return Tk[j] + r / kv[j]
        return Tk[j] + (-kv[j] + np.sqrt(kv[j] ** 2 + 2.0 * s * r)) / s

    ua, ub = U(T_left), U(T_right)
    return np.array([U_inv(ua + (ub - ua) * xi / L) for xi in np.asarray(x)])


def hex_box_lambda(nx, ny, nz, h):
    """Largest eigenvalue of (sum_e A_e) v = lambda diag(V) v for one-point
    hexahedra on a regular box of nx*ny*nz cubes of edge h, all surface nodes
    fixed.

    At the element centre the gradient of a nodal field is, in each
    direction, the difference along that direction averaged over the four
    parallel edges.  So the conduction form is h^3 sum_d (D_d^T D_d) (x)
    (A^T A) (x) (A^T A) over the other two directions, with D the 1-D
    difference (T_{j+1} - T_j)/h and A the 1-D average (T_j + T_{j+1})/2; the
    lumped capacity is h^3 per node.  With zero boundary values the sine
    vectors sin(p pi j / n) diagonalise D^T D (eigenvalue 4/h^2 sin^2(p pi/2n))
    and A^T A (eigenvalue cos^2(p pi / 2n)), so the eigenvalues are
        4/h^2 (s_x c_y c_z + c_x s_y c_z + c_x c_y s_z)
    over all modes (p, q, r), 1 <= p < nx, 1 <= q < ny, 1 <= r < nz.
    """
    def sc(n):
        th = np.arange(1, n) * np.pi / (2.0 * n)
        return np.sin(th) ** 2, np.cos(th) ** 2
    sx, cx = sc(nx)
    sy, cy = sc(ny)
    sz, cz = sc(nz)
    lam = (sx[:, None, None] * cy[None, :, None] * cz[None, None, :]
           + cx[:, None, None] * sy[None, :, None] * cz[None, None, :]
           + cx[:, None, None] * cy[None, :, None] * sz[None, None, :])
    return 4.0 / h**2 * float(lam.max())
