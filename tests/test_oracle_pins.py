"""Pins of the FP64 CPU oracle against what the paper and mathematics fix.

Each test states which passage of the paper (arXiv 1909.05098) it follows and
what kind of mistake in the oracle it would catch.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import closed_forms as cf
from oracle import dense
from synth import mesh, scenarios as sc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def jittered_box(nx, ny, nz, h, seed, jitter=0.2):
    xyz, tets = mesh.kuhn_box(nx, ny, nz, h)
    bnd = mesh.boundary_nodes_by_faces(len(xyz), tets)
    rng = np.random.default_rng(seed)
    mask = np.ones(len(xyz), bool)
    mask[bnd] = False
    xyz[mask] += rng.uniform(-jitter * h, jitter * h, (mask.sum(), 3))
    return xyz, tets, bnd


def ti_materials(**kw):
    base = dict(rho0=1060.0, c0=3600.0, k0=0.512, w_b=6.4, c_b=4180.0,
                T_a=37.0, Q_m=0.0)
    base.update(kw)
    return sc.Materials(**base)


# --------------------------------------------------------------------------
# Pin 1: uniform fields are invariant (zero row sums of A, Eq 16; perfusion
# vanishes at T_a, Eq 1).  Catches a non-zero-sum element matrix, a sign
# slip in the perfusion term, or a stray source.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("td", [False, True])
def test_uniform_field_invariant(td):
    xyz, tets, bnd = jittered_box(5, 4, 3, 1e-3, seed=1)
    mat = sc.td_materials() if td else ti_materials()
    m = oracle.OracleModel(xyz, tets, mat, bnd, np.full(len(bnd), 37.0))
    m.dt = 0.9 * m.dt_cr()
    T = m.run(m.initial(37.0), 1000)
    assert np.max(np.abs(T - 37.0)) <= 1e-12


# --------------------------------------------------------------------------
# Pin 2: node update terms on a uniform, adiabatic mesh (F = 0), mirroring
# the separate perfusion and metabolic verifications (Sec 3.1.3, 3.1.4).
# Catches a wrong C_i, K_b,i, Q_b,i or Q_m,i in Eq 19.
# --------------------------------------------------------------------------
def test_uniform_perfusion_recurrence():
    xyz, tets, _ = jittered_box(4, 3, 3, 1e-3, seed=2)
    mat = ti_materials(T_a=39.0, w_b=26.6, c_b=3617.0)
    m = oracle.OracleModel(xyz, tets, mat)
    m.dt = 0.01
    n = 3000
    T = m.run(np.full(m.N, 37.0), n)
    mrate = 26.6 * 3617.0 / (1060.0 * 3600.0)
    expect = 39.0 + cf.uniform_perfusion(37.0 - 39.0, 0.01, mrate, n)
    assert np.max(np.abs(T - expect)) <= 1e-12 * 39.0


def test_uniform_metabolic_ti_and_td():
    xyz, tets, _ = jittered_box(4, 3, 3, 1e-3, seed=3)
    ti = ti_materials(w_b=0.0, Q_m=33800.0)
    m = oracle.OracleModel(xyz, tets, ti)
    m.dt = 0.01
    T = m.run(np.full(m.N, 37.0), 2000)
    expect = cf.uniform_metabolic_ti(37.0, 0.01, 33800.0, 1060.0 * 3600.0, 2000)
    assert np.max(np.abs(T - expect)) <= 1e-12 * expect
    # paper's two-point table (Sec 3.1.6) with constant extension above
    # 65 C; the scalar recurrence interpolates the printed points directly
    g = json.load(open(os.path.join(GOLDEN, "paper_values.json")))
    tab = g["td_table_sec_3_1_6"]
    td = sc.paper_table_materials()
    td.Q_m = 2.0e7
    m2 = oracle.OracleModel(xyz, tets, td)
    m2.dt = 0.05
    n = 400

    def rho_c(T):
        return (np.interp(T, tab["T_points"], tab["rho"])
                * np.interp(T, tab["T_points"], tab["c"]))
    T2 = m2.run(np.full(m2.N, 37.0), n)
    expect2 = cf.uniform_metabolic_td(37.0, 0.05, 2.0e7, rho_c, n)
    assert expect2 > 65.0  # the run crosses the upper table point
    assert np.max(np.abs(T2 - expect2)) <= 1e-11 * expect2


# --------------------------------------------------------------------------
# Pin 3: linear patch test (Sec 3.1, standard patch tests): with constant k,
# no perfusion and no source, a linear field is the steady state, so interior
# loads vanish and T stays linear on a jittered mesh.  Catches wrong element
# gradients or volumes (Eq 15-16).
# --------------------------------------------------------------------------
def test_linear_patch():
    xyz, tets, bnd = jittered_box(6, 5, 4, 1e-3, seed=4)
    g = np.array([900.0, -400.0, 250.0])
    lin = 37.0 + xyz @ g
    mat = ti_materials(w_b=0.0)
    m = oracle.OracleModel(xyz, tets, mat, bnd, lin[bnd])
    m.dt = 0.9 * m.dt_cr()
    T1, F, _ = m.step(lin)
    interior = np.ones(m.N, bool)
    interior[bnd] = False
    assert np.max(np.abs(F[interior])) <= 1e-12 * np.max(np.abs(F))
    T = m.run(lin, 500)
    assert np.max(np.abs(T - lin)) <= 1e-10


# --------------------------------------------------------------------------
# Pin 4: global energy balance.  The element loads conserve heat
# (sum_i F_i = 0), and each step's stored heat equals dt times the heat
# supplied by sources, perfusion and the Dirichlet reaction.  Catches a
# dropped term in Eq 19 or a non-conservative assembly (Eq 11).
# --------------------------------------------------------------------------
def test_energy_balance_td():
    xyz, tets, bnd = jittered_box(6, 5, 4, 1e-3, seed=5)
    mat = sc.td_materials()
    mat.Q_m = 4000.0
    m = oracle.OracleModel(xyz, tets, mat, bnd, np.full(len(bnd), 37.0))
    m.dt = 0.9 * m.dt_cr()
    q = m.source_consistent([[3e-3, 2.5e-3, 2e-3, 1e-3, 5e7]])
    D = m.is_dir.astype(bool)
    T = m.initial(37.0)
    wbcb = mat.w_b * mat.c_b
    # bound on the size of the individual terms k_e A_ab T_b
    term_scale = 0.6 * np.abs(m.A).sum()
    for _ in range(60):
        Tn, F, Cm = m.step(T, q)
        assert abs(F.sum()) <= 1e-13 * term_scale * np.abs(T).max()
        stored = np.sum(Cm[~D] * (Tn[~D] - T[~D]))
        supplied = m.dt * (np.sum(q[~D] + mat.Q_m * m.Vi[~D]
                                  + wbcb * m.Vi[~D] * (mat.T_a - T[~D]))
                           + np.sum(F[D]))
        scale = m.dt * (np.abs(q).sum() + np.abs(F).sum())
        assert abs(stored - supplied) <= 1e-12 * scale
        T = Tn
    assert T.max() > 37.5


# --------------------------------------------------------------------------
# Pin 5: 1-D slab against the exact discrete sine-mode solution and, with
# refinement, the continuous Pennes series (Eq 1).  Sign-sensitive: the
# anti-diffusive reading of Eq 19 diverges.  Conduction, perfusion, source
# and time stepping all enter.
# --------------------------------------------------------------------------
def slab_setup(M, L, extra_dt=0.5):
    h = L / M
    xyz, tets = mesh.kuhn_box(M, 2, 2, h)
    x = xyz[:, 0]
    dn = np.nonzero((np.abs(x) < 1e-12 * L) | (np.abs(x - L) < 1e-12 * L))[0]
    mat = ti_materials(T_a=37.0)
    m = oracle.OracleModel(xyz, tets, mat, dn, np.full(len(dn), 37.0))
    rho_c = 1060.0 * 3600.0
    alpha = 0.512 / rho_c
    mrate = 6.4 * 4180.0 / rho_c
    # 3-D stability limit of the 7-point scheme: dt < 2 / (12 alpha/h^2 + m)
    m.dt = extra_dt * 2.0 / (12.0 * alpha / h**2 + mrate)
    return m, x, h, alpha, mrate, rho_c


def test_slab_discrete_closed_form():
    L = 12e-3
    m, x, h, alpha, mrate, rho_c = slab_setup(12, L)
    theta0 = 5.0 * np.sin(np.pi * x / L) + 2.0 * np.sin(3 * np.pi * x / L)
    src_density = 3e5 * (x / L) * (1 - x / L)
    T0 = 37.0 + theta0
    q = src_density * m.Vi
    n = 400
    T = m.run(T0, n, q)
    xg = np.arange(1, 12) * h
    th0 = 5.0 * np.sin(np.pi * xg / L) + 2.0 * np.sin(3 * np.pi * xg / L)
    sg = 3e5 * (xg / L) * (1 - xg / L)
    expect = cf.slab_discrete(th0, sg, alpha, mrate, h, m.dt, n, rho_c)
    j = np.rint(x / h).astype(int)
    inner = (j > 0) & (j < 12)
    assert np.max(np.abs(T[inner] - 37.0 - expect[j[inner] - 1])) <= 1e-11


def test_slab_continuous_second_order():
    L = 12e-3
    t_end = 40.0
    errs = []
    hs = []
    for M in (6, 12, 24):
        m, x, h, alpha, mrate, rho_c = slab_setup(M, L, extra_dt=0.5)
        # dt proportional to h^2 and landing on t_end
        n = int(np.ceil(t_end / m.dt))
        m.dt = t_end / n
        def th0(z):
            return 5.0 * np.sin(np.pi * z / L) + 3.0 * np.sin(2 * np.pi * z / L)

        def src(z):
            return 2e5 * np.ones_like(z)
        q = src(x) * m.Vi
        T = m.run(37.0 + th0(x), n, q)
        ex = cf.slab_series(x, t_end, L, alpha, mrate, rho_c, th0, src,
                            n_terms=600, n_quad=20000)
        errs.append(np.max(np.abs(T - 37.0 - ex)))
        hs.append(h)
    orders = np.log(np.array(errs[:-1]) / np.array(errs[1:])) / np.log(2.0)
    assert np.all(np.abs(orders - 2.0) <= 0.2), (errs, orders)


# --------------------------------------------------------------------------
# Pin 6: the 1 cm cube case.  On the Kuhn lattice, linear tetrahedra with
# lumped capacity reduce to the 7-point finite-difference FTCS scheme, and
# the largest eigenvalue has a closed form (Eq 9).  Catches any slip in
# element matrices, lumping, perfusion, source or step.
# --------------------------------------------------------------------------
def test_config1_equals_7point_fd_and_lambda():
    s = sc.config1()
    m = oracle.build_model(s)
    lam = m.geometry_lambda(method="dense")
    assert abs(lam / cf.kuhn_cube_lambda(10, 1e-3) - 1.0) <= 1e-12
    dtcr, _ = dense.critical_dt_from_lambda(lam, m.mat)
    n, dt = sc.steps_for(300.0, dtcr)
    assert n == 263
    m.dt = dt
    q = m.source_nodal(s.sources)
    T = m.run(m.initial(37.0), n, q)
    h = 1e-3
    rho_c = 1060.0 * 3600.0
    alpha = 0.512 / rho_c
    mrate = 6.4 * 4180.0 / rho_c
    G = np.full((11, 11, 11), 37.0)
    # nodal-sampled source density at the lattice nodes (independent of Vi)
    zz, yy, xx = np.meshgrid(*(np.arange(11) * h,) * 3, indexing="ij")
    r2 = (xx - 5e-3) ** 2 + (yy - 5e-3) ** 2 + (zz - 5e-3) ** 2
    Qd = 5e6 * np.exp(-r2 / (2 * 1.5e-3 ** 2))
    for _ in range(n):
        lap = np.zeros_like(G)
        c = G[1:-1, 1:-1, 1:-1]
        lap[1:-1, 1:-1, 1:-1] = (G[2:, 1:-1, 1:-1] + G[:-2, 1:-1, 1:-1]
                                 + G[1:-1, 2:, 1:-1] + G[1:-1, :-2, 1:-1]
                                 + G[1:-1, 1:-1, 2:] + G[1:-1, 1:-1, :-2]
                                 - 6 * c) / h**2
        Gn = G + dt * (alpha * lap + mrate * (37.0 - G) + Qd / rho_c)
        Gn[[0, -1], :, :] = 37.0
        Gn[:, [0, -1], :] = 37.0
        Gn[:, :, [0, -1]] = 37.0
        G = Gn
    assert np.max(np.abs(G.ravel() - T)) <= 1e-12
    # full cube symmetry of the solution (48 symmetries generated by axis
    # swaps and reflections)
    Tg = T.reshape(11, 11, 11)
    for op in (lambda a: a.transpose(1, 0, 2), lambda a: a.transpose(0, 2, 1),
               lambda a: a[::-1], lambda a: a[:, ::-1], lambda a: a[:, :, ::-1]):
        assert np.max(np.abs(op(Tg) - Tg)) <= 1e-12
    assert 50.0 < Tg[5, 5, 5] < 51.0


# --------------------------------------------------------------------------
# Pin 7: the element-level step equals the assembled one (Eq 10-11), with
# element matrices derived independently; and the time step converges at
# first order to the exact semi-discrete solution (Eq 6).
# --------------------------------------------------------------------------
def test_element_level_equals_dense_td():
    xyz, tets, bnd = jittered_box(4, 4, 3, 1e-3, seed=7)
    mat = sc.td_materials()
    m = oracle.OracleModel(xyz, tets, mat, bnd, np.full(len(bnd), 37.0))
    m.dt = 0.9 * m.dt_cr()
    q = m.source_consistent([[2e-3, 2e-3, 1.5e-3, 0.8e-3, 3e8]])
    dm = dense.DenseModel(xyz, tets, m.mat, bnd, np.full(len(bnd), 37.0),
                          m.dt)
    T0 = m.initial(37.0)
    To = m.run(T0, 80, q)
    Td = dm.run(T0, 80, q)
    assert To.max() > 60.0  # TD laws are exercised over a wide range
    assert np.max(np.abs(To - Td)) <= 1e-12 * np.max(np.abs(To))


def test_first_order_in_time_against_expm():
    xyz, tets, bnd = jittered_box(3, 3, 3, 1e-3, seed=8)
    mat = ti_materials()
    m = oracle.OracleModel(xyz, tets, mat, bnd, np.full(len(bnd), 37.0))
    dm = dense.DenseModel(xyz, tets, m.mat, bnd, np.full(len(bnd), 37.0), 0)
    rng = np.random.default_rng(0)
    T0 = m.initial(37.0) + np.where(m.is_dir.astype(bool), 0.0,
                                    rng.uniform(0, 5, m.N))
    q = np.where(m.is_dir.astype(bool), 0.0, rng.uniform(0, 1e-3, m.N))
    t_end = 2.0
    exact = dm.expm_solution(T0, t_end, q)
    dtcr = m.dt_cr()
    errs = []
    for n in (int(np.ceil(t_end / (0.05 * dtcr))) * k for k in (1, 2, 4)):
        m.dt = t_end / n
        errs.append(np.max(np.abs(m.run(T0, n, q) - exact)))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(orders - 1.0) <= 0.05), (errs, orders)


# --------------------------------------------------------------------------
# Pin 8: the critical step (Eq 9).  Slightly above dt_cr a tiny perturbation
# grows; slightly below it decays.
# --------------------------------------------------------------------------
def test_critical_dt_threshold():
    s = sc.config1()
    m = oracle.build_model(s)
    dtcr = m.dt_cr(method="dense")
    rng = np.random.default_rng(11)
    pert = np.where(m.is_dir.astype(bool), 0.0, rng.uniform(-1e-8, 1e-8, m.N))
    T0 = m.initial(37.0) + pert
    m.dt = 1.01 * dtcr
    Tu = m.run(T0, 1000)
    m.dt = 0.99 * dtcr
    Ts = m.run(T0, 1000)
    assert np.max(np.abs(Tu - 37.0)) > 1e-2
    assert np.max(np.abs(Ts - 37.0)) < 1e-8


# --------------------------------------------------------------------------
# Pin 9: temperature-dependent conduction.  The 1-D steady state with
# k = k0 (1 + beta (T - T_r)) has a linear Kirchhoff transform; the long-run
# explicit solution (Eq 13, 17, 19) converges to it at (at least) second
# order.
# --------------------------------------------------------------------------
def test_td_kirchhoff_steady_state_order():
    L = 6e-3
    errs = []
    for M in (3, 6, 12):
        h = L / M
        xyz, tets = mesh.kuhn_box(M, 1, 1, h)
        x = xyz[:, 0]
        left = np.abs(x) < 1e-12
        right = np.abs(x - L) < 1e-12
        dn = np.nonzero(left | right)[0]
        dT = np.where(left[dn], 37.0, 90.0)
        beta = 0.02
        mat = sc.Materials(rho0=1000.0, c0=4000.0, k0=0.5, dk_dT=0.5 * beta,
                           T_ref=37.0, T_lo=0.0, T_hi=100.0, w_b=0.0)
        m = oracle.OracleModel(xyz, tets, mat, dn, dT)
        m.dt = 0.9 * m.dt_cr(method="dense")
        T = m.initial(37.0)
        for _ in range(200):
            Tn = m.run(T, 2000)
            if np.max(np.abs(Tn - T)) < 1e-13:
                T = Tn
                break
            T = Tn
        ex = cf.kirchhoff_slab(x, L, 37.0, 90.0, 0.5, beta, 37.0)
        errs.append(np.max(np.abs(T - ex)))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    # at least second order (the Kuhn slab converges slightly faster than
    # h^2 here); using k0 instead of k(T) would stall at an O(1) error
    assert np.all(orders >= 1.8), (errs, orders)
    assert errs[-1] < 1e-2


# --------------------------------------------------------------------------
# Pin 10: numbering invariance.  Renumbering nodes and elements (and the
# corner order inside elements) changes only the rounding order.
# --------------------------------------------------------------------------
def test_ordering_invariance():
    xyz, tets, bnd = jittered_box(5, 4, 4, 1e-3, seed=10)
    mat = sc.td_materials()
    src = [[2.5e-3, 2e-3, 2e-3, 1e-3, 2e8]]
    m = oracle.OracleModel(xyz, tets, mat, bnd, np.full(len(bnd), 37.0))
    m.dt = 0.9 * m.dt_cr()
    T = m.run(m.initial(37.0), 200, m.source_consistent(src))
    x2, t2, b2, nperm, _ = mesh.shuffle_mesh(xyz, tets, bnd,
                                             np.random.default_rng(3))
    m2 = oracle.OracleModel(x2, t2, mat, b2, np.full(len(b2), 37.0))
    m2.dt = m.dt
    T2 = m2.run(m2.initial(37.0), 200, m2.source_consistent(src))
    assert T.max() > 45.0
    assert np.max(np.abs(T2 - T[nperm])) <= 1e-11


# --------------------------------------------------------------------------
# Pin 11: the paper's own arithmetic (Sec 3.1.3, 3.1.4, 3.1.6, Table 6).
# --------------------------------------------------------------------------
def test_paper_internal_arithmetic():
    g = json.load(open(os.path.join(GOLDEN, "paper_values.json")))
    tab = g["td_table_sec_3_1_6"]
    dT = tab["T_points"][1] - tab["T_points"][0]
    for key in ("rho", "k", "c"):
        slope = (tab[key][1] - tab[key][0]) / dT
        assert abs(slope - tab["printed_slopes"][key]) <= 5e-5 * abs(slope)
    pm = sc.paper_table_materials()
    assert abs(pm.k0 + pm.dk_dT * 28.0 - 0.57) < 1e-15
    assert abs(pm.rho0 + pm.drho_dT * 28.0 - 1000.0) < 1e-12
    assert abs(pm.c0 + pm.dc_dT * 28.0 - 3800.0) < 1e-12
    f = g["perfusion_film_sec_3_1_3"]
    h = f["w_b"] * f["c_b"] * f["volume_m3"] / f["n_nodes"]
    assert abs(h - f["printed_h"]) <= 0.5e-4
    mq = g["metabolic_flux_sec_3_1_4"]
    qn = mq["Q_m"] * mq["volume_m3"] / mq["n_nodes"]
    assert abs(qn - mq["printed_q"]) <= 0.5e-4
    t = g["timing_sec_3_2_table_6"]
    r = t["printed_ratios"]
    assert abs(t["A_threads_total_ms"] / t["P_TD_openmp_total_ms"]
               - r["TD_vs_A_threads"]) < 0.01
    assert abs(t["A_serial_total_ms"] / t["P_TD_openmp_total_ms"]
               - r["TD_vs_A_serial"]) < 0.01
    assert abs(t["A_threads_total_ms"] / t["P_TI_openmp_total_ms"]
               - r["TI_vs_A_threads"]) < 0.01
    assert abs(t["A_serial_total_ms"] / t["P_TI_openmp_total_ms"]
               - r["TI_vs_A_serial"]) < 0.01
    assert abs(t["P_TD_openmp_total_ms"] / t["P_TI_openmp_total_ms"]
               - r["TI_vs_TD"]) < 0.005
    assert abs(t["P_TD_serial_total_ms"] / t["P_TD_openmp_total_ms"]
               - r["TD_openmp_vs_serial"]) < 0.001
    for k in ("P_TD_openmp", "P_TI_openmp", "P_TD_serial"):
        assert abs(t[k + "_ms_per_step"] * t["steps"] - t[k + "_total_ms"]) < 1


# --------------------------------------------------------------------------
# Assembly order and sources.
# --------------------------------------------------------------------------
def test_assembly_is_sequential_scatter():
    """Eq 11 as a plain sequential scatter in element order, bitwise."""
    xyz, tets, bnd = jittered_box(3, 3, 2, 1e-3, seed=12)
    mat = sc.td_materials()
    m = oracle.OracleModel(xyz, tets, mat, bnd, np.full(len(bnd), 37.0))
    m.dt = 0.1
    rng = np.random.default_rng(1)
    T = 37.0 + rng.uniform(0, 30, m.N)
    _, F, _ = m.step(T)
    Fs = [0.0] * m.N
    for e in range(m.E):
        n = tets[e]
        ke = 0.0
        for a in range(4):
            ke += 0.512 + 0.512 * 0.0013 * (min(max(T[n[a]], 0.0), 100.0) - 37.0)
        ke /= 4.0
        for a in range(4):
            s = 0.0
            for b in range(4):
                s += m.A[e, a, b] * T[n[b]]
            Fs[n[a]] += ke * s
    assert np.array_equal(np.array(Fs), F)


def test_quadrature_rule_degree_two():
    P = oracle.quadrature_points()
    assert P.shape == (256, 4)
    assert np.allclose(P.sum(axis=1), 1.0, atol=1e-15)
    assert np.all(P > 0)
    # int over the reference tet of lambda_a lambda_b / V = (1 + delta_ab)/20
    M2 = P.T @ P / 256.0
    assert np.allclose(M2, (np.ones((4, 4)) + np.eye(4)) / 20.0, atol=1e-15)
    assert np.allclose(P.mean(axis=0), 0.25, atol=1e-15)


def test_consistent_source_constant_and_total_power():
    xyz, tets, bnd = jittered_box(6, 6, 6, 1e-3, seed=13)
    m = oracle.OracleModel(xyz, tets, ti_materials())
    # a very wide Gaussian is constant to 1e-12 over the box
    q = m.source_consistent([[3e-3, 3e-3, 3e-3, 1e4, 7e5]])
    assert np.max(np.abs(q - 7e5 * m.Vi)) <= 1e-11 * np.max(q)
    # a resolved Gaussian well inside the box carries its analytic power
    q2 = m.source_consistent([[3e-3, 3e-3, 3e-3, 0.5e-3, 1e7]])
    tot = cf.gaussian_total_power(1e7, 0.5e-3)
    assert abs(q2.sum() / tot - 1.0) < 2e-3
    # nodal sampling: Q(x_i) V_i exactly
    q3 = m.source_nodal([[3e-3, 3e-3, 3e-3, 0.5e-3, 1e7]])
    r2 = np.sum((xyz - 3e-3) ** 2, axis=1)
    assert np.allclose(q3, 1e7 * np.exp(-r2 / (2 * 0.25e-6)) * m.Vi,
                       rtol=1e-14, atol=0)


def test_degenerate_element_reported():
    xyz, tets = mesh.kuhn_box(2, 2, 2, 1e-3)
    xyz = xyz.copy()
    t = tets[5]
    # collapse element 5 onto a plane: move its last vertex into the plane of
    # the first three (shared vertices move, so pick the first bad index)
    p0, p1, p2 = xyz[t[0]], xyz[t[1]], xyz[t[2]]
    xyz[t[3]] = (p0 + p1 + p2) / 3.0
    with pytest.raises(ValueError, match="degenerate"):
        oracle.OracleModel(xyz, tets, ti_materials())


# --------------------------------------------------------------------------
# Scheduled sources (the external heat applied at every step of Algorithm 1;
# the heat-then-relax runs of Sec 3.1.5) and surface heat flux (Eq 4).
# --------------------------------------------------------------------------
def test_schedule_amplitude_values():
    t = [1.0, 3.0, 3.0, 5.0]
    a = [2.0, 6.0, -1.0, 0.0]
    cases = {0.0: 2.0, 1.0: 2.0, 2.0: 4.0, 2.5: 5.0, 3.0: -1.0, 4.0: -0.5, 5.0: 0.0, 9.0: 0.0}
    for x, v in cases.items():
        assert oracle.schedule_amplitude(t, a, x) == pytest.approx(v, abs=1e-15), x
    assert oracle.schedule_amplitude([2.0], [7.0], -1.0) == 7.0
    assert oracle.schedule_amplitude([2.0], [7.0], 5.0) == 7.0


def test_scheduled_uniform_source_closed_form():
    """Adiabatic box, constant properties, a uniform source q0 per unit volume
    ramped by a(t): the field stays uniform (zero row sums) and
    T_n = T0 + dt q0 / (rho c) * sum_{k<n} a(t_k), an exact finite sum."""
    xyz, tets, _ = jittered_box(4, 3, 3, 1e-3, seed=21)
    mat = ti_materials(w_b=0.0)
    m = oracle.OracleModel(xyz, tets, mat)
    m.dt = 0.05
    q0 = 2e6
    Q = q0 * m.Vi
    sched = ([0.0, 1.0, 1.0, 2.0], [0.0, 1.0, 0.5, 0.5])
    n = 60
    T = m.run_schedule(np.full(m.N, 37.0), n, [Q], [sched])
    amps = [oracle.schedule_amplitude(*sched, k * m.dt) for k in range(n)]
    # hand values of the same ramp: t/1 before 1 s, then 0.5
    assert amps == pytest.approx([min(k * 0.05, 1.0) if k * 0.05 < 1.0 else 0.5
                                  for k in range(n)], abs=1e-15)
    expect = 37.0 + m.dt * q0 / (1060.0 * 3600.0) * sum(amps)
    assert np.max(np.abs(T - expect)) <= 1e-12 * expect


def test_two_stage_schedule_equals_two_runs():
    xyz, tets, bnd = jittered_box(5, 4, 3, 1e-3, seed=22)
    mat = sc.td_materials()
    m = oracle.OracleModel(xyz, tets, mat, bnd, np.full(len(bnd), 37.0))
    m.dt = 0.9 * m.dt_cr()
    q = m.source_consistent([[2.5e-3, 2e-3, 1.5e-3, 1e-3, 3e7]])
    n1, n2 = 40, 35
    t1 = (n1 - 0.5) * m.dt  # switched off between steps n1 - 1 and n1
    T_sched = m.run_schedule(m.initial(37.0), n1 + n2, [q], [([t1, t1], [1.0, 0.0])])
    T_two = m.run(m.run(m.initial(37.0), n1, q), n2, None)
    assert np.array_equal(T_sched, T_two)


def test_flux_loads_total_and_lattice_face():
    """On the x = 0 face of a Kuhn box every interior face node carries
    q h^2 (six triangles of area h^2 / 2, a third each) and the loads sum to
    q times the face area."""
    nx, ny, nz, h = 4, 5, 3, 1e-3
    xyz, tets = mesh.kuhn_box(nx, ny, nz, h)
    faces = mesh.boundary_faces(tets)
    on_x0 = np.all(xyz[faces][:, :, 0] == 0.0, axis=1)
    q = 1.5e4
    out = oracle.flux_loads(xyz, faces[on_x0], np.full(on_x0.sum(), q))
    assert out.sum() == pytest.approx(q * (ny * h) * (nz * h), rel=1e-14)
    j = np.round(xyz[:, 1] / h).astype(int)
    k = np.round(xyz[:, 2] / h).astype(int)
    inner = (xyz[:, 0] == 0.0) & (j > 0) & (j < ny) & (k > 0) & (k < nz)
    assert inner.sum() == (ny - 1) * (nz - 1)
    assert np.allclose(out[inner], q * h * h, rtol=1e-14, atol=0.0)
    assert np.all(out[xyz[:, 0] > 0.0] == 0.0)


# --------------------------------------------------------------------------
# Property tables (Eq 2; the paper's two-point tissue data of Sec 3.1.6 and
# their generalisation to piecewise-linear tables).
# --------------------------------------------------------------------------
def test_two_point_tables_equal_linear_law():
    """The paper's two-point data written as tables reproduce the clamped
    linear law (rounding only), and the critical step is the same."""
    xyz, tets, bnd = jittered_box(5, 4, 4, 1e-3, seed=41)
    mat = sc.paper_table_materials()
    lin = oracle.OracleModel(xyz, tets, mat, bnd, np.full(len(bnd), 37.0))
    tables = {"k": ([37.0, 65.0], [0.53, 0.57]), "rho": ([37.0, 65.0], [1040.0, 1000.0]),
              "c": ([37.0, 65.0], [3600.0, 3800.0])}
    tab = oracle.OracleModel(xyz, tets, mat, bnd, np.full(len(bnd), 37.0), tables=tables)
    assert tab.dt_cr() == pytest.approx(lin.dt_cr(), rel=1e-13)
    lin.dt = tab.dt = 0.9 * lin.dt_cr()
    q = lin.source_consistent([[2.5e-3, 2e-3, 2e-3, 1e-3, 6e7]])
    Ta = lin.run(lin.initial(37.0), 300, q)
    Tb = tab.run(tab.initial(37.0), 300, q)
    assert Ta.max() > 60.0  # the run crosses the table's range
    assert np.max(np.abs(Ta - Tb)) <= 1e-11


def test_table_conductivity_kirchhoff_order():
    """Piecewise-linear k(T): the long-run FED-FEM field converges at second
    order to the Kirchhoff steady state; the linear law of the first piece
    alone would stall at an O(1) error."""
    L = 6e-3
    Tk, kv = [37.0, 60.0, 90.0], [0.5, 0.65, 0.55]
    errs = []
    for M_ in (3, 6, 12):
        h = L / M_
        xyz, tets = mesh.kuhn_box(M_, 1, 1, h)
        x = xyz[:, 0]
        left, right = np.abs(x) < 1e-12, np.abs(x - L) < 1e-12
        dn = np.nonzero(left | right)[0]
        dT = np.where(left[dn], 37.0, 90.0)
        mat = sc.Materials(rho0=1000.0, c0=4000.0, k0=0.5, T_ref=37.0, T_lo=0.0, T_hi=100.0,
                           w_b=0.0)
        m = oracle.OracleModel(xyz, tets, mat, dn, dT, tables={"k": (Tk, kv)})
        m.dt = 0.9 * m.dt_cr(method="dense")
        T = m.initial(37.0)
        for _ in range(200):
            Tn = m.run(T, 2000)
            if np.max(np.abs(Tn - T)) < 1e-13:
                T = Tn
                break
            T = Tn
        ex = cf.kirchhoff_slab_table(x, L, 37.0, 90.0, Tk, kv)
        errs.append(np.max(np.abs(T - ex)))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders >= 1.8), (errs, orders)
    # the kink of k at 60 C keeps the constant larger than for a linear k
    assert errs[-1] < 0.05


def test_table_window_bound_is_the_exact_extreme():
    """k_max and (rho c)_min of tables (with rho c dipping inside a piece)
    against dense sampling of the same functions."""
    mat = sc.td_materials()
    m = oracle.mat_vector(mat)
    tables = {"k": ([10.0, 40.0, 80.0], [0.4, 0.7, 0.6]),
              "rho": ([20.0, 90.0], [1100.0, 900.0]),
              "c": ([0.0, 50.0, 100.0], [3000.0, 4200.0, 3300.0])}
    kmax, rcmin = dense.material_window(m, tables)
    Ts = np.linspace(-20.0, 130.0, 300001)
    k = dense.prop_value(Ts, m, tables, "k")
    rc = dense.prop_value(Ts, m, tables, "rho") * dense.prop_value(Ts, m, tables, "c")
    assert kmax == pytest.approx(k.max(), rel=1e-12)
    assert rcmin <= rc.min() * (1 + 1e-12)
    assert rcmin >= rc.min() * (1 - 1e-6)
