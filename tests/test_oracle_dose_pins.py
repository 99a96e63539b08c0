"""Pins of the thermal-dose oracle (oracle/dose.py) against what the two
published models and the mathematics fix.  Each test says which mistake it
catches."""
import numpy as np
import pytest

import oracle
from oracle import dose
from synth import mesh, scenarios as sc


def uniform_model(T, w_b=0.0, n=3, h=1e-3):
    """A small Kuhn box with no source and every node at T: without
    perfusion the field stays exactly uniform (zero row sums), whatever dt
    is."""
    xyz, tets = mesh.kuhn_box(n, n, n, h)
    mat = sc.Materials(w_b=w_b, T_a=37.0)
    m = oracle.OracleModel(xyz, tets, mat)
    return m, np.full(len(xyz), float(T))


@pytest.mark.parametrize("T,minutes", [(43.0, 60.0), (44.0, 30.0), (45.0, 15.0),
                                       (42.0, 240.0), (41.0, 960.0)])
def test_cem43_equivalent_exposures(T, minutes):
    """The defining equivalences of CEM43: 60 min at 43 C, 30 min at 44 C,
    15 min at 45 C, 240 min at 42 C and 960 min at 41 C are all 60
    equivalent minutes.  Catches a wrong base R on either side of 43 C, a
    wrong sign of the exponent, or seconds taken for minutes."""
    m, T0 = uniform_model(T)
    m.dt = 60.0
    T, D = dose.accumulate(lambda T, n: m.run(T, 1), T0, int(minutes), m.dt, dose.cem43_rate)
    assert np.max(np.abs(T - T0)) == 0.0
    assert np.max(np.abs(D - 60.0)) <= 1e-12 * 60.0


def test_cem43_is_continuous_at_43():
    """Both branches give one equivalent minute per minute at 43 C, so the
    rate is continuous there; below it R = 1/4 (half a degree halves the
    rate, a degree quarters it), above it R = 1/2 (a degree doubles it)."""
    r = dose.cem43_rate(np.array([43.0 - 1e-12, 43.0, 42.5, 42.0, 44.0]))
    assert abs(r[0] * 60 - 1.0) <= 1e-11 and r[1] * 60 == 1.0
    assert abs(r[2] / r[1] - 0.5) <= 1e-15 and abs(r[3] / r[1] - 0.25) <= 1e-15
    assert abs(r[4] / r[1] - 2.0) <= 1e-15


def test_arrhenius_at_its_reference_temperature():
    """With A = exp(E_a / (R_gas T*)) the rate is exactly 1/s at T*; ten
    minutes there give Omega = 600.  Catches a missing Kelvin offset, a
    wrong sign in the exponent or a dropped gas constant."""
    Ea = 2.0e5
    Tstar = 55.0
    A = np.exp(Ea / (dose.R_GAS * (Tstar + 273.15)))
    m, T0 = uniform_model(Tstar)
    m.dt = 30.0
    _, D = dose.accumulate(lambda T, n: m.run(T, 1), T0, 20, m.dt,
                           lambda T: dose.arrhenius_rate(T, A, Ea))
    assert np.max(np.abs(D - 600.0)) <= 1e-9 * 600.0
    # one kelvin hotter multiplies the rate by exp(Ea / R (1/T1 - 1/T2))
    r = dose.arrhenius_rate(np.array([Tstar, Tstar + 1.0]), A, Ea)
    expect = np.exp(Ea / 8.314462618 * (1 / 328.15 - 1 / 329.15))
    assert abs(r[1] / r[0] - expect) <= 1e-13 * expect


def test_left_endpoint_on_perfusion_decay():
    """A uniform field relaxing by perfusion alone follows the closed form
    T_n - T_a = (1 - dt m)^n (T_0 - T_a), m = w_b c_b / (rho c); the dose is
    the sum of the rates at T_0 .. T_{n-1}.  Catches a dose taken at the end
    of the step, or a step skipped or counted twice."""
    m, T0 = uniform_model(50.0, w_b=6.4, h=1e-2)
    rho_c = 1060.0 * 3600.0
    rate = 6.4 * 4180.0 / rho_c
    m.dt = 0.9 * m.dt_cr("dense")   # rounding leaves the field uniform only to 1e-16
    n = int(np.ceil(np.log(6.0 / 13.0) / np.log(1.0 - m.dt * rate))) + 10
    T, D = dose.accumulate(lambda T, k: m.run(T, 1), T0, n, m.dt, dose.cem43_rate)
    g = (1.0 - m.dt * rate) ** np.arange(n + 1)
    Tn = 37.0 + g * 13.0
    assert np.max(np.abs(T - Tn[n])) <= 1e-11
    hot = Tn[:n] >= 43.0
    expect = m.dt / 60.0 * (np.sum(2.0 ** (Tn[:n][hot] - 43.0))
                            + np.sum(4.0 ** (Tn[:n][~hot] - 43.0)))
    assert np.any(hot) and np.any(~hot)
    assert np.max(np.abs(D - expect)) <= 1e-12 * expect


def test_dirichlet_nodes_accumulate_at_held_temperature():
    """Held nodes keep T_Gamma, so their dose is n dt R^(43 - T_Gamma) / 60
    exactly, while the heated interior accumulates more."""
    xyz, tets = mesh.kuhn_box(5, 5, 5, 1e-3)
    bnd = mesh.boundary_nodes_by_faces(len(xyz), tets)
    m = oracle.OracleModel(xyz, tets, sc.td_materials(), bnd,
                           np.full(len(bnd), 37.0))
    m.dt = 0.9 * m.dt_cr("dense")
    q = m.source_nodal([[2.5e-3, 2.5e-3, 2.5e-3, 1e-3, 5e8]])
    n = 60
    T, D = dose.accumulate(lambda T, k: m.run(T, 1, q), m.initial(37.0), n, m.dt,
                           dose.cem43_rate)
    held = n * m.dt / 60.0 * 0.25 ** 6
    assert np.max(np.abs(D[bnd] - held)) <= 1e-14 * held
    assert T.max() > 43.0 and D.max() > 10 * held
