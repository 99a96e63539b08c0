"""Thermal dose along an FED-FEM run, in FP64 -- TEST INFRASTRUCTURE.

Only the tests and the scripts that write their stored values use this
module; the product never imports it.

The paper names thermal dose computation for hyperthermia treatment planning
as a use of fast bio-heat solutions (Sec 1) and extending the method to it as
future work (Sec 5), but states no dose model.  Two published ones are used:

- CEM43, the cumulative equivalent minutes at 43 C of Sapareto and Dewey
  (1984): each second at temperature T counts R^(43 - T) / 60 minutes, with
  R = 1/2 at or above 43 C and R = 1/4 below.
- The Arrhenius damage integral of Henriques and Moritz (1947): each second
  adds A exp(-E_a / (R_gas T_K)) with T_K = T + 273.15 and the molar gas
  constant R_gas (2019 SI value 8.314462618 J/(mol K)).

Reading taken here: the explicit update (Eq 19) evaluates every term at the
start of a step, and so does the dose: step n, from t_n to t_n + dt, adds
dt * rate(T_n).  Every node accumulates, Dirichlet nodes at their held
temperature.  The dose is zero when accumulation starts.
"""
from __future__ import annotations

import numpy as np

R_GAS = 8.314462618   # J/(mol K)
KELVIN = 273.15


def cem43_rate(T):
    """Equivalent minutes at 43 C per second spent at T [C]."""
    T = np.asarray(T, dtype=np.float64)
    R = np.where(T >= 43.0, 0.5, 0.25)
    return R ** (43.0 - T) / 60.0


def arrhenius_rate(T, A, Ea):
    """Damage rate [1/s] at T [C] for frequency factor A [1/s] and
    activation energy Ea [J/mol]."""
    T = np.asarray(T, dtype=np.float64)
    return A * np.exp(-Ea / (R_GAS * (T + KELVIN)))


def accumulate(step, T, n_steps, dt, rate):
    """Run n_steps steps T_{n+1} = step(T_n, n) from T and add dt * rate(T_n)
    for each; returns (T after the run, dose per node)."""
    T = np.array(T, dtype=np.float64, copy=True)
    D = np.zeros_like(T)
    for n in range(int(n_steps)):
        D += dt * rate(T)
        T = step(T, n)
    return T, D
