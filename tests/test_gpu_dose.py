"""GPU parity of the thermal dose fused into the nodal update (CEM43 and the
Arrhenius damage integral) with the FP64 oracle (oracle/dose.py).

Tolerance, derived from the temperature tolerance: the dose of a step is
dt * rate(T), and d ln(rate)/dT is at most ln 4 per kelvin for CEM43 (below
43 C) and E_a / (R_gas T_K^2) for Arrhenius, so a temperature error e gives a
relative dose error of at most slope * e (1e-10 K for the FP64 path, 1e-3 K
for compensated FP32), plus summation rounding.
"""
import numpy as np
import pytest

import oracle
from oracle import dose
from oracle import hex as ohx
from paper_1909_05098_amd import fedfem as ff
from synth import mesh, scenarios as sc

from helpers import jittered_box

pytestmark = pytest.mark.gpu

TOL_T = {ff.FP64: 1e-10, ff.FP32C: 1e-3}
EA = 2.5e5                                          # J/mol
A = float(np.exp(EA / (dose.R_GAS * (60.0 + 273.15))))   # rate 1/s at 60 C
SRC = np.array([[4e-3, 3e-3, 3e-3, 1.2e-3, 4e8], [7e-3, 5e-3, 2e-3, 0.6e-3, 2e8]])


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    torch.cuda.set_device(0)
    ff.load()


def rate_and_slope(model):
    if model == ff.DOSE_CEM43:
        return dose.cem43_rate, np.log(4.0)
    return (lambda T: dose.arrhenius_rate(T, A, EA)), EA / (dose.R_GAS * 310.15 ** 2)


def check(D, D_ref, rel, name):
    err = np.max(np.abs(D - D_ref) / np.maximum(D_ref, 1e-300))
    print(f"[dose] {name}: max relative error {err:.3e} (dose max {D_ref.max():.4e})",
          flush=True)
    assert np.all(D_ref > 0)
    assert err <= rel


def tet_case():
    xyz, tets, bnd = jittered_box(9, 7, 6, 1e-3, seed=21)
    xyz, tets, bnd, _, _ = mesh.shuffle_mesh(xyz, tets, bnd, np.random.default_rng(5))
    mat = sc.td_materials()
    om = oracle.OracleModel(xyz, tets, mat, bnd, np.full(len(bnd), 37.0))
    om.dt = 0.9 * om.dt_cr()
    q = om.source(SRC, sc.SOURCE_NODAL)
    return xyz, tets, bnd, mat, om, q


@pytest.mark.parametrize("prec", [ff.FP64, ff.FP32C])
@pytest.mark.parametrize("model", [ff.DOSE_CEM43, ff.DOSE_ARRHENIUS])
def test_dose_parity_tets(prec, model):
    """700 steps in two calls (the second crosses a 512-step graph chunk),
    every node against the oracle's dose."""
    xyz, tets, bnd, mat, om, q = tet_case()
    rate, slope = rate_and_slope(model)
    T_ref, D_ref = dose.accumulate(lambda T, n: om.run(T, 1, q), om.initial(37.0), 700,
                                   om.dt, rate)
    h = ff.Handle(xyz, tets, mat, 37.0, bnd, np.full(len(bnd), 37.0), dt=om.dt,
                  precision=prec)
    h.precompute()
    h.set_gaussian_sources(SRC, ff.SOURCE_NODAL)
    h.set_dose(model, A, EA)
    h.step(100)
    h.step(600)
    assert np.max(np.abs(h.read_T() - T_ref)) <= TOL_T[prec]
    assert T_ref.max() > 60.0
    check(h.read_dose(), D_ref, slope * TOL_T[prec] + 1e-12, f"tets prec={prec} model={model}")
    h.close()


@pytest.mark.parametrize("prec", [ff.FP64, ff.FP32C])
def test_dose_parity_hexahedra(prec):
    xyz, hexes = mesh.hex_box(12, 10, 8, 1e-3)
    bnd = mesh.box_surface_nodes(12, 10, 8)
    rng = np.random.default_rng(13)
    inner = np.ones(len(xyz), bool)
    inner[bnd] = False
    xyz[inner] += rng.uniform(-2e-4, 2e-4, (inner.sum(), 3))
    mat = sc.td_materials()
    om = ohx.HexModel(xyz, hexes, oracle.mat_vector(mat), bnd, np.full(len(bnd), 37.0))
    om.dt = 0.9 * om.dt_cr()
    src = np.array([[6e-3, 5e-3, 4e-3, 1.5e-3, 5e7]])
    q = om.source_nodal(src)
    T_ref, D_ref = dose.accumulate(lambda T, n: om.step(T, q), om.initial(37.0), 400, om.dt,
                                   dose.cem43_rate)
    h = ff.Handle(xyz, hexes, mat, 37.0, bnd, np.full(len(bnd), 37.0), dt=om.dt,
                  precision=prec)
    h.precompute()
    h.set_gaussian_sources(src, ff.SOURCE_NODAL)
    h.set_dose(ff.DOSE_CEM43)
    h.step(400)
    assert np.max(np.abs(h.read_T() - T_ref)) <= TOL_T[prec]
    assert 50.0 < T_ref.max() < 300.0
    check(h.read_dose(), D_ref, np.log(4.0) * TOL_T[prec] + 1e-12, f"hexahedra prec={prec}")
    h.close()


def test_dose_leaves_temperature_alone_and_resets():
    """The dose changes no temperature (bit for bit), restarts from zero on
    every fedfem_set_dose, and the API refuses what it should."""
    xyz, tets, bnd, mat, om, q = tet_case()
    hs = []
    for with_dose in (False, True):
        h = ff.Handle(xyz, tets, mat, 37.0, bnd, np.full(len(bnd), 37.0), dt=om.dt,
                      precision=ff.FP32C)
        h.precompute()
        h.set_gaussian_sources(SRC, ff.SOURCE_NODAL)
        if with_dose:
            with pytest.raises(ff.FedFemError) as ei:
                h.read_dose()
            assert ei.value.code == ff.E_STATE
            h.set_dose(ff.DOSE_CEM43)
        h.step(150)
        hs.append(h)
    a, b = hs
    T_ref = om.run(om.initial(37.0), 150, q)
    print(f"[dose] without / with dose: max|T - T_oracle| {np.max(np.abs(a.read_T() - T_ref)):.3e}"
          f" / {np.max(np.abs(b.read_T() - T_ref)):.3e} K", flush=True)
    assert np.array_equal(a.read_T(), b.read_T())
    d1 = b.read_dose()
    assert d1.max() > 0
    b.set_dose(ff.DOSE_CEM43)
    assert np.all(b.read_dose() == 0.0)
    b.step(10)
    a.step(10)
    assert 0 < b.read_dose().max() < d1.max()
    for bad in ((7, 0.0, 0.0), (ff.DOSE_ARRHENIUS, 0.0, EA), (ff.DOSE_ARRHENIUS, A, -1.0),
                (ff.DOSE_ARRHENIUS, float("nan"), EA)):
        with pytest.raises(ff.FedFemError) as ei:
            b.set_dose(*bad)
        assert ei.value.code == ff.E_INVALID
    with pytest.raises(ff.FedFemError) as ei:
        ff.Batch([a, b])
    assert ei.value.code == ff.E_STATE
    b.set_dose(ff.DOSE_OFF)
    with pytest.raises(ff.FedFemError) as ei:
        b.read_dose()
    assert ei.value.code == ff.E_STATE
    b.step(5)
    a.step(5)
    assert np.array_equal(a.read_T(), b.read_T())
    bt = ff.Batch([a, b])   # no dose model left: accepted
    bt.close()
    for h in hs:
        h.close()
