"""GPU parity of table-driven temperature-dependent properties (Eq 2; the
paper's two-point tissue data of Sec 3.1.6, generalised to piecewise-linear
tables of k, rho and c) with the FP64 oracle.  Tolerances as for the plain
path: FP64 1e-10 K, FP32C 1e-3 K."""
import numpy as np
import pytest

import oracle
from oracle import dense
from paper_1909_05098_amd import fedfem as ff
from synth import scenarios as sc

from helpers import jittered_box

pytestmark = pytest.mark.gpu

TOL = {ff.FP64: 1e-10, ff.FP32C: 1e-3}
TABLES = {"k": ([30.0, 45.0, 60.0, 80.0], [0.50, 0.56, 0.66, 0.60]),
          "rho": ([37.0, 70.0], [1060.0, 1000.0]),
          "c": ([20.0, 50.0, 75.0, 100.0], [3500.0, 3800.0, 3600.0, 3300.0])}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    torch.cuda.set_device(0)
    ff.load()


def case(seed=51):
    xyz, tets, bnd = jittered_box(9, 8, 7, 1e-3, seed=seed)
    return xyz, tets, bnd, sc.td_materials()


def handle(xyz, tets, bnd, mat, prec, dt, tables):
    h = ff.Handle(xyz, tets, mat, 37.0, bnd, np.full(len(bnd), 37.0), dt=dt, precision=prec,
                  tile_elems=128)
    if tables:
        h.set_property_tables(tables)
    h.precompute()
    return h


@pytest.mark.parametrize("prec", [ff.FP64, ff.FP32C])
def test_tables_parity_and_critical_step(prec):
    xyz, tets, bnd, mat = case()
    om = oracle.OracleModel(xyz, tets, mat, bnd, np.full(len(bnd), 37.0), tables=TABLES)
    dt_o = om.dt_cr()
    # the library's own critical step from its Lanczos estimate
    h0 = handle(xyz, tets, bnd, mat, prec, -0.9, TABLES)
    _, dt_g = h0.dt()
    h0.close()
    print(f"[tables] dt_cr gpu {dt_g:.9e} oracle {dt_o:.9e}", flush=True)
    assert dt_o / (1 + 1e-3) <= dt_g <= dt_o / (1 - 1e-4)
    om.dt = 0.9 * dt_o
    q = om.source_consistent([[4e-3, 3.5e-3, 3e-3, 1.2e-3, 6e7]])
    n = 400
    T_ref = om.run(om.initial(37.0), n, q)
    h = handle(xyz, tets, bnd, mat, prec, om.dt, TABLES)
    h.step(n, q)
    err = float(np.max(np.abs(h.read_T() - T_ref)))
    print(f"[tables] prec={prec}: max|dT| {err:.3e} K, peak {T_ref.max():.2f} C", flush=True)
    assert T_ref.max() > 85.0  # the run crosses every table's points
    assert err <= TOL[prec]
    h.close()


def test_two_point_tables_equal_linear_law_on_gpu():
    xyz, tets, bnd, _ = case(52)
    mat = sc.paper_table_materials()
    two = {"k": ([37.0, 65.0], [0.53, 0.57]), "rho": ([37.0, 65.0], [1040.0, 1000.0]),
           "c": ([37.0, 65.0], [3600.0, 3800.0])}
    om = oracle.OracleModel(xyz, tets, mat, bnd, np.full(len(bnd), 37.0))
    dt = 0.9 * om.dt_cr()
    q = om.source_consistent([[4e-3, 3.5e-3, 3e-3, 1.2e-3, 6e7]])
    out = []
    for tables in (None, two):
        h = handle(xyz, tets, bnd, mat, ff.FP64, dt, tables)
        h.step(300, q)
        out.append(h.read_T())
        h.close()
    assert out[0].max() > 60.0
    assert np.max(np.abs(out[0] - out[1])) <= 1e-10


def test_table_arguments_and_batch():
    xyz, tets, bnd, mat = case(53)
    h = ff.Handle(xyz, tets, mat, 37.0, bnd, np.full(len(bnd), 37.0), dt=-0.9,
                  precision=ff.FP32C)
    with pytest.raises(ff.FedFemError):
        h.set_property_tables({"k": ([40.0, 40.0], [0.5, 0.6])})
    with pytest.raises(ff.FedFemError):
        h.set_property_tables({"c": ([40.0, 50.0], [3600.0, 0.0])})
    h.set_property_tables(TABLES)
    h.precompute()
    with pytest.raises(ff.FedFemError) as ei:
        h.set_property_tables(TABLES)
    assert ei.value.code == ff.E_STATE
    # batched stepping carries each handle's tables
    q = oracle.OracleModel(xyz, tets, mat, bnd, np.full(len(bnd), 37.0)).source_consistent(
        [[4e-3, 3.5e-3, 3e-3, 1.2e-3, 6e7]])
    h2 = ff.Handle(xyz, tets, mat, 37.0, bnd, np.full(len(bnd), 37.0), dt=-0.9,
                   precision=ff.FP32C)
    h2.set_property_tables(TABLES)
    h2.precompute()
    for x in (h, h2):
        x.set_source(q)
    h.step(120)
    b = ff.Batch([h2])
    b.run([120])
    b.close()
    assert np.array_equal(h.read_state()[0], h2.read_state()[0])
    h.close()
    h2.close()
