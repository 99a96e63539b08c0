"""GPU parity of scheduled sources and surface heat flux with the FP64 oracle.

Algorithm 1 applies the external heat at every step; the paper heats and
then lets the tissue relax (Sec 3.1.5), and prescribes heat flux on a
boundary part Gamma_H (Eq 4).  The library takes source patterns with
piecewise-linear amplitude schedules (fedfem_set_schedule) and computes the
nodal loads of a surface flux (fedfem_flux_loads); the oracle does both with
its own code.  Tolerances as for the plain path: FP64 1e-10 K, FP32C 1e-3 K;
flux loads 1e-12 relative (FP64 both sides, different summation order).
"""
import numpy as np
import pytest

import oracle
from paper_1909_05098_amd import fedfem as ff
from synth import mesh, scenarios as sc

from helpers import jittered_box

pytestmark = pytest.mark.gpu

TOL = {ff.FP64: 1e-10, ff.FP32C: 1e-3}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    torch.cuda.set_device(0)
    ff.load()


def setup_case(prec, seed=31):
    """Jittered box held at 37 C on its x = max face only; its x = 0 face is
    a flux boundary (Gamma_H), the other faces are insulated."""
    xyz, tets, bnd = jittered_box(9, 8, 7, 1e-3, seed=seed)
    dn = bnd[np.isclose(xyz[bnd, 0], xyz[:, 0].max())]
    mat = sc.td_materials()
    om = oracle.OracleModel(xyz, tets, mat, dn, np.full(len(dn), 37.0))
    om.dt = 0.9 * om.dt_cr()
    h = ff.Handle(xyz, tets, mat, 37.0, dn, np.full(len(dn), 37.0), dt=om.dt, precision=prec,
                  tile_elems=128)
    h.precompute()
    q_src = om.source_consistent([[4e-3, 3.5e-3, 3e-3, 1.2e-3, 4e7]])
    faces = mesh.boundary_faces(tets)
    x0 = np.all(np.isclose(xyz[faces][:, :, 0], xyz[:, 0].min()), axis=1)
    return xyz, tets, dn, mat, om, h, q_src, faces[x0]


def test_flux_loads_match_oracle():
    xyz, tets, bnd = jittered_box(9, 8, 7, 1e-3, seed=33)
    h = ff.Handle(xyz, tets, sc.td_materials(), 37.0, bnd, np.full(len(bnd), 37.0), dt=-0.9)
    h.precompute()
    faces = mesh.boundary_faces(tets)
    rng = np.random.default_rng(5)
    flux = rng.uniform(-2e4, 5e4, len(faces))
    got = h.flux_loads(faces, flux)
    ref = oracle.flux_loads(xyz, faces, flux)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    print(f"[schedule] flux loads: max rel {err:.2e}, total {got.sum():.6e} W", flush=True)
    assert err <= 1e-12
    assert abs(got.sum() - ref.sum()) <= 1e-12 * np.abs(ref).sum()
    # argument checks
    with pytest.raises(ff.FedFemError):
        h.flux_loads(np.array([[0, 0, 1]]), [1.0])
    with pytest.raises(ff.FedFemError):
        h.flux_loads(np.array([[0, 1, len(xyz)]]), [1.0])
    assert np.all(h.flux_loads(np.zeros((0, 3), dtype=np.int32), []) == 0.0)
    with pytest.raises(ff.FedFemError) as ei:   # quadrilaterals belong to hexahedral meshes
        h.flux_loads(np.array([[0, 1, 2, 3]], dtype=np.int32), [1.0])
    assert ei.value.code == ff.E_INVALID
    h.close()


@pytest.mark.parametrize("prec", [ff.FP64, ff.FP32C])
def test_schedule_parity_across_chunks_and_calls(prec):
    """Two patterns over 700 steps (two graph chunks), run as one call and as
    two calls: the source switched off mid-run and a ramped flux pattern."""
    xyz, tets, bnd, mat, om, h, q_src, faces = setup_case(prec)
    flux_nodes = h.flux_loads(faces, np.full(len(faces), 3e4))
    assert np.allclose(flux_nodes, oracle.flux_loads(xyz, faces, np.full(len(faces), 3e4)),
                       rtol=1e-12, atol=0.0)
    dt = om.dt
    scheds = [([300.5 * dt, 300.5 * dt], [1.0, 0.0]),          # heat, then relax
              ([0.0, 200.0 * dt, 650.0 * dt], [0.0, 1.0, 0.25])]  # flux ramp
    pats = [q_src, flux_nodes]
    n = 700
    T_ref = om.run_schedule(om.initial(37.0), n, pats, scheds)
    h.set_schedule(np.stack(pats), scheds)
    h.step(n)
    e1 = float(np.max(np.abs(h.read_T() - T_ref)))
    # the same run again as two calls (time carries over between calls)
    h.write_state(h_state0(h, om), 0.0, 0)
    h.step(430)
    h.step(n - 430)
    e2 = float(np.max(np.abs(h.read_T() - T_ref)))
    print(f"[schedule] prec={prec}: one call {e1:.3e} K, two calls {e2:.3e} K, "
          f"peak rise {T_ref.max() - 37.0:.3f} K", flush=True)
    assert T_ref.max() - 37.0 > 1.0
    assert e1 <= TOL[prec] and e2 <= TOL[prec]
    h.close()


def h_state0(h, om):
    """Raw state of the initial field in the handle's own format."""
    T0 = om.initial(37.0)
    if h.precision == ff.FP64:
        return T0.astype(np.float64).view(np.uint8)
    hi = T0.astype(np.float32)
    lo = (T0 - hi.astype(np.float64)).astype(np.float32)
    return np.concatenate([hi, lo]).view(np.uint8)


@pytest.mark.parametrize("prec", [ff.FP64, ff.FP32C])
def test_constant_schedule_equals_static_source(prec):
    xyz, tets, bnd, mat, om, h, q_src, _ = setup_case(prec, seed=34)
    h.set_source(q_src)
    h.step(150)
    static = h.read_state()[0]
    h.write_state(h_state0(h, om), 0.0, 0)
    h.set_source(None)
    h.set_schedule(q_src[None, :], [([0.0], [1.0])])
    h.step(150)
    assert np.array_equal(h.read_state()[0], static)
    # removing the schedule stops the pattern
    h.set_schedule(None, [])
    h.write_state(h_state0(h, om), 0.0, 0)
    h.step(20)
    assert np.array_equal(h.read_T(), om.initial(37.0))
    h.close()


def test_batch_refuses_scheduled_handle():
    xyz, tets, bnd, mat, om, h, q_src, _ = setup_case(ff.FP32C, seed=35)
    h.set_schedule(q_src[None, :], [([0.0], [1.0])])
    with pytest.raises(ff.FedFemError) as ei:
        ff.Batch([h])
    assert ei.value.code == ff.E_STATE
    with pytest.raises(ff.FedFemError) as ei:   # kernel timing applies no schedule
        h.time_kernels(3)
    assert ei.value.code == ff.E_STATE
    h.set_schedule(None, [])
    b = ff.Batch([h])
    b.close()
    assert min(h.time_kernels(3)) > 0
    h.close()
