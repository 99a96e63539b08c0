"""fedfem_step_static (stepping without allocation: the tile partials in the
library's fixed per-device scratch array) against fedfem_step, through the C
ABI, on two calls in a row, the second on a smaller mesh.  Both run the same
kernels in the same order, so the temperatures must agree bit for bit (which
is inside the 1e-3 K compensated-FP32 and 1e-10 K FP64 parity bars); the
smaller case is also held to the FP64 oracle at those bars."""
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


def _box(n, h, seed):
    xyz, tets, bnd = jittered_box(n, n, n, h, seed)
    src = np.zeros(len(xyz))
    c = xyz.mean(axis=0)
    r2 = np.sum((xyz - c) ** 2, axis=1)
    src[:] = 2e-3 * np.exp(-r2 / (2 * (3 * h) ** 2))
    return xyz, tets, bnd, src


def _pair(xyz, tets, bnd, prec, dt):
    mat = sc.td_materials()
    hs = []
    for _ in range(2):
        h = ff.Handle(xyz, tets, mat, 37.0, bnd, np.full(len(bnd), 37.0), dt=dt,
                      precision=prec)
        h.precompute()
        hs.append(h)
    return hs


@pytest.mark.parametrize("prec", [ff.FP32C, ff.FP64])
def test_step_static_equals_step_on_two_calls(prec):
    cases = [("larger", 40, 0.5e-3, 11, 300), ("smaller", 10, 1e-3, 12, 200)]
    for name, n, h_, seed, steps in cases:
        xyz, tets, bnd, src = _box(n, h_, seed)
        print(f"[no-alloc] {name} box {len(tets)} tets prec={prec} steps={steps}", flush=True)
        ref, st = _pair(xyz, tets, bnd, prec, -0.9)
        dt = ref.dt()[0]
        st.set_dt(dt)
        assert st.info()["n_partials"] * (4 if prec == ff.FP32C else 8) <= 32 << 20
        # two calls each, the second keeping the source of the first
        ref.step(steps // 2, src)
        ref.step(steps - steps // 2)
        st.step_static(steps // 2, src)
        st.step_static(steps - steps // 2)
        T_ref, T_st = ref.read_T(), st.read_T()
        assert st.time() == ref.time()
        print(f"[no-alloc] {name}: max|T_static - T_step| = "
              f"{np.max(np.abs(T_st - T_ref)):.3e} K (peak {T_ref.max():.3f})", flush=True)
        assert np.array_equal(T_st, T_ref)
        if name == "smaller":
            om = oracle.OracleModel(xyz, tets, sc.td_materials(), bnd, np.full(len(bnd), 37.0))
            om.dt = dt
            T_o = om.run(om.initial(37.0), steps, src)
            err = float(np.max(np.abs(T_st - T_o)))
            print(f"[no-alloc] smaller vs oracle: max|dT| = {err:.3e} K", flush=True)
            assert err <= TOL[prec]
        ref.close()
        st.close()


def test_step_static_hexahedra_and_dose():
    xyz, hexes = mesh.hex_box(8, 7, 6, 1e-3)
    bnd = mesh.box_surface_nodes(8, 7, 6)
    src = np.full(len(xyz), 1e-3)
    out = []
    for use_static in (False, True):
        h = ff.Handle(xyz, hexes, sc.td_materials(), 37.0, bnd, np.full(len(bnd), 37.0),
                      precision=ff.FP32C)
        h.precompute()
        h.set_dose(ff.DOSE_CEM43)
        if use_static:
            h.step_static(150, src)
        else:
            h.step(150, src)
        out.append((h.read_T(), h.read_dose()))
        h.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])


def test_step_static_refusals():
    # a random element order kept as it is puts about four partials on each
    # element: the 2.18M tetrahedra of the h = 1.2 mm ellipsoid, shuffled,
    # need more than 32 MiB of them in FP64
    s = sc.config2()
    xyz, tets, bnd, _, _ = mesh.shuffle_mesh(s.xyz, s.tets, s.dir_nodes,
                                             np.random.default_rng(5))
    h = ff.Handle(xyz, tets, s.materials, s.T0, bnd, np.full(len(bnd), 37.0),
                  precision=ff.FP64, reorder=False)
    h.precompute()
    need = h.info()["n_partials"] * 8
    print(f"[no-alloc] config 2 random order FP64: partials need {need} bytes", flush=True)
    assert need > 32 << 20
    t0 = h.time()
    with pytest.raises(ff.FedFemError) as e:
        h.step_static(3)
    assert e.value.code == ff.E_TOO_LARGE
    assert "static scratch" in h.last_error()
    assert h.time() == t0
    h.step(2)  # the handle still steps through fedfem_step
    h.close()
    # schedules are applied by fedfem_step only
    xyz, tets, bnd, src = _box(6, 1e-3, 3)
    h = ff.Handle(xyz, tets, sc.td_materials(), 37.0, bnd, np.full(len(bnd), 37.0))
    h.precompute()
    h.set_schedule([src], [([0.0, 10.0], [1.0, 0.0])])
    with pytest.raises(ff.FedFemError) as e:
        h.step_static(2)
    assert e.value.code == ff.E_STATE
    with pytest.raises(ValueError):
        h.step_static(2, src[:-1])
    h.close()
