"""GPU parity of the eight-node reduced-integration hexahedron (Sec 2.3.3,
Eq 14, 16) with the FP64 NumPy oracle (oracle/hex.py).

Tolerances as for tetrahedra: FP64 path 1e-10 K, compensated FP32 path
1e-3 K, critical-step eigenvalue within the Lanczos bound of the oracle's.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import closed_forms as cf
from oracle import hex as ohx
from paper_1909_05098_amd import fedfem as ff
from synth import mesh, scenarios as sc

pytestmark = pytest.mark.gpu

TOL = {ff.FP64: 1e-10, ff.FP32C: 1e-3}
ROTATE_Z = [1, 2, 3, 0, 5, 6, 7, 4]   # same hexahedron, corners relabelled
MIRROR = [4, 5, 6, 7, 0, 1, 2, 3]     # same hexahedron, det J < 0


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    torch.cuda.set_device(0)
    ff.load()


def jittered_hex_box(nx, ny, nz, h, seed, jitter=0.2):
    xyz, hexes = mesh.hex_box(nx, ny, nz, h)
    bnd = mesh.box_surface_nodes(nx, ny, nz)
    rng = np.random.default_rng(seed)
    mask = np.ones(len(xyz), bool)
    mask[bnd] = False
    xyz[mask] += rng.uniform(-jitter * h, jitter * h, (mask.sum(), 3))
    return xyz, hexes, bnd


def shuffled(xyz, hexes, bnd, seed):
    """Random node and element numbering, and each element's corners
    relabelled by a rotation or a mirror of the reference cube."""
    rng = np.random.default_rng(seed)
    n_perm = rng.permutation(len(xyz))
    inv = np.empty_like(n_perm)
    inv[n_perm] = np.arange(len(xyz))
    e_perm = rng.permutation(len(hexes))
    hx = inv[hexes[e_perm]]
    pick = rng.integers(0, 3, len(hx))
    hx[pick == 1] = hx[pick == 1][:, ROTATE_Z]
    hx[pick == 2] = hx[pick == 2][:, MIRROR]
    return xyz[n_perm], hx.astype(np.int32), np.sort(inv[bnd]).astype(np.int32)


def oracle_model(xyz, hexes, mat, bnd, dt=None):
    m = ohx.HexModel(xyz, hexes, oracle.mat_vector(mat), bnd, np.full(len(bnd), 37.0))
    m.dt = 0.9 * m.dt_cr() if dt is None else dt
    return m


@pytest.mark.parametrize("prec", [ff.FP64, ff.FP32C])
@pytest.mark.parametrize("reorder,tile", [(1, 1024), (0, 64), (1, 128)])
def test_hex_parity_jittered_box(prec, reorder, tile):
    xyz, hexes, bnd = jittered_hex_box(18, 14, 10, 1e-3, seed=41)
    xyz, hexes, bnd = shuffled(xyz, hexes, bnd, seed=3)
    mat = sc.td_materials()
    mat.Q_m = 3000.0
    om = oracle_model(xyz, hexes, mat, bnd)
    src = [[9e-3, 7e-3, 5e-3, 1.5e-3, 4e8], [4e-3, 4e-3, 3e-3, 1e-3, 2e8]]
    q = om.source_nodal(src)
    n = 300
    T_ref = om.run(om.initial(37.0), n, q)
    h = ff.Handle(xyz, hexes, mat, 37.0, bnd, np.full(len(bnd), 37.0), dt=om.dt,
                  precision=prec, reorder=bool(reorder), tile_elems=tile)
    h.precompute()
    h.set_gaussian_sources(np.array(src), ff.SOURCE_NODAL)
    qg = h.read_source()
    assert np.max(np.abs(qg - q)) <= (1e-12 if prec == ff.FP64 else 1e-6) * q.max()
    h.step(n)
    err = float(np.max(np.abs(h.read_T() - T_ref)))
    info = h.info()
    print(f"[hex] prec={prec} reorder={reorder} tile={tile}: tiles={info['n_tiles']} "
          f"max|dT|={err:.3e} K peak={T_ref.max():.2f}", flush=True)
    assert T_ref.max() > 60.0
    assert info["n_tiles"] >= 3
    assert err <= TOL[prec]
    h.close()


def test_hex_critical_step():
    """Lanczos on the GPU against the closed-form mode maximum (regular box)
    and the oracle's eigenvalue (jittered box), and dt = 0.9 dt_cr."""
    xyz, hexes = mesh.hex_box(12, 10, 9, 0.8e-3)
    bnd = mesh.box_surface_nodes(12, 10, 9)
    mat = sc.td_materials()
    h = ff.Handle(xyz, hexes, mat, 37.0, bnd, np.full(len(bnd), 37.0), dt=-0.9,
                  precision=ff.FP32C)
    h.precompute()
    lam = cf.hex_box_lambda(12, 10, 9, 0.8e-3)
    lam_g = h.info()["lambda_geometry"]
    print(f"[hex] regular box lambda gpu={lam_g:.10e} closed form={lam:.10e}", flush=True)
    assert (1 - 1e-4) * lam <= lam_g <= (1 + 1e-3) * lam
    dt, dtcr = h.dt()
    assert abs(dt - 0.9 * dtcr) <= 1e-15 * dt
    h.close()
    xyz, hexes, bnd = jittered_hex_box(10, 9, 8, 1e-3, seed=5)
    om = oracle_model(xyz, hexes, mat, bnd, dt=1.0)
    lam_o = om.geometry_lambda()
    h = ff.Handle(xyz, hexes, mat, 37.0, bnd, np.full(len(bnd), 37.0), dt=-0.9,
                  precision=ff.FP64)
    h.precompute()
    lam_g = h.info()["lambda_geometry"]
    print(f"[hex] jittered lambda gpu={lam_g:.10e} oracle={lam_o:.10e}", flush=True)
    assert (1 - 1e-4) * lam_o <= lam_g <= (1 + 1e-3) * lam_o
    h.close()


@pytest.mark.parametrize("prec", [ff.FP64, ff.FP32C])
def test_hex_zero_energy_mode_is_kept(prec):
    """Eq 14 read without hourglass control: on a regular box a checkerboard
    field (held on the surface too) has zero gradient at every element
    centre, so with no perfusion and no source it stays as it is."""
    nx, ny, nz = 8, 6, 5
    xyz, hexes = mesh.hex_box(nx, ny, nz, 1e-3)
    K, J, I = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1),
                          indexing="ij")
    chk = 37.0 + 2.0 * ((-1.0) ** (I + J + K)).ravel()
    bnd = mesh.box_surface_nodes(nx, ny, nz)
    mat = sc.td_materials(w_b=0.0)
    om = ohx.HexModel(xyz, hexes, oracle.mat_vector(mat), bnd, chk[bnd])
    om.dt = 0.9 * om.dt_cr()
    T_ref = om.run(chk.copy(), 100)
    h = ff.Handle(xyz, hexes, mat, 37.0, bnd, chk[bnd], dt=om.dt, precision=prec)
    h.precompute()
    # start from the checkerboard (raw state, caller's node order)
    T0 = chk
    if prec == ff.FP64:
        raw = T0.astype(np.float64).view(np.uint8)
    else:
        hi = T0.astype(np.float32)
        raw = np.concatenate([hi, (T0 - hi).astype(np.float32)]).view(np.uint8)
    h.write_state(raw, 0.0, 0)
    h.step(100)
    err = float(np.max(np.abs(h.read_T() - T_ref)))
    print(f"[hex] checkerboard prec={prec}: max|dT| {err:.3e} K, oracle drift "
          f"{float(np.max(np.abs(T_ref - chk))):.1e} K", flush=True)
    assert np.max(np.abs(T_ref - chk)) <= 1e-12
    assert err <= TOL[prec]
    h.close()


def test_hex_autotune_and_errors():
    xyz, hexes, bnd = jittered_hex_box(16, 12, 10, 1e-3, seed=8)
    mat = sc.td_materials()
    om = oracle_model(xyz, hexes, mat, bnd)
    q = om.source_nodal([[8e-3, 6e-3, 5e-3, 1.5e-3, 4e8]])
    T_ref = om.run(om.initial(37.0), 200, q)
    h = ff.Handle(xyz, hexes, mat, 37.0, bnd, np.full(len(bnd), 37.0), dt=om.dt,
                  precision=ff.FP32C)
    chosen = h.autotune(None)
    h.precompute()
    h.set_gaussian_sources(np.array([[8e-3, 6e-3, 5e-3, 1.5e-3, 4e8]]), ff.SOURCE_NODAL)
    h.step(200)
    err = float(np.max(np.abs(h.read_T() - T_ref)))
    print(f"[hex] autotuned {chosen}: max|dT| {err:.3e} K", flush=True)
    assert err <= 1e-3
    # what a hexahedral handle refuses
    with pytest.raises(ff.FedFemError) as ei:
        h.flux_loads(np.array([[0, 1, 2]], dtype=np.int32), [1.0])
    assert ei.value.code == ff.E_INVALID
    with pytest.raises(ff.FedFemError) as ei:
        ff.Batch([h])
    assert ei.value.code == ff.E_STATE
    import torch
    from paper_1909_05098_amd import surrogate as sg
    Tg = torch.empty(8 ** 3, dtype=torch.float32, device="cuda")
    mg = torch.empty(8 ** 3, dtype=torch.uint8, device="cuda")
    with pytest.raises(ff.FedFemError) as ei:   # P1 resampling is defined on tetrahedra
        sg.resample(h, 8, [8e-3, 6e-3, 5e-3, 0.02], Tg, mg)
    assert ei.value.code == ff.E_INVALID
    with pytest.raises(ff.FedFemError) as ei:   # more tile nodes than 8 per element
        ff.Handle(xyz, hexes, mat, 37.0, bnd, np.full(len(bnd), 37.0), dt=om.dt,
                  precision=ff.FP32C, tile_elems=256, max_tile_nodes=2049)
    assert ei.value.code == ff.E_INVALID
    h.close()
    # a flattened hexahedron is degenerate
    bad = xyz.copy()
    c = hexes[len(hexes) // 2]
    bad[c[4:]] = bad[c[:4]]
    g = ff.Handle(bad, hexes, mat, 37.0, bnd, np.full(len(bnd), 37.0), dt=-0.9)
    with pytest.raises(ff.FedFemError) as ei:
        g.precompute()
    assert ei.value.code == ff.E_DEGENERATE
    g.close()


GOLDEN_HEX = os.path.join(os.path.dirname(__file__), "golden", "hex_ellipsoid_oracle.json")


@pytest.mark.parametrize("order", ["morton", "random"])
def test_hex_ellipsoid_sampled_parity(order):
    """Full size: the 2.91M-hexahedron ellipsoid, 1000 steps at the oracle's
    own step, in the launch configuration the benchmark times (library
    defaults), against the oracle's stored sample of 4096 nodes
    (tests/golden/make_hex_ellipsoid.py), to 1e-3 K."""
    g = json.load(open(GOLDEN_HEX))
    s = sc.hex_ellipsoid("random", n_steps=g["n_steps"])
    assert s.n_tets == g["n_hexes"] and s.n_nodes == g["n_nodes"]
    h = ff.Handle(s.xyz, s.tets, s.materials, s.T0, s.dir_nodes, s.dir_T, dt=g["dt"],
                  precision=ff.FP32C, reorder=(order == "morton"))
    h.precompute()
    lam = h.info()["lambda_geometry"]
    print(f"[hex] ellipsoid lambda gpu={lam:.9e} oracle={g['lambda_geometry']:.9e}", flush=True)
    assert (1 - 1e-4) * g["lambda_geometry"] <= lam <= (1 + 1e-3) * g["lambda_geometry"]
    h.set_gaussian_sources(s.sources, ff.SOURCE_NODAL)
    assert abs(h.read_source().sum() - g["source_total_W"]) <= 1e-9 * g["source_total_W"]
    h.step(g["n_steps"])
    T = h.read_T()
    idx = np.asarray(g["idx"])
    err = float(np.max(np.abs(T[idx] - np.asarray(g["T"]))))
    print(f"[hex] ellipsoid {order}: max|dT| over {len(idx)} sampled nodes = {err:.3e} K "
          f"(Tmax gpu {T.max():.4f}, oracle {g['T_max']:.4f})", flush=True)
    assert err <= 1e-3
    assert abs(T.max() - g["T_max"]) <= 1e-3
    h.close()


@pytest.mark.parametrize("prec", [ff.FP64, ff.FP32C])
def test_hex_schedule_parity(prec):
    """A heating pattern switched off part-way (two points at one time),
    applied by the nodal update of a hexahedral handle over two calls,
    against the oracle stepping with q_n = a(t_n) Q."""
    xyz, hexes, bnd = jittered_hex_box(12, 10, 8, 1e-3, seed=17)
    mat = sc.td_materials()
    om = oracle_model(xyz, hexes, mat, bnd)
    Q = om.source_nodal([[6e-3, 5e-3, 4e-3, 1.5e-3, 8e7]])
    times, amps = [0.0, 200 * om.dt, 200 * om.dt], [1.0, 1.0, 0.0]
    T = om.initial(37.0)
    for n in range(450):
        T = om.step(T, oracle.schedule_amplitude(times, amps, n * om.dt) * Q)
    h = ff.Handle(xyz, hexes, mat, 37.0, bnd, np.full(len(bnd), 37.0), dt=om.dt,
                  precision=prec)
    h.precompute()
    h.set_schedule(Q[None, :], [(times, amps)])
    h.step(300)
    h.step(150)
    err = float(np.max(np.abs(h.read_T() - T)))
    print(f"[hex] schedule prec={prec}: max|dT| {err:.3e} K", flush=True)
    assert err <= TOL[prec]
    h.close()


def test_hex_two_point_tables_equal_linear_law():
    """Tables through two points of the linear laws give the same run as
    the laws themselves on a hexahedral handle (FP64)."""
    xyz, hexes, bnd = jittered_hex_box(10, 9, 8, 1e-3, seed=19)
    mat = sc.paper_table_materials()
    two = {"k": ([37.0, 65.0], [0.53, 0.57]), "rho": ([37.0, 65.0], [1040.0, 1000.0]),
           "c": ([37.0, 65.0], [3600.0, 3800.0])}
    out = []
    dt = -0.9
    for tables in (None, two):
        h = ff.Handle(xyz, hexes, mat, 37.0, bnd, np.full(len(bnd), 37.0), dt=dt,
                      precision=ff.FP64)
        if tables:
            h.set_property_tables(tables)
        h.precompute()
        h.set_gaussian_sources(np.array([[5e-3, 4.5e-3, 4e-3, 1.2e-3, 1.5e8]]), ff.SOURCE_NODAL)
        h.step(300)
        out.append((h.read_T(), h.dt()))
        dt = h.dt()[0]   # the same step for the table run
        h.close()
    assert out[0][0].max() > 60.0
    assert abs(out[0][1][1] - out[1][1][1]) <= 1e-12 * out[0][1][1]   # same critical step
    assert np.max(np.abs(out[0][0] - out[1][0])) <= 1e-10


@pytest.mark.parametrize("prec", [ff.FP64, ff.FP32C])
def test_hex_consistent_source_parity(prec):
    """Gaussian sources integrated against the trilinear shape functions
    (4 x 4 x 4 Gauss-Legendre on each element's map) on a jittered,
    relabelled box: the nodal loads against the oracle's, then 300 steps."""
    xyz, hexes, bnd = jittered_hex_box(14, 12, 10, 1e-3, seed=23)
    xyz, hexes, bnd = shuffled(xyz, hexes, bnd, seed=4)
    mat = sc.td_materials()
    om = oracle_model(xyz, hexes, mat, bnd)
    src = [[7e-3, 6e-3, 5e-3, 1.2e-3, 4e8], [3e-3, 9e-3, 4e-3, 0.8e-3, 2e8]]
    q = om.source_consistent(src)
    T_ref = om.run(om.initial(37.0), 300, q)
    h = ff.Handle(xyz, hexes, mat, 37.0, bnd, np.full(len(bnd), 37.0), dt=om.dt,
                  precision=prec, tile_elems=256)
    h.precompute()
    h.set_gaussian_sources(np.array(src), ff.SOURCE_CONSISTENT)
    qg = h.read_source()
    qerr = float(np.max(np.abs(qg - q)) / q.max())
    h.step(300)
    err = float(np.max(np.abs(h.read_T() - T_ref)))
    print(f"[hex] consistent source prec={prec}: loads {qerr:.2e} relative, max|dT| "
          f"{err:.3e} K, peak {T_ref.max():.1f} C", flush=True)
    assert qerr <= (1e-12 if prec == ff.FP64 else 1e-6)
    assert T_ref.max() > 60.0
    assert err <= TOL[prec]
    h.close()


def test_hex_quad_flux_loads():
    """Surface flux on quadrilaterals of a hexahedral mesh against the
    oracle's 2 x 2 rule: planar faces of the box top and warped quadrilaterals
    through interior nodes, then a run heated by the loads."""
    nx, ny, nz = 10, 8, 6
    xyz, hexes, bnd = jittered_hex_box(nx, ny, nz, 1e-3, seed=29)
    nid = lambda i, j, k: i + (nx + 1) * (j + (ny + 1) * k)
    faces = [[nid(i, j, nz), nid(i + 1, j, nz), nid(i + 1, j + 1, nz), nid(i, j + 1, nz)]
             for i in range(3, 7) for j in range(2, 6)]
    faces += [[nid(i, j, 3), nid(i + 1, j, 3), nid(i + 1, j + 1, 4), nid(i, j + 1, 3)]
              for i in range(2, 5) for j in range(2, 4)]          # warped
    faces = np.array(faces, dtype=np.int32)
    flux = np.linspace(2e4, 5e4, len(faces))
    ref = ohx.flux_loads_quad(xyz, faces, flux)
    mat = sc.td_materials()
    om = oracle_model(xyz, hexes, mat, bnd)
    for prec in (ff.FP64, ff.FP32C):
        h = ff.Handle(xyz, hexes, mat, 37.0, bnd, np.full(len(bnd), 37.0), dt=om.dt,
                      precision=prec)
        h.precompute()
        q = h.flux_loads(faces, flux)
        err = float(np.max(np.abs(q - ref)) / np.max(np.abs(ref)))
        h.set_source(q)
        h.step(200)
        T_ref = om.run(om.initial(37.0), 200, ref)
        terr = float(np.max(np.abs(h.read_T() - T_ref)))
        print(f"[hex] quad flux prec={prec}: loads {err:.2e} relative, max|dT| {terr:.3e} K",
              flush=True)
        assert err <= 1e-13
        assert terr <= TOL[prec]
        with pytest.raises(ff.FedFemError) as ei:
            h.flux_loads(np.array([[0, 1, 2, 1]], dtype=np.int32), [1.0])   # repeated node
        assert ei.value.code == ff.E_INVALID
        h.close()
