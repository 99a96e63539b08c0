"""GPU parity of the gfx950 library against the FP64 CPU oracle.

Every case runs the HIP path through the C ABI and the oracle on the same
seeded inputs and compares all nodal temperatures.  Tolerances: FP64 path
1e-10 K (rounding order only), compensated FP32 path 1e-3 K (the target the
precision design is held to).
"""
import numpy as np
import pytest

import oracle
from oracle import closed_forms as cf
from oracle import dense
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


def oracle_run(xyz, tets, mat, bnd, src, mode, n, dt=None, T0=37.0, schedule=None):
    om = oracle.OracleModel(xyz, tets, mat, bnd, np.full(len(bnd), 37.0))
    om.dt = dt if dt is not None else 0.9 * om.dt_cr()
    q = om.source(src, mode)
    T = om.initial(T0)
    if schedule is None:
        T = om.run(T, n, q)
    else:
        for k, use_src in schedule:
            T = om.run(T, k, q if use_src else None)
    return om, q, T


def gpu_handle(xyz, tets, mat, bnd, dt, prec, **opt):
    h = ff.Handle(xyz, tets, mat, 37.0, bnd, np.full(len(bnd), 37.0), dt=dt,
                  precision=prec, **opt)
    h.precompute()
    return h


def print_case(name, err, extra=""):
    print(f"[parity] {name}: max|dT|={err:.3e} K {extra}", flush=True)


# --------------------------------------------------------------------------
def test_config1_fp64_and_lambda():
    s = sc.config1()
    om = oracle.build_model(s)
    lam_o = om.geometry_lambda(method="dense")
    dtcr_o, _ = dense.critical_dt_from_lambda(lam_o, om.mat)
    n, dt = sc.steps_for(s.t_end, dtcr_o)
    assert n == 263
    om.dt = dt
    q = om.source(s.sources, s.source_mode)
    T_ref = om.run(om.initial(37.0), n, q)
    h = gpu_handle(s.xyz, s.tets, s.materials, s.dir_nodes, dt, ff.FP64)
    info = h.info()
    lam_g = info["lambda_geometry"]
    closed = cf.kuhn_cube_lambda(10, 1e-3)
    print(f"[lambda] gpu={lam_g:.10e} oracle={lam_o:.10e} closed={closed:.10e} "
          f"iters={info['lanczos_iterations']}", flush=True)
    assert lam_g >= (1 - 1e-4) * closed
    assert lam_g <= (1 + 1e-3) * closed
    _, dtcr_g = h.dt()
    assert abs(dtcr_g / dtcr_o - 1) < 1e-3
    h.set_gaussian_sources(s.sources, s.source_mode)
    assert np.max(np.abs(h.read_source() - q)) <= 1e-14 * q.max()
    h.step(n)
    T = h.read_T()
    err = np.max(np.abs(T - T_ref))
    print_case("config1 fp64", err, f"centre={T.max():.4f}")
    assert err <= 1e-10
    assert 50.0 < T.max() < 51.0


def test_config1_fp32c():
    s = sc.config1()
    om = oracle.build_model(s)
    dtcr_o, _ = dense.critical_dt_from_lambda(om.geometry_lambda("dense"), om.mat)
    n, dt = sc.steps_for(s.t_end, dtcr_o)
    om.dt = dt
    q = om.source(s.sources, s.source_mode)
    T_ref = om.run(om.initial(37.0), n, q)
    h = gpu_handle(s.xyz, s.tets, s.materials, s.dir_nodes, dt, ff.FP32C)
    h.set_gaussian_sources(s.sources, s.source_mode)
    h.step(n)
    err = np.max(np.abs(h.read_T() - T_ref))
    print_case("config1 fp32c", err)
    assert err <= 1e-3


@pytest.mark.parametrize("prec", [ff.FP64, ff.FP32C])
@pytest.mark.parametrize("reorder", [0, 1])
@pytest.mark.parametrize("tile", [64, 1024])
def test_td_jittered_box(prec, reorder, tile):
    xyz, tets, bnd = jittered_box(9, 7, 6, 1e-3, seed=21)
    # corner order scrambled and random numbering: orientation and order vary
    xyz, tets, bnd, _, _ = mesh.shuffle_mesh(xyz, tets, bnd, np.random.default_rng(5))
    mat = sc.td_materials()
    mat.Q_m = 3000.0
    src = np.array([[4e-3, 3e-3, 3e-3, 1.2e-3, 4e8], [7e-3, 5e-3, 2e-3, 0.6e-3, 2e8]])
    om, q, T_ref = oracle_run(xyz, tets, mat, bnd, src, sc.SOURCE_CONSISTENT, 300)
    h = gpu_handle(xyz, tets, mat, bnd, om.dt, prec, reorder=bool(reorder), tile_elems=tile)
    h.set_gaussian_sources(src, ff.SOURCE_CONSISTENT)
    qg = h.read_source()
    assert np.max(np.abs(qg - q)) <= (1e-12 if prec == ff.FP64 else 1e-6) * q.max()
    h.step(300)
    T = h.read_T()
    err = np.max(np.abs(T - T_ref))
    print_case(f"td box prec={prec} reorder={reorder} tile={tile}", err,
               f"peak={T_ref.max():.2f}")
    assert T_ref.max() > 70.0
    assert err <= TOL[prec]


@pytest.mark.parametrize("prec", [ff.FP64, ff.FP32C])
@pytest.mark.parametrize("xcd", [0, 1])
def test_single_tile_nodes_and_xcd_remap(prec, xcd):
    """Reordered layouts number the nodes of a single tile first and read
    their one tile sum at the node's own index (Eq 11 with one term); the
    nodal update takes whole 512-node blocks of them in one load round, with
    or without the XCD remap of its blocks.  The box is large enough for
    several such blocks and a mixed one."""
    xyz, tets, bnd = jittered_box(30, 24, 20, 1e-3, seed=33)
    xyz, tets, bnd, _, _ = mesh.shuffle_mesh(xyz, tets, bnd, np.random.default_rng(9))
    mat = sc.td_materials()
    src = np.array([[12e-3, 10e-3, 8e-3, 3e-3, 5e6], [22e-3, 14e-3, 12e-3, 2e-3, 4e6]])
    om, q, T_ref = oracle_run(xyz, tets, mat, bnd, src, sc.SOURCE_CONSISTENT, 200)
    h = gpu_handle(xyz, tets, mat, bnd, om.dt, prec, reorder=True, tile_elems=2048,
                   xcd=bool(xcd))
    info = h.info()
    n_single = info["n_single_tile_nodes"]
    assert 3 * 512 <= n_single < len(xyz)
    h.set_gaussian_sources(src, ff.SOURCE_CONSISTENT)
    h.step(200)
    T = h.read_T()
    err = np.max(np.abs(T - T_ref))
    print_case(f"single-tile nodes prec={prec} xcd={xcd}", err,
               f"single={n_single}/{len(xyz)} tiles={info['n_tiles']}")
    assert T_ref.max() > 60.0
    assert err <= TOL[prec]


@pytest.mark.parametrize("xcd", [0, 1])
def test_one_tile_mesh_has_only_single_tile_nodes(xcd):
    """A mesh that fits one tile: every node is a single-tile node (the
    partial of each at its own index, no slot list read), including the
    last, partly filled block of the nodal update."""
    xyz, tets, bnd = jittered_box(7, 6, 5, 1e-3, seed=41)
    xyz, tets, bnd, _, _ = mesh.shuffle_mesh(xyz, tets, bnd, np.random.default_rng(3))
    mat = sc.td_materials()
    src = np.array([[3e-3, 3e-3, 2.5e-3, 1.5e-3, 2e7]])
    om, q, T_ref = oracle_run(xyz, tets, mat, bnd, src, sc.SOURCE_CONSISTENT, 150)
    h = gpu_handle(xyz, tets, mat, bnd, om.dt, ff.FP64, reorder=True, tile_elems=2048,
                   xcd=bool(xcd))
    info = h.info()
    assert info["n_tiles"] == 1 and info["n_single_tile_nodes"] == len(xyz)
    h.set_gaussian_sources(src, ff.SOURCE_CONSISTENT)
    h.step(150)
    err = np.max(np.abs(h.read_T() - T_ref))
    print_case(f"one-tile mesh xcd={xcd}", err, f"nodes={len(xyz)} peak={T_ref.max():.2f}")
    assert T_ref.max() > 45.0
    assert err <= TOL[ff.FP64]


@pytest.mark.parametrize("prec", [ff.FP64, ff.FP32C])
def test_wide_tiles_keep_16_bit_corner_ids(prec):
    """Tiles of more than 1024 nodes keep 16-bit local corner ids (smaller
    tiles use the packed 10-bit form); both forms must give the oracle's
    temperatures."""
    xyz, tets, bnd = jittered_box(16, 16, 8, 1e-3, seed=23)
    mat = sc.td_materials()
    src = np.array([[8e-3, 8e-3, 4e-3, 2e-3, 4e8]])
    om, q, T_ref = oracle_run(xyz, tets, mat, bnd, src, sc.SOURCE_CONSISTENT, 200)
    for reorder, tile in ((0, 4096), (1, 1024)):
        h = gpu_handle(xyz, tets, mat, bnd, om.dt, prec, reorder=bool(reorder), tile_elems=tile)
        wide = h.info()["max_tile_nodes"]
        h.set_gaussian_sources(src, ff.SOURCE_CONSISTENT)
        h.step(200)
        err = float(np.max(np.abs(h.read_T() - T_ref)))
        print_case(f"tile nodes {wide} prec={prec} reorder={reorder} tile={tile}", err,
                   f"peak={T_ref.max():.2f}")
        assert (wide > 1024) == (tile == 4096)
        assert err <= TOL[prec]
        h.close()


def test_nodal_and_consistent_sources_fp64():
    xyz, tets, bnd = jittered_box(8, 8, 8, 1e-3, seed=3)
    mat = sc.td_materials()
    om = oracle.OracleModel(xyz, tets, mat, bnd, np.full(len(bnd), 37.0))
    h = gpu_handle(xyz, tets, mat, bnd, -0.9, ff.FP64)
    for src in ([[4e-3, 4e-3, 4e-3, 0.3e-3, 1e9]], [[1e-3, 2e-3, 7e-3, 2e-3, 1e7],
                                                    [6e-3, 6e-3, 1e-3, 1e-3, 5e7]]):
        for mode in (ff.SOURCE_NODAL, ff.SOURCE_CONSISTENT):
            h.set_gaussian_sources(src, mode)
            qg = h.read_source()
            qo = om.source(src, mode)
            assert np.max(np.abs(qg - qo)) <= 1e-13 * np.abs(qo).max(), mode


def test_lambda_matches_oracle_on_jittered_mesh():
    xyz, tets, bnd = jittered_box(14, 12, 10, 1e-3, seed=9)
    mat = sc.td_materials()
    om = oracle.OracleModel(xyz, tets, mat, bnd, np.full(len(bnd), 37.0))
    lam_o = om.geometry_lambda()
    h = gpu_handle(xyz, tets, mat, bnd, -0.9, ff.FP32C)
    lam_g = h.info()["lambda_geometry"]
    print(f"[lambda] jittered gpu={lam_g:.8e} oracle={lam_o:.8e}", flush=True)
    assert lam_g >= (1 - 1e-4) * lam_o
    assert lam_g <= (1 + 1e-3) * lam_o
    dt, dtcr = h.dt()
    assert abs(dt - 0.9 * dtcr) <= 1e-15 * dt


@pytest.mark.parametrize("dims", [(2, 2, 2), (3, 2, 2), (3, 3, 3), (4, 3, 3), (5, 4, 4)])
def test_lambda_on_few_free_nodes(dims):
    """Boxes with 1, 2, 8, 12 and 36 free nodes: the Lanczos recurrence breaks
    down once the Krylov space holds every free node, before, at or after a
    point where the host reads the coefficients, and must then return the
    exact top eigenvalue of the (dense) oracle."""
    xyz, tets, bnd = jittered_box(*dims, 1e-3, seed=17)
    mat = sc.td_materials()
    om = oracle.OracleModel(xyz, tets, mat, bnd, np.full(len(bnd), 37.0))
    lam_o = om.geometry_lambda()
    h = gpu_handle(xyz, tets, mat, bnd, -0.9, ff.FP64)
    inf = h.info()
    lam_g = inf["lambda_geometry"]
    n_free = len(xyz) - len(bnd)
    print(f"[lambda] {dims}: {n_free} free nodes, {inf['lanczos_iterations']} iterations, "
          f"gpu={lam_g:.12e} oracle={lam_o:.12e}", flush=True)
    assert inf["lanczos_iterations"] <= max(n_free, 1) + 16
    if inf["lanczos_iterations"] >= n_free:  # broke down: exact
        assert abs(lam_g - lam_o) <= 1e-8 * lam_o
    else:  # converged first: an upper bound
        assert (1 - 1e-10) * lam_o <= lam_g <= (1 + 1e-6) * lam_o
    h.close()


def test_bitwise_determinism_and_checkpoint():
    xyz, tets, bnd = jittered_box(10, 8, 7, 1e-3, seed=4)
    mat = sc.td_materials()
    src = [[5e-3, 4e-3, 3e-3, 1e-3, 5e8]]
    outs = []
    for _ in range(2):
        h = gpu_handle(xyz, tets, mat, bnd, -0.9, ff.FP32C)
        h.set_gaussian_sources(src)
        h.step(120)
        outs.append(h.read_state()[0])
    assert np.array_equal(outs[0], outs[1])
    # 70 steps, checkpoint, restore into a fresh handle, 50 more steps
    h1 = gpu_handle(xyz, tets, mat, bnd, -0.9, ff.FP32C)
    h1.set_gaussian_sources(src)
    h1.step(70)
    buf, t, n = h1.read_state()
    h2 = gpu_handle(xyz, tets, mat, bnd, -0.9, ff.FP32C)
    h2.set_gaussian_sources(src)
    h2.write_state(buf, t, n)
    h2.step(50)
    b2, t2, n2 = h2.read_state()
    assert n2 == 120 and abs(t2 - 120 * h2.dt()[0]) < 1e-9
    assert np.array_equal(b2, outs[0])
    # several calls equal one call when the source is unchanged
    h3 = gpu_handle(xyz, tets, mat, bnd, -0.9, ff.FP32C)
    h3.set_gaussian_sources(src)
    for k in (1, 33, 64, 22):
        h3.step(k)
    assert np.array_equal(h3.read_state()[0], outs[0])


def test_two_stage_heat_then_relax():
    """Heating, then relaxation with the source removed (Sec 3.1.5)."""
    xyz, tets, bnd = jittered_box(9, 8, 6, 1e-3, seed=12)
    mat = sc.td_materials()
    src = np.array([[4.5e-3, 4e-3, 3e-3, 1e-3, 6e8]])
    om, q, T_ref = oracle_run(xyz, tets, mat, bnd, src, sc.SOURCE_CONSISTENT, 0,
                              schedule=[(60, True), (240, False)])
    for prec in (ff.FP64, ff.FP32C):
        h = gpu_handle(xyz, tets, mat, bnd, om.dt, prec)
        h.set_gaussian_sources(src)
        h.step(60)
        h.set_source(None)
        h.step(240)
        err = np.max(np.abs(h.read_T() - T_ref))
        print_case(f"two-stage prec={prec}", err)
        assert err <= TOL[prec]


def test_error_paths():
    xyz, tets, bnd = jittered_box(4, 4, 4, 1e-3, seed=2)
    mat = sc.td_materials()
    # stepping before precompute
    h = ff.Handle(xyz, tets, mat, 37.0, bnd, np.full(len(bnd), 37.0), dt=-0.9)
    with pytest.raises(ff.FedFemError) as ei:
        h.step(1)
    assert ei.value.code == ff.E_NOT_PRECOMPUTED
    h.precompute()
    dt, dtcr = h.dt()
    with pytest.raises(ff.FedFemError) as ei:
        h.set_dt(1.0001 * dtcr)
    assert ei.value.code == ff.E_UNSTABLE
    # fixed dt above the critical step is refused at precompute
    h2 = ff.Handle(xyz, tets, mat, 37.0, bnd, np.full(len(bnd), 37.0), dt=1.01 * dtcr)
    with pytest.raises(ff.FedFemError) as ei:
        h2.precompute()
    assert ei.value.code == ff.E_UNSTABLE
    # degenerate element: flatten one tet; the caller's element id is named
    x3 = xyz.copy()
    t = tets[137]
    x3[t[3]] = (x3[t[0]] + x3[t[1]] + x3[t[2]]) / 3.0
    P = x3[tets]
    det = np.linalg.det(P[:, 1:] - P[:, :1])
    edges = [np.linalg.norm(P[:, a] - P[:, b], axis=1)
             for a in range(4) for b in range(a + 1, 4)]
    lmax = np.max(edges, axis=0)
    first_bad = int(np.nonzero(np.abs(det) <= 1e-12 * lmax**3)[0].min())
    h3 = ff.Handle(x3, tets, mat, 37.0, bnd, np.full(len(bnd), 37.0), dt=-0.9)
    with pytest.raises(ff.FedFemError) as ei:
        h3.precompute()
    assert ei.value.code == ff.E_DEGENERATE
    assert str(ei.value).split("degenerate tetrahedron ")[1].split()[0] == str(first_bad)
    # a runaway source is reported as divergence (kernels still finish)
    q = np.zeros(len(xyz))
    q[np.setdiff1d(np.arange(len(xyz)), bnd)[0]] = 1e9
    with pytest.raises(ff.FedFemError) as ei:
        h.step(20, q)
    assert ei.value.code == ff.E_DIVERGED


def test_read_T_device_matches_host():
    import torch
    xyz, tets, bnd = jittered_box(5, 5, 5, 1e-3, seed=6)
    h = gpu_handle(xyz, tets, sc.td_materials(), bnd, -0.9, ff.FP32C)
    h.set_gaussian_sources([[2.5e-3, 2.5e-3, 2.5e-3, 1e-3, 5e8]])
    s = torch.cuda.Stream()
    h.set_stream(s.cuda_stream)
    h.step(40)
    out = torch.empty(len(xyz), dtype=torch.float64, device="cuda")
    h.read_T_device(out)
    assert np.array_equal(out.cpu().numpy(), h.read_T())
    h.set_stream(0)


def test_config2_fp32c_fp64_vs_oracle():
    s = sc.config2()
    om = oracle.build_model(s)
    dtcr_o, _ = dense.critical_dt_from_lambda(om.geometry_lambda(), om.mat)
    n, dt = sc.steps_for(s.t_end, dtcr_o)
    om.dt = dt
    q = om.source(s.sources, s.source_mode)
    T_ref = om.run(om.initial(37.0), n, q)
    res = {}
    for prec in (ff.FP64, ff.FP32C):
        h = gpu_handle(s.xyz, s.tets, s.materials, s.dir_nodes, dt, prec)
        _, dtcr_g = h.dt()
        h.set_gaussian_sources(s.sources, s.source_mode)
        h.step(n)
        res[prec] = h.read_T()
        print(f"[lambda] config2 gpu dt_cr={dtcr_g:.8f} oracle={dtcr_o:.8f}", flush=True)
        assert dtcr_g <= dtcr_o * (1 + 1e-4)
        h.close()
    e64 = np.max(np.abs(res[ff.FP64] - T_ref))
    e32 = np.max(np.abs(res[ff.FP32C] - T_ref))
    e32_64 = np.max(np.abs(res[ff.FP32C] - res[ff.FP64]))
    print_case("config2 fp64", e64, f"steps={n} peak={T_ref.max():.2f}")
    print_case("config2 fp32c", e32, f"vs fp64 gpu {e32_64:.3e}")
    assert e64 <= 1e-9
    assert e32 <= 1e-3


def test_time_kernels_leaves_state_clock_and_dose():
    """fedfem_time_kernels times each pass from the current state without
    advancing it: the temperatures, clock and dose are unchanged, and the
    run continues bit for bit as if it had not been called."""
    xyz, tets, bnd = jittered_box(9, 8, 7, 1e-3, seed=31)
    src = np.full(len(xyz), 2e-3)
    out = []
    for timed in (False, True):
        h = gpu_handle(xyz, tets, sc.td_materials(), bnd, -0.9, ff.FP32C)
        h.set_dose(ff.DOSE_CEM43)
        h.step(40, src)
        if timed:
            T0, D0, t0 = h.read_T(), h.read_dose(), h.time()
            e_ms, n_ms = h.time_kernels(7)
            assert e_ms > 0 and n_ms > 0
            assert np.array_equal(h.read_T(), T0) and np.array_equal(h.read_dose(), D0)
            assert h.time() == t0
        h.step(30)
        out.append((h.read_T(), h.read_dose(), h.time()))
        h.close()
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    assert out[0][2] == out[1][2]
