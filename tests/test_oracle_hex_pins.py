"""Pins of the FP64 hexahedral oracle (Sec 2.3.3, Eq 14, 16) against what the
mathematics fixes.  Each test says which mistake in the oracle it catches.
"""
import numpy as np

import oracle
from oracle import closed_forms as cf
from oracle import hex as ohx
from synth import mesh, scenarios as sc


def ti_materials(**kw):
    base = dict(rho0=1060.0, c0=3600.0, k0=0.512, w_b=6.4, c_b=4180.0, T_a=37.0, Q_m=0.0)
    base.update(kw)
    return sc.Materials(**base)


def jittered_hex_box(nx, ny, nz, h, seed, jitter=0.2):
    xyz, hexes = mesh.hex_box(nx, ny, nz, h)
    bnd = mesh.box_surface_nodes(nx, ny, nz)
    rng = np.random.default_rng(seed)
    mask = np.ones(len(xyz), bool)
    mask[bnd] = False
    xyz[mask] += rng.uniform(-jitter * h, jitter * h, (mask.sum(), 3))
    return xyz, hexes, bnd


def model(xyz, hexes, mat, dir_nodes=(), dir_T=(), frac=0.9):
    m = ohx.HexModel(xyz, hexes, oracle.mat_vector(mat), dir_nodes, dir_T)
    m.dt = frac * m.dt_cr("dense")
    return m


def test_uniform_field_invariant():
    """Zero row sums of A_e (Eq 16) and perfusion vanishing at T_a: a
    uniform field stays put.  Catches a non-zero-sum element matrix or a
    sign slip in the perfusion term."""
    xyz, hexes, bnd = jittered_hex_box(5, 4, 3, 1e-3, seed=1)
    m = model(xyz, hexes, sc.td_materials(), bnd, np.full(len(bnd), 37.0))
    T = m.run(m.initial(37.0), 500)
    assert np.max(np.abs(T - 37.0)) <= 1e-12


def test_element_volume_and_gradients_on_a_brick():
    """A rectangular brick hx x hy x hz: V = hx hy hz and, at the centre,
    dN_a/dx = xi_a / (4 hx) (and likewise in y, z).  Catches a wrong weight
    (the 8 of Eq 14), a transposed Jacobian or a wrong node order."""
    xyz, hexes = mesh.hex_box(1, 1, 1, (2e-3, 3e-3, 5e-3))
    A, V, grad = ohx.element_matrices(xyz, hexes)
    assert abs(V[0] - 30e-9) <= 1e-22
    expect = ohx.NAT / (4.0 * np.array([2e-3, 3e-3, 5e-3]))
    assert np.allclose(grad[0], expect, rtol=1e-13, atol=0)
    # A = V grad grad^T is symmetric with zero row sums
    assert np.allclose(A[0], A[0].T, rtol=0, atol=1e-18)
    assert np.max(np.abs(A[0].sum(axis=1))) <= 1e-18


def test_orientation_does_not_matter():
    """A mirrored node order (det J < 0) gives the same element matrix
    (|det J| in V_e)."""
    xyz, hexes, _ = jittered_hex_box(3, 3, 3, 1e-3, seed=4)
    A, V, _ = ohx.element_matrices(xyz, hexes)
    mirrored = hexes[:, [4, 5, 6, 7, 0, 1, 2, 3]]
    A2, V2, _ = ohx.element_matrices(xyz, mirrored)
    perm = [4, 5, 6, 7, 0, 1, 2, 3]
    assert np.allclose(V, V2, rtol=1e-14, atol=0)
    assert np.allclose(A[:, perm][:, :, perm], A2, rtol=1e-12, atol=1e-18)


def test_patch_test_on_parallelepipeds():
    """Linear fields are reproduced (the patch test of Sec 3.1.1) on a mesh
    of parallelepipeds, where one-point integration of grad N at the centre is
    exact: constant k, no perfusion, the boundary held at a + g.x and the
    interior starting there must stay there.  Catches wrong gradients or a
    wrong gather."""
    xyz, hexes = mesh.hex_box(6, 5, 4, 1e-3)
    Mx = np.array([[1.0, 0.25, -0.1], [0.1, 0.9, 0.2], [0.05, -0.15, 1.1]])
    xyz = xyz @ Mx.T + np.array([0.01, -0.02, 0.005])
    bnd = mesh.box_surface_nodes(6, 5, 4)
    g = np.array([300.0, -150.0, 80.0])
    lin = 37.0 + xyz @ g
    mat = ti_materials(w_b=0.0)
    m = model(xyz, hexes, mat, bnd, lin[bnd])
    T = m.run(lin.copy(), 200)
    assert np.max(np.abs(T - lin)) <= 1e-10


def test_slab_discrete_closed_form():
    """On a regular box with the x = 0 and x = L faces held and the other
    faces insulated, the one-point hexahedron reduces to the 3-point scheme
    in x (the averages over the four parallel edges are exact for fields
    constant in y and z), so every column follows the discrete Pennes
    solution.  Catches a wrong sign of F, a wrong lumped capacity, or
    perfusion and source terms off by a factor."""
    nx, L = 12, 12e-3
    h = L / nx
    xyz, hexes = mesh.hex_box(nx, 3, 2, h)
    x = xyz[:, 0]
    j = np.rint(x / h).astype(int)
    ends = np.nonzero((j == 0) | (j == nx))[0]
    mat = ti_materials()
    m = ohx.HexModel(xyz, hexes, oracle.mat_vector(mat), ends, np.full(len(ends), 37.0))
    rho_c = 1060.0 * 3600.0
    alpha = 0.512 / rho_c
    mrate = 6.4 * 4180.0 / rho_c
    m.dt = 0.9 * 2.0 / (4.0 * alpha / h**2 + mrate)
    theta0 = 5.0 * np.sin(np.pi * x / L) + 2.0 * np.sin(3 * np.pi * x / L)
    src = 3e5 * (x / L) * (1 - x / L)
    n = 400
    T = m.run(37.0 + theta0, n, src * m.Vi)
    xg = np.arange(1, nx) * h
    expect = cf.slab_discrete(5.0 * np.sin(np.pi * xg / L) + 2.0 * np.sin(3 * np.pi * xg / L),
                              3e5 * (xg / L) * (1 - xg / L), alpha, mrate, h, m.dt, n, rho_c)
    inner = (j > 0) & (j < nx)
    assert np.max(np.abs(T[inner] - 37.0 - expect[j[inner] - 1])) <= 1e-11


def test_critical_step_eigenvalue_closed_form():
    """The geometry eigenvalue of Eq 9's pencil on a regular box with its
    surface held equals the mode maximum of the one-point stencil.  Catches
    a wrong lumped volume or element matrix scale in the critical step."""
    for dims, h in (((4, 3, 5), 1e-3), ((7, 6, 9), 0.5e-3)):
        xyz, hexes = mesh.hex_box(*dims, h)
        bnd = mesh.box_surface_nodes(*dims)
        m = ohx.HexModel(xyz, hexes, oracle.mat_vector(ti_materials()), bnd,
                         np.full(len(bnd), 37.0))
        lam = m.geometry_lambda("dense")
        assert abs(lam - cf.hex_box_lambda(*dims, h)) <= 1e-12 * lam


def test_hourglass_mode_has_zero_energy():
    """The reading of Eq 14 without hourglass control: on a regular grid the
    checkerboard field (-1)^(i+j+k) has zero gradient at every element centre,
    so it carries no conduction load (A_e T_e = 0)."""
    nx, ny, nz = 4, 3, 3
    xyz, hexes = mesh.hex_box(nx, ny, nz, 1e-3)
    K, J, I = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1),
                          indexing="ij")
    chk = ((-1.0) ** (I + J + K)).ravel()
    A, _, _ = ohx.element_matrices(xyz, hexes)
    Fe = np.einsum("eab,eb->ea", A, chk[hexes])
    assert np.max(np.abs(Fe)) <= 1e-15 * np.max(np.abs(A))


def test_element_loads_equal_assembled_matrix_and_energy_balance():
    """Eq 11: the element-level loads equal K(T) T with K assembled from
    k_e A_e (Eq 13, 17), and each step closes the energy balance
    sum_free C_i dT_i = dt [sum_free (q + Q_m V + w_b c_b V (T_a - T)) +
    sum_D F_i] (all loads sum to zero).  Catches a dropped or doubled
    element, a wrong k_e average or a term missing from Eq 19."""
    xyz, hexes, bnd = jittered_hex_box(5, 4, 4, 1e-3, seed=7)
    mat = sc.td_materials()
    mat.Q_m = 2000.0
    m = model(xyz, hexes, mat, bnd, np.full(len(bnd), 37.0))
    rng = np.random.default_rng(3)
    T = m.initial(37.0) + rng.uniform(0, 20, m.N) * ~m.is_dir
    q = m.source_nodal([[2.5e-3, 2e-3, 2e-3, 1e-3, 5e7]])
    ke = dense_k(T, m)
    K = ohx.assemble(m.N, hexes, m.A, ke)
    F = m.loads(T)
    assert np.max(np.abs(F - K @ T)) <= 1e-12 * np.max(np.abs(F))
    mv = m.m
    Tn = m.step(T, q)
    free = ~m.is_dir
    C = oracle.dense.rho_c_of(T, mv) * m.Vi
    lhs = np.sum((C * (Tn - T))[free])
    rhs = m.dt * (np.sum((q + mv[oracle.dense.M["Q_m"]] * m.Vi
                          + mv[oracle.dense.M["w_b"]] * mv[oracle.dense.M["c_b"]] * m.Vi
                          * (mv[oracle.dense.M["T_a"]] - T))[free]) + np.sum(F[~free]))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), abs(rhs))


def dense_k(T, m):
    return oracle.dense.k_of(T[m.hexes], m.m).mean(axis=1)


def test_element_order_invariance():
    """Reordering the elements changes only the order of the gather:
    results agree to rounding.  Catches loads attached to the wrong element."""
    xyz, hexes, bnd = jittered_hex_box(4, 4, 3, 1e-3, seed=9)
    mat = sc.td_materials()
    m1 = model(xyz, hexes, mat, bnd, np.full(len(bnd), 37.0))
    perm = np.random.default_rng(5).permutation(len(hexes))
    m2 = ohx.HexModel(xyz, hexes[perm], oracle.mat_vector(mat), bnd, np.full(len(bnd), 37.0))
    m2.dt = m1.dt
    q = m1.source_nodal([[2e-3, 2e-3, 1.5e-3, 1e-3, 4e8]])
    T1 = m1.run(m1.initial(37.0), 100, q)
    T2 = m2.run(m2.initial(37.0), 100, q)
    assert T1.max() > 40.0
    assert np.max(np.abs(T1 - T2)) <= 1e-10


def test_one_point_matrix_factors_through_3x3():
    """At the single integration point every corner's gradient is one 3x3
    map applied to its natural coordinates, so A_e = Xi^T S Xi with
    S = (V_e / 64) (J J^T)^-1 (J[j, i] = dx_i / dxi_j): six numbers per
    element, the form the library stores.  Checked against the oracle's
    A_e, built from B, on jittered and mirrored hexahedra; A_e has rank 3."""
    xyz, hexes, _ = jittered_hex_box(4, 3, 3, 1e-3, seed=12)
    hexes = hexes.copy()
    hexes[::2] = hexes[::2][:, [4, 5, 6, 7, 0, 1, 2, 3]]
    A, V, _ = ohx.element_matrices(xyz, hexes)
    X = xyz[hexes]                                       # [E, 8, 3]
    Jn = np.einsum("aj,eai->eji", ohx.NAT / 8.0, X)     # dx_i / dxi_j
    S = V[:, None, None] / 64.0 * np.linalg.inv(Jn @ np.transpose(Jn, (0, 2, 1)))
    A2 = np.einsum("aj,ejk,bk->eab", ohx.NAT, S, ohx.NAT)
    assert np.max(np.abs(A2 - A)) <= 1e-12 * np.max(np.abs(A))
    assert np.all(np.linalg.matrix_rank(A, tol=1e-9 * np.abs(A).max()) == 3)


def test_consistent_source_reduces_to_lumped_for_uniform_density():
    """On parallelepipeds (constant det J) the integral of N_a over an
    element is V_e / 8, so a uniform density (a Gaussian far wider than the
    mesh) gives Q_i = Q V_i, the lumped volume.  Catches a wrong shape
    function, weight or Jacobian in the quadrature."""
    xyz, hexes = mesh.hex_box(4, 3, 3, 1e-3)
    Mx = np.array([[1.0, 0.2, -0.1], [0.05, 0.9, 0.15], [0.1, -0.2, 1.2]])
    xyz = xyz @ Mx.T
    m = ohx.HexModel(xyz, hexes, oracle.mat_vector(sc.td_materials()))
    q = m.source_consistent([[1e-3, 1e-3, 1e-3, 1e3, 5e6]])
    assert np.max(np.abs(q - 5e6 * m.Vi)) <= 1e-9 * np.max(5e6 * m.Vi)


def test_consistent_source_total_power_and_relabelling():
    """Summed over the nodes the loads integrate the density over the box
    (N_a sum to one): for a Gaussian well inside a regular box that is the
    product of erf terms, to the rule's error.  Relabelling the corners of
    every element changes nothing.  Catches lost weight or an orientation-
    dependent Jacobian."""
    from math import erf, sqrt, pi
    n, h = 8, 1e-3
    xyz, hexes = mesh.hex_box(n, n, n, h)
    c, sg, Q0 = np.array([4.1e-3, 3.8e-3, 4.3e-3]), 1.2e-3, 7e6
    m = ohx.HexModel(xyz, hexes, oracle.mat_vector(sc.td_materials()))
    q = m.source_consistent([[*c, sg, Q0]])
    exact = Q0
    for ax in range(3):
        lo, hi = (0.0 - c[ax]) / (sqrt(2) * sg), (n * h - c[ax]) / (sqrt(2) * sg)
        exact *= sg * sqrt(pi / 2) * (erf(hi) - erf(lo))
    assert abs(q.sum() - exact) <= 1e-5 * exact
    rel = hexes[:, [5, 6, 7, 4, 1, 2, 3, 0]]    # a turn with top and bottom swapped
    m2 = ohx.HexModel(xyz, rel, oracle.mat_vector(sc.td_materials()))
    assert np.max(np.abs(m2.source_consistent([[*c, sg, Q0]]) - q)) <= 1e-12 * q.max()


def test_quad_flux_loads_on_parallelograms():
    """On a planar parallelogram each corner receives a quarter of q |f|
    (the bilinear shape functions integrate to |f| / 4), so the loads sum
    to q |f|, whatever the corner the list starts at and its direction; unit
    flux on two faces of a regular box sums to their area.  Catches a wrong
    area element, shape function or gather."""
    xyz = np.array([[0.0, 0.0, 0.0], [2e-3, 0.5e-3, 0.0], [2.7e-3, 3.5e-3, 0.0],
                    [0.7e-3, 3.0e-3, 0.0], [1e-3, 1e-3, 1e-3]])
    face = np.array([[0, 1, 2, 3]])
    area = np.linalg.norm(np.cross(xyz[1] - xyz[0], xyz[3] - xyz[0]))
    q = ohx.flux_loads_quad(xyz, face, [3e4])
    assert np.max(np.abs(q[:4] - 3e4 * area / 4)) <= 1e-12 * 3e4 * area and q[4] == 0.0
    # a corner order turned and reversed gives the same loads
    for f in ([[1, 2, 3, 0]], [[3, 2, 1, 0]]):
        assert np.max(np.abs(ohx.flux_loads_quad(xyz, np.array(f), [3e4]) - q)) <= 1e-12 * q.max()
    # unit flux on the six faces of a regular box: total = surface area
    n, h = 3, 1e-3
    bx, _ = mesh.hex_box(n, n, n, h)
    nid = lambda i, j, k: i + (n + 1) * (j + (n + 1) * k)
    quads = []
    for a in range(n):
        for b in range(n):
            quads += [[nid(a, b, 0), nid(a + 1, b, 0), nid(a + 1, b + 1, 0), nid(a, b + 1, 0)],
                      [nid(a, 0, b), nid(a + 1, 0, b), nid(a + 1, 0, b + 1), nid(a, 0, b + 1)]]
    tot = ohx.flux_loads_quad(bx, np.array(quads), np.ones(len(quads))).sum()
    assert abs(tot - 2 * (n * h) ** 2) <= 1e-15
