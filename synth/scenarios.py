"""Seeded workload definitions: meshes, materials, boundary sets and sources.

Every quantity here is an input of the bio-heat problem (geometry, material
laws, Dirichlet set, Gaussian source parameters, simulated time).  Nothing in
this module evaluates the FED-FEM discretisation; converting a Gaussian power
density into nodal heat flows is done separately by each implementation.

Units: metres, seconds, kilograms, degrees Celsius, watts.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import mesh as _mesh

SEED_ROOT = 1909_05098

# Source modes for turning a Gaussian density (W/m^3) into nodal heat flows.
SOURCE_NODAL = 0       # Q_i = Q_r(x_i) * (lumped nodal volume)
SOURCE_CONSISTENT = 1  # Q_i = integral of Q_r * N_i over the mesh (quadrature)


@dataclass
class Materials:
    """Linear property laws p(T) = p0 + dp_dT * (clamp(T, T_lo, T_hi) - T_ref).

    w_b is the blood perfusion mass rate in kg/(m^3 s) (omega_b * rho_b).
    """
    rho0: float = 1060.0
    c0: float = 3600.0
    k0: float = 0.512
    drho_dT: float = 0.0
    dc_dT: float = 0.0
    dk_dT: float = 0.0
    T_ref: float = 37.0
    T_lo: float = 0.0
    T_hi: float = 100.0
    w_b: float = 0.0064 * 1000.0
    c_b: float = 4180.0
    T_a: float = 37.0
    Q_m: float = 0.0

    def as_tuple(self):
        return (self.rho0, self.c0, self.k0, self.drho_dT, self.dc_dT,
                self.dk_dT, self.T_ref, self.T_lo, self.T_hi, self.w_b,
                self.c_b, self.T_a, self.Q_m)


@dataclass
class Scenario:
    name: str
    xyz: np.ndarray
    tets: np.ndarray
    materials: Materials
    dir_nodes: np.ndarray
    dir_T: np.ndarray
    T0: float
    sources: np.ndarray          # [n_src, 5]: x, y, z, sigma, Q0
    source_mode: int
    t_end: float
    dt_fraction: float = 0.9     # dt = t_end / ceil(t_end / (f * dt_cr))
    n_steps: int | None = None   # fixed step count (overrides t_end logic)
    h: float = 0.0
    semi_axes: tuple | None = None
    extra: dict = field(default_factory=dict)

    @property
    def n_nodes(self):
        return len(self.xyz)

    @property
    def n_tets(self):
        return len(self.tets)


def seed_rng(*keys):
    return np.random.default_rng(np.random.SeedSequence([SEED_ROOT, *keys]))


def steps_for(t_end, dt_cr, fraction=0.9):
    """Step count and step size that land exactly on t_end with dt <= f*dt_cr."""
    n = int(np.ceil(t_end / (fraction * dt_cr) - 1e-12))
    n = max(n, 1)
    return n, t_end / n


def _sample_in_ellipsoid(rng, semi_axes, scale=1.0, centre=(0, 0, 0)):
    a, b, c = (s * scale for s in semi_axes)
    while True:
        p = rng.uniform(-1.0, 1.0, size=3)
        if p @ p <= 1.0:
            return np.array([centre[0] + a * p[0], centre[1] + b * p[1],
                             centre[2] + c * p[2]])


def _interior_point(rng, semi_axes, margin):
    """Uniform point of the ellipsoid shrunk by `margin` along every axis.

    The shrunk ellipsoid lies inside the set of points at distance >= margin
    from the original surface.
    """
    inner = tuple(s - margin for s in semi_axes)
    return _sample_in_ellipsoid(rng, inner)


def config1():
    """1 cm cube, 10^3 Kuhn cubes (6000 tets, 1331 nodes), constant properties."""
    h = 1.0e-3
    xyz, tets = _mesh.kuhn_box(10, 10, 10, h)
    bnd = _mesh.boundary_nodes_by_faces(len(xyz), tets)
    mat = Materials(rho0=1060.0, c0=3600.0, k0=0.512, w_b=0.0064 * 1000.0,
                    c_b=4180.0, T_a=37.0, Q_m=0.0, T_lo=0.0, T_hi=100.0)
    src = np.array([[5e-3, 5e-3, 5e-3, 1.5e-3, 5.0e6]])
    return Scenario("config1_cube_fp64", xyz, tets, mat, bnd,
                    np.full(len(bnd), 37.0), 37.0, src, SOURCE_NODAL, 300.0,
                    h=h)


def td_materials(k0=0.512, w_b=0.0064 * 1000.0):
    """k(T)=k0(1+0.0013(T-37)), c(T)=3600(1-0.0005(T-37)), window [0,100] C."""
    return Materials(rho0=1060.0, c0=3600.0, k0=k0, drho_dT=0.0,
                     dc_dT=-0.0005 * 3600.0, dk_dT=0.0013 * k0, T_ref=37.0,
                     T_lo=0.0, T_hi=100.0, w_b=w_b, c_b=4180.0, T_a=37.0,
                     Q_m=0.0)


ELLIPSOID_AXES = (75e-3, 50e-3, 40e-3)


def config2(h=1.2e-3):
    """Ellipsoid 75x50x40 mm, jittered lattice h=1.2 mm, TD properties, 600 s."""
    rng = seed_rng(2)
    xyz, tets, bnd = _mesh.jittered_ellipsoid(ELLIPSOID_AXES, h, rng)
    sigma = 4e-3
    p = _interior_point(rng, ELLIPSOID_AXES, 3 * sigma)
    src = np.array([[p[0], p[1], p[2], sigma, 2.0e7]])
    return Scenario("config2_ellipsoid_h1.2", xyz, tets, td_materials(), bnd,
                    np.full(len(bnd), 37.0), 37.0, src, SOURCE_CONSISTENT,
                    600.0, h=h, semi_axes=ELLIPSOID_AXES)


def config3(order="random", h=0.6e-3, n_steps=1000):
    """Ellipsoid at h=0.6 mm, two Gaussian sources, 1000 steps.

    The mesh is handed over in a seeded random node and element order; the
    library's own Morton reordering is what separates the two orderings.
    """
    rng = seed_rng(3)
    xyz, tets, bnd = _mesh.jittered_ellipsoid(ELLIPSOID_AXES, h, rng)
    sigma = 4e-3
    srcs = []
    for _ in range(2):
        p = _interior_point(rng, ELLIPSOID_AXES, 3 * sigma)
        srcs.append([p[0], p[1], p[2], sigma, 2.0e7])
    if order == "random":
        xyz, tets, bnd, _, _ = _mesh.shuffle_mesh(xyz, tets, bnd,
                                                  seed_rng(3, 1))
    return Scenario(f"config3_ellipsoid_h{h * 1e3:g}", xyz, tets,
                    td_materials(), bnd, np.full(len(bnd), 37.0), 37.0,
                    np.array(srcs), SOURCE_CONSISTENT, 0.0, n_steps=n_steps,
                    h=h, semi_axes=ELLIPSOID_AXES)


def hex_ellipsoid(order="random", h=0.6e-3, n_steps=1000):
    """The 75x50x40 mm ellipsoid of config3 as eight-node hexahedra: the same
    lattice (h = 0.6 mm), TD properties, surface held at 37 C, two seeded
    Gaussian sources (nodal conversion), 1000 steps.  Handed over in seeded
    random node, element and corner order."""
    rng = seed_rng(5)
    xyz, hexes, bnd = _mesh.jittered_hex_ellipsoid(ELLIPSOID_AXES, h, rng)
    sigma = 4e-3
    srcs = []
    for _ in range(2):
        p = _interior_point(rng, ELLIPSOID_AXES, 3 * sigma)
        srcs.append([p[0], p[1], p[2], sigma, 2.0e7])
    if order == "random":
        xyz, hexes, bnd, _, _ = _mesh.shuffle_hex_mesh(xyz, hexes, bnd, seed_rng(5, 1))
    return Scenario(f"hex_ellipsoid_h{h * 1e3:g}", xyz, hexes, td_materials(), bnd,
                    np.full(len(bnd), 37.0), 37.0, np.array(srcs), SOURCE_NODAL, 0.0,
                    n_steps=n_steps, h=h, semi_axes=ELLIPSOID_AXES)


def sweep_params(j):
    """Parameters of planning-sweep scenario j (no mesh built)."""
    rng = seed_rng(4, j)
    axes = tuple(rng.uniform(30e-3, 80e-3, size=3))
    n_target = float(np.exp(rng.uniform(np.log(20e3), np.log(400e3))))
    vol = 4.0 / 3.0 * np.pi * axes[0] * axes[1] * axes[2]
    h = (6.0 * vol / n_target) ** (1.0 / 3.0)
    k0 = rng.uniform(0.45, 0.6)
    omega_b = rng.uniform(0.002, 0.02)
    q0 = rng.uniform(5e6, 3e7)
    sigma = rng.uniform(2e-3, 6e-3)
    pos = _sample_in_ellipsoid(rng, axes, 0.7)
    mesh_seed = int(rng.integers(0, 2**31 - 1))
    return dict(axes=axes, n_target=n_target, h=h, k0=k0, omega_b=omega_b,
                q0=q0, sigma=sigma, pos=pos, mesh_seed=mesh_seed)


def sweep_scenario(j, mesh_variant=1):
    """Planning-sweep scenario j: seeded ellipsoid, TD properties, 300 s.

    mesh_variant picks the seed of the node jitter only: two variants of one
    scenario share every parameter, the lattice, the kept elements and the
    (unjittered) surface, and differ in where the interior nodes sit."""
    p = sweep_params(j)
    rng = np.random.default_rng(np.random.SeedSequence([SEED_ROOT, 4, j, int(mesh_variant)]))
    xyz, tets, bnd = _mesh.jittered_ellipsoid(p["axes"], p["h"], rng)
    mat = td_materials(k0=p["k0"], w_b=p["omega_b"] * 1000.0)
    src = np.array([[p["pos"][0], p["pos"][1], p["pos"][2], p["sigma"],
                     p["q0"]]])
    return Scenario(f"sweep_{j}", xyz, tets, mat, bnd,
                    np.full(len(bnd), 37.0), 37.0, src, SOURCE_CONSISTENT,
                    300.0, h=p["h"], semi_axes=p["axes"], extra=p)


def paper_table_materials():
    """Two-point tissue data (37 C and 65 C) with linear interpolation."""
    return Materials(rho0=1040.0, c0=3600.0, k0=0.53,
                     drho_dT=(1000.0 - 1040.0) / 28.0,
                     dc_dT=(3800.0 - 3600.0) / 28.0,
                     dk_dT=(0.57 - 0.53) / 28.0, T_ref=37.0, T_lo=37.0,
                     T_hi=65.0, w_b=0.0, c_b=3617.0, T_a=37.0, Q_m=0.0)
