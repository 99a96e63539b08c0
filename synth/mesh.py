"""Seeded synthetic tetrahedral meshes.

This module only places points and lists connectivity; it holds none of the
FED-FEM arithmetic (no Jacobians, volumes, element matrices or lumping).  Both
the FP64 CPU oracle and the GPU library consume what it produces.

Meshes are built on the Kuhn (Freudenthal) triangulation of a cubic lattice:
every lattice cube is split into six tetrahedra that all share the cube's main
diagonal from corner (0,0,0) to corner (1,1,1).  Neighbouring cubes then match
face to face, so the mesh is conforming.  Coordinates are in metres.
"""
from __future__ import annotations

import itertools

import numpy as np

# The six Kuhn tetrahedra of a unit cube: one per ordering (a, b, c) of the
# three axes; vertices are 0, e_a, e_a+e_b, e_a+e_b+e_c = (1,1,1).
_KUHN_PATHS = [np.array(p) for p in itertools.permutations(range(3))]

# In the Kuhn triangulation an interior lattice vertex is shared by exactly
# 24 tetrahedra (6 from the two cubes where it is the (0,0,0) or (1,1,1)
# corner, 2 from each of the six other cubes).
KUHN_VERTEX_DEGREE = 24


def _kuhn_corner_offsets():
    """Integer lattice offsets (6 tets x 4 vertices x 3 axes)."""
    out = np.zeros((6, 4, 3), dtype=np.int64)
    for t, perm in enumerate(_KUHN_PATHS):
        cur = np.zeros(3, dtype=np.int64)
        out[t, 0] = cur
        for s, ax in enumerate(perm):
            cur = cur.copy()
            cur[ax] += 1
            out[t, s + 1] = cur
    return out


KUHN_OFFSETS = _kuhn_corner_offsets()


def kuhn_box(nx, ny, nz, h, origin=(0.0, 0.0, 0.0)):
    """Box of nx*ny*nz cubes of edge h, each split into 6 Kuhn tetrahedra.

    Returns (xyz float64[N,3], tets int32[E,4]) with
    N = (nx+1)(ny+1)(nz+1) and E = 6 nx ny nz.  Node (i,j,k) has index
    i + (nx+1)*(j + (ny+1)*k).
    """
    nx, ny, nz = int(nx), int(ny), int(nz)
    hx, hy, hz = (h, h, h) if np.isscalar(h) else h
    i = np.arange(nx + 1)
    j = np.arange(ny + 1)
    k = np.arange(nz + 1)
    K, J, I = np.meshgrid(k, j, i, indexing="ij")
    xyz = np.stack([origin[0] + I.ravel() * hx,
                    origin[1] + J.ravel() * hy,
                    origin[2] + K.ravel() * hz], axis=1).astype(np.float64)
    ci, cj, ck = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz),
                             indexing="ij")
    cubes = np.stack([ci.ravel(), cj.ravel(), ck.ravel()], axis=1)
    # order cubes by (k, j, i) so the element order follows the node order
    cubes = cubes[np.lexsort((cubes[:, 0], cubes[:, 1], cubes[:, 2]))]
    lat = cubes[:, None, None, :] + KUHN_OFFSETS[None, :, :, :]
    nid = lat[..., 0] + (nx + 1) * (lat[..., 1] + (ny + 1) * lat[..., 2])
    tets = nid.reshape(-1, 4).astype(np.int32)
    return xyz, tets


def hex_box(nx, ny, nz, h, origin=(0.0, 0.0, 0.0)):
    """Box of nx*ny*nz cubes of edge h as eight-node hexahedra.

    Node (i,j,k) has index i + (nx+1)*(j + (ny+1)*k) (as kuhn_box).  Each
    hexahedron lists its bottom face (k) counter-clockwise seen from +z,
    starting at its (i,j) corner, then the top face (k+1) in the same order.
    Elements are ordered by (k, j, i).  Returns (xyz float64[N,3],
    hexes int32[E,8]).
    """
    nx, ny, nz = int(nx), int(ny), int(nz)
    hx, hy, hz = (h, h, h) if np.isscalar(h) else h
    K, J, I = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1),
                          indexing="ij")
    xyz = np.stack([origin[0] + I.ravel() * hx, origin[1] + J.ravel() * hy,
                    origin[2] + K.ravel() * hz], axis=1).astype(np.float64)
    ck, cj, ci = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ci, cj, ck = ci.ravel(), cj.ravel(), ck.ravel()

    def nid(i, j, k):
        return i + (nx + 1) * (j + (ny + 1) * k)

    corners = [(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0),
               (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)]
    hexes = np.stack([nid(ci + a, cj + b, ck + c) for a, b, c in corners], axis=1)
    return xyz, hexes.astype(np.int32)


def box_surface_nodes(nx, ny, nz):
    """Node ids (index rule of kuhn_box / hex_box) on the surface of the box."""
    K, J, I = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1),
                          indexing="ij")
    on = (I == 0) | (I == nx) | (J == 0) | (J == ny) | (K == 0) | (K == nz)
    return np.nonzero(on.ravel())[0].astype(np.int32)


def boundary_nodes_by_faces(n_nodes, tets):
    """Nodes lying on a triangle that belongs to exactly one tetrahedron."""
    tets = np.asarray(tets, dtype=np.int64)
    faces = np.concatenate([tets[:, [1, 2, 3]], tets[:, [0, 2, 3]],
                            tets[:, [0, 1, 3]], tets[:, [0, 1, 2]]])
    faces.sort(axis=1)
    order = np.lexsort((faces[:, 2], faces[:, 1], faces[:, 0]))
    f = faces[order]
    same_next = np.all(f[1:] == f[:-1], axis=1)
    dup = np.zeros(len(f), dtype=bool)
    dup[1:] |= same_next
    dup[:-1] |= same_next
    mask = np.zeros(n_nodes, dtype=bool)
    mask[f[~dup].ravel()] = True
    return np.nonzero(mask)[0].astype(np.int32)


def boundary_faces(tets):
    """Triangles (sorted node ids) that belong to exactly one tetrahedron."""
    tets = np.asarray(tets, dtype=np.int64)
    faces = np.concatenate([tets[:, [1, 2, 3]], tets[:, [0, 2, 3]],
                            tets[:, [0, 1, 3]], tets[:, [0, 1, 2]]])
    faces.sort(axis=1)
    uniq, count = np.unique(faces, axis=0, return_counts=True)
    return uniq[count == 1].astype(np.int32)


def boundary_nodes_by_degree(n_nodes, tets):
    """Boundary nodes of a sub-mesh of a Kuhn lattice.

    A kept lattice vertex is interior exactly when all 24 tetrahedra of its
    star are kept; if some are missing, a face shared by a kept and a missing
    tetrahedron touches it, so it lies on the boundary surface.
    """
    deg = np.bincount(np.asarray(tets).ravel(), minlength=n_nodes)
    return np.nonzero(deg < KUHN_VERTEX_DEGREE)[0].astype(np.int32)


def jittered_ellipsoid(semi_axes, h, rng, jitter=0.2, centre=(0.0, 0.0, 0.0)):
    """Ellipsoid filled with a Kuhn lattice of spacing h, interior nodes jittered.

    A lattice tetrahedron is kept when its vertex mean lies inside the
    ellipsoid (x/a)^2 + (y/b)^2 + (z/c)^2 <= 1, which gives a stair-stepped
    surface.  Unused lattice nodes are dropped.  Every node that is not on the
    boundary surface is moved by an independent U[-jitter*h, jitter*h] offset
    on each axis.

    Returns (xyz float64[N,3], tets int32[E,4], boundary int32[B]).
    """
    a, b, c = (float(s) for s in semi_axes)
    n = [int(np.ceil(s / h)) + 1 for s in (a, b, c)]
    nx, ny, nz = 2 * n[0], 2 * n[1], 2 * n[2]
    org = (centre[0] - n[0] * h, centre[1] - n[1] * h, centre[2] - n[2] * h)
    # keep tetrahedra by their lattice-cube position without building the
    # whole box first (the box holds ~2x the ellipsoid's tetrahedra)
    kept = []
    for kz in range(nz):
        ci, cj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
        ci = ci.ravel()
        cj = cj.ravel()
        base = np.stack([ci, cj, np.full_like(ci, kz)], axis=1)
        lat = base[:, None, None, :] + KUHN_OFFSETS[None]
        cen = lat.mean(axis=2)  # (cubes, 6, 3) in lattice units
        px = (org[0] + cen[..., 0] * h - centre[0]) / a
        py = (org[1] + cen[..., 1] * h - centre[1]) / b
        pz = (org[2] + cen[..., 2] * h - centre[2]) / c
        inside = px * px + py * py + pz * pz <= 1.0
        if not inside.any():
            continue
        # order within the layer by (j, i), then tet index
        sel = lat[inside]  # (m, 4, 3)
        cube_j = np.broadcast_to(cj.reshape(-1, 1), inside.shape)[inside]
        cube_i = np.broadcast_to(ci.reshape(-1, 1), inside.shape)[inside]
        tet_k = np.broadcast_to(np.arange(6)[None, :], inside.shape)[inside]
        o = np.lexsort((tet_k, cube_i, cube_j))
        kept.append(sel[o])
    lat = np.concatenate(kept)
    gid = lat[..., 0] + (nx + 1) * (lat[..., 1] + (ny + 1) * lat[..., 2])
    used, inv = np.unique(gid.ravel(), return_inverse=True)
    tets = inv.reshape(-1, 4).astype(np.int32)
    gi = used % (nx + 1)
    gj = (used // (nx + 1)) % (ny + 1)
    gk = used // ((nx + 1) * (ny + 1))
    xyz = np.stack([org[0] + gi * h, org[1] + gj * h, org[2] + gk * h],
                   axis=1).astype(np.float64)
    bnd = boundary_nodes_by_degree(len(xyz), tets)
    if jitter:
        mask = np.ones(len(xyz), dtype=bool)
        mask[bnd] = False
        d = rng.uniform(-jitter * h, jitter * h, size=xyz.shape)
        xyz[mask] += d[mask]
    return xyz, tets, bnd


# The eight corners of a lattice cube in the hexahedral node order (bottom
# face counter-clockwise seen from +z, then the top face above it).
HEX_CORNERS = np.array([(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0),
                        (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)], dtype=np.int64)


def jittered_hex_ellipsoid(semi_axes, h, rng, jitter=0.2, centre=(0.0, 0.0, 0.0)):
    """Ellipsoid filled with lattice cubes of edge h as eight-node hexahedra.

    A cube is kept when its centre lies inside the ellipsoid; unused lattice
    nodes are dropped.  A kept node is interior exactly when all eight cubes
    around it are kept; every other node is on the boundary surface.
    Interior nodes are moved by independent U[-jitter*h, jitter*h] offsets on
    each axis.  Elements are ordered by cube (k, j, i).

    Returns (xyz float64[N,3], hexes int32[E,8], boundary int32[B]).
    """
    a, b, c = (float(s) for s in semi_axes)
    n = [int(np.ceil(s / h)) + 1 for s in (a, b, c)]
    nx, ny, nz = 2 * n[0], 2 * n[1], 2 * n[2]
    org = (centre[0] - n[0] * h, centre[1] - n[1] * h, centre[2] - n[2] * h)
    ck, cj, ci = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    px = (org[0] + (ci + 0.5) * h - centre[0]) / a
    py = (org[1] + (cj + 0.5) * h - centre[1]) / b
    pz = (org[2] + (ck + 0.5) * h - centre[2]) / c
    inside = (px * px + py * py + pz * pz <= 1.0).ravel()
    cubes = np.stack([ci.ravel()[inside], cj.ravel()[inside], ck.ravel()[inside]], axis=1)
    lat = cubes[:, None, :] + HEX_CORNERS[None]
    gid = lat[..., 0] + (nx + 1) * (lat[..., 1] + (ny + 1) * lat[..., 2])
    used, inv = np.unique(gid.ravel(), return_inverse=True)
    hexes = inv.reshape(-1, 8).astype(np.int32)
    gi = used % (nx + 1)
    gj = (used // (nx + 1)) % (ny + 1)
    gk = used // ((nx + 1) * (ny + 1))
    xyz = np.stack([org[0] + gi * h, org[1] + gj * h, org[2] + gk * h],
                   axis=1).astype(np.float64)
    deg = np.bincount(hexes.ravel(), minlength=len(xyz))
    bnd = np.nonzero(deg < 8)[0].astype(np.int32)
    if jitter:
        mask = deg == 8
        d = rng.uniform(-jitter * h, jitter * h, size=xyz.shape)
        xyz[mask] += d[mask]
    return xyz, hexes, bnd


# Corner relabellings that keep a hexahedron's topology: the four turns about
# the bottom-top axis, each also with bottom and top exchanged.
HEX_RELABELS = np.array([[(q + r) % 4 + 4 * f for q in range(4)]
                         + [(q + r) % 4 + 4 * (1 - f) for q in range(4)]
                         for f in (0, 1) for r in range(4)], dtype=np.int64)


def shuffle_hex_mesh(xyz, hexes, marked, rng):
    """shuffle_mesh for hexahedra: seeded node and element permutations, and
    each element's corners relabelled by one of HEX_RELABELS."""
    n = len(xyz)
    node_perm = rng.permutation(n)
    inv = np.empty(n, dtype=np.int64)
    inv[node_perm] = np.arange(n)
    elem_perm = rng.permutation(len(hexes))
    hx = inv[hexes[elem_perm]]
    pick = HEX_RELABELS[rng.integers(0, len(HEX_RELABELS), len(hx))]
    hx = np.take_along_axis(hx, pick, axis=1).astype(np.int32)
    return xyz[node_perm], hx, np.sort(inv[marked]).astype(np.int32), node_perm, elem_perm


def shuffle_mesh(xyz, tets, marked, rng):
    """Apply a seeded random permutation to nodes and to elements.

    `marked` is an int array of node ids (e.g. the boundary set) that is
    renumbered along with the nodes.  Returns (xyz, tets, marked, node_perm,
    elem_perm) where new node p is old node node_perm[p].
    """
    n = len(xyz)
    node_perm = rng.permutation(n)
    inv = np.empty(n, dtype=np.int64)
    inv[node_perm] = np.arange(n)
    elem_perm = rng.permutation(len(tets))
    xyz2 = xyz[node_perm]
    tets2 = inv[tets[elem_perm]].astype(np.int32)
    # permute the corner order of each element too, so nothing downstream may
    # rely on the lattice's corner pattern
    cperm = np.argsort(rng.random((len(tets2), 4)), axis=1)
    tets2 = np.take_along_axis(tets2, cperm, axis=1)
    marked2 = np.sort(inv[marked]).astype(np.int32)
    return xyz2, tets2, marked2, node_perm, elem_perm


def flat_fan(m, radius, height, rng):
    """m flat tetrahedra sharing node 0 (the origin).

    Element i is (0, a_i, b_i, c_i) with its own base triangle: an
    equilateral triangle of circumradius `radius` in the plane
    z = -height, centred below node 0 and turned by 2 pi i / m plus a small
    seeded angle.  The elements overlap (the list is not a conforming mesh),
    which is allowed: each is a valid, non-degenerate tetrahedron.  With
    height << radius node 0 sits close to every opposite face, and its m
    corners all fall into one tile of the library's layout.  Returns
    (xyz [1 + 3m, 3], tets [m, 4]); nodes 1.. are the base corners.
    """
    xyz = np.zeros((1 + 3 * m, 3))
    tets = np.zeros((m, 4), dtype=np.int32)
    turn = 2.0 * np.pi * np.arange(m) / m + rng.uniform(-0.05, 0.05, m)
    for i in range(m):
        for c in range(3):
            a = turn[i] + 2.0 * np.pi * c / 3.0
            xyz[1 + 3 * i + c] = (radius * np.cos(a), radius * np.sin(a), -height)
        tets[i] = (0, 1 + 3 * i, 2 + 3 * i, 3 + 3 * i)
    return xyz, tets
