"""Small shared test helpers (inputs only)."""
import numpy as np

from synth import mesh


def jittered_box(nx, ny, nz, h, seed, jitter=0.2):
    xyz, tets = mesh.kuhn_box(nx, ny, nz, h)
    bnd = mesh.boundary_nodes_by_faces(len(xyz), tets)
    rng = np.random.default_rng(seed)
    mask = np.ones(len(xyz), bool)
    mask[bnd] = False
    xyz[mask] += rng.uniform(-jitter * h, jitter * h, (mask.sum(), 3))
    return xyz, tets, bnd


def header_functions(path):
    """Names of the functions declared in a C header."""
    import re
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b((?:fedfem|fedsur)_[A-Za-z_0-9]+)\s*\(", text)))
