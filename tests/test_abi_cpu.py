"""CPU checks of the C ABI: the library loads, exports what the header
declares, and rejects bad input before touching the GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1909_05098_amd import fedfem as ff
from synth import mesh

from helpers import header_functions

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fedfem.h")
HEADER_SUR = os.path.join(ROOT, "include", "fedfem_surrogate.h")


def declared():
    return sorted(set(header_functions(HEADER)) | set(header_functions(HEADER_SUR)))


def test_header_declares_binding_surface():
    from paper_1909_05098_amd import surrogate as sg
    assert declared() == sorted(set(ff.exported_symbols()) | set(sg.exported_symbols()))


def test_library_exports_every_declared_symbol():
    L = ff.load()
    for name in declared():
        assert hasattr(L, name), name
    out = os.popen(f"nm -D --defined-only {ff.LIB_PATH}").read()
    exported = set(re.findall(r"\bT ((?:fedfem|fedsur)_[A-Za-z_0-9]+)", out))
    assert exported == set(declared())


def test_strerror_and_null_handling():
    L = ff.load()
    assert L.fedfem_strerror(0) == b"ok"
    assert L.fedfem_strerror(ff.E_DIVERGED) == b"solution diverged"
    assert L.fedfem_destroy(None) == ff.OK
    assert L.fedfem_batch_destroy(None) == ff.OK
    assert L.fedfem_create(None, None, None, None) == ff.E_INVALID
    assert L.fedfem_step(None, 1, None) == ff.E_INVALID
    assert L.fedfem_precompute(None) == ff.E_INVALID
    # precompute_many checks its arguments before any device work
    L.fedfem_precompute_many.argtypes = [C.c_void_p, C.c_int32, C.c_int32,
                                         C.c_void_p]
    arr = (C.c_void_p * 2)(None, None)
    assert L.fedfem_precompute_many(arr, 2, 0, None) == ff.E_INVALID
    assert L.fedfem_precompute_many(None, 1, 0, None) == ff.E_INVALID
    assert L.fedfem_precompute_many(arr, -1, 0, None) == ff.E_INVALID
    assert L.fedfem_precompute_many(arr, 0, 0, None) == ff.OK


def _mat():
    return {f: v for f, v in zip(ff.MAT_FIELDS, (1060.0, 3600.0, 0.512, 0.0, 0.0,
                                                  0.0, 37.0, 0.0, 100.0, 6.4,
                                                  4180.0, 37.0, 0.0))}


@pytest.mark.parametrize("case", ["bad_id", "unused_node", "nan_xyz", "dup_dir",
                                  "bad_prec", "bad_window", "neg_k", "bad_dt"])
def test_create_rejects_bad_input(case):
    xyz, tets = mesh.kuhn_box(2, 2, 2, 1e-3)
    mat = _mat()
    dn = [0, 1]
    dt = -0.9
    prec = ff.FP32C
    if case == "bad_id":
        tets = tets.copy()
        tets[3, 2] = len(xyz)
    elif case == "unused_node":
        xyz = np.vstack([xyz, [[9.0, 9.0, 9.0]]])
    elif case == "nan_xyz":
        xyz = xyz.copy()
        xyz[4, 1] = np.nan
    elif case == "dup_dir":
        dn = [0, 0]
    elif case == "bad_prec":
        prec = 7
    elif case == "bad_window":
        mat["T_lo"], mat["T_hi"] = 50.0, 40.0
    elif case == "neg_k":
        mat["dk_dT"] = -0.1
    elif case == "bad_dt":
        dt = -1.5
    with pytest.raises(ff.FedFemError) as ei:
        ff.Handle(xyz, tets, mat, 37.0, dn, [37.0] * len(dn), dt=dt,
                  precision=prec)
    assert ei.value.code == ff.E_INVALID


def test_product_never_imports_oracle():
    pkg = os.path.join(ROOT, "paper_1909_05098_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "libfedfem_oracle" not in text, f
    for f in ("fedfem_oracle.c", "__init__.py", "dense.py"):
        text = open(os.path.join(ROOT, "oracle", f)).read()
        assert "paper_1909_05098_amd" not in text


@pytest.mark.parametrize("case", ["bad_id", "unused_node", "nan_xyz"])
def test_create_hex_rejects_bad_input(case):
    xyz, hexes = mesh.hex_box(3, 2, 2, 1e-3)
    if case == "bad_id":
        hexes = hexes.copy()
        hexes[2, 7] = -1
    elif case == "unused_node":
        xyz = np.vstack([xyz, [[9.0, 9.0, 9.0]]])
    elif case == "nan_xyz":
        xyz = xyz.copy()
        xyz[5, 2] = np.inf
    with pytest.raises(ff.FedFemError) as ei:
        ff.Handle(xyz, hexes, _mat(), 37.0, [0, 1], [37.0, 37.0])
    assert ei.value.code == ff.E_INVALID
    assert "fedfem_create_hex" in str(ei.value)


@pytest.mark.parametrize("faces, flux", [
    (np.zeros((4, 2), np.int32), np.ones(4)),     # two columns
    (np.zeros((4, 5), np.int32), np.ones(4)),     # five columns
    (np.zeros(12, np.int32), np.ones(4)),         # flat array
    (np.zeros((4, 3), np.int32), np.ones(3)),     # short flux
    (np.zeros((4, 4), np.int32), np.ones(5)),     # long flux
])
def test_flux_loads_rejects_bad_shapes(faces, flux):
    """The binding refuses face arrays that are not [F, 3] or [F, 4] and
    flux vectors of another length before the C call (which reads F fluxes
    and takes the face width from the entry point)."""
    h = ff.Handle.__new__(ff.Handle)  # no device handle: the check comes first
    h.xyz = np.zeros((8, 3))
    with pytest.raises(ValueError):
        h.flux_loads(faces, flux)


@pytest.mark.parametrize("grid,batch", [(0, 1), (6, 1), (260, 1), (64, 0), (64, 4097),
                                        (256, 128)])
def test_network_create_rejects_bad_sizes(grid, batch):
    """fedsur_create checks its sizes before any device work: the grid a
    multiple of 4 in [4, 256], the batch in [1, 4096] and batch G^3 below
    2^31 (the 2 x 2 x 2 kernels index voxels in 32 bits)."""
    from paper_1909_05098_amd import surrogate as sg
    L = sg.lib()
    out = C.c_void_p()
    assert L.fedsur_create(grid, batch, C.c_uint64(0), C.byref(out)) == ff.E_INVALID
    assert not out.value
