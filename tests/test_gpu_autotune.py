"""The autotuner picks a layout by timing candidates, caches the choice per
mesh-size bucket, and the tuned layout keeps parity with the oracle."""
import os

import numpy as np
import pytest

import oracle
from paper_1909_05098_amd import fedfem as ff
from synth import scenarios as sc

from helpers import jittered_box

pytestmark = pytest.mark.gpu


def test_autotune_choice_cache_and_parity(tmp_path):
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    xyz, tets, bnd = jittered_box(24, 20, 16, 1e-3, seed=31)
    mat = sc.td_materials()
    src = [[12e-3, 10e-3, 8e-3, 2e-3, 1e8]]
    om = oracle.OracleModel(xyz, tets, mat, bnd, np.full(len(bnd), 37.0))
    om.dt = 0.9 * om.dt_cr()
    T_ref = om.run(om.initial(37.0), 200, om.source_consistent(src))
    cache = str(tmp_path / "tune.txt")
    h = ff.Handle(xyz, tets, mat, 37.0, bnd, np.full(len(bnd), 37.0), dt=om.dt)
    opt = h.autotune(cache)
    print(f"[autotune] {len(tets)} tets -> {opt}", flush=True)
    assert opt["tile_elems"] in (1024, 2048, 4096)
    assert opt["tile_elems"] % opt["threads"] == 0
    lines = open(cache).read().split("\n")
    assert len([l for l in lines if l.strip()]) == 1
    # a second handle of the same size class takes the cached choice
    h2 = ff.Handle(xyz, tets, mat, 37.0, bnd, np.full(len(bnd), 37.0), dt=om.dt)
    assert h2.autotune(cache) == opt
    assert len([l for l in open(cache).read().split("\n") if l.strip()]) == 1
    h.precompute()
    h.set_gaussian_sources(src)
    h.step(200)
    err = float(np.max(np.abs(h.read_T() - T_ref)))
    print(f"[parity] autotuned layout: max|dT|={err:.3e} K", flush=True)
    assert err <= 1e-3
    with pytest.raises(ff.FedFemError) as ei:
        h.autotune(cache)
    assert ei.value.code == ff.E_STATE
