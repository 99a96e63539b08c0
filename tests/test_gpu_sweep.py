"""All 256 planning-sweep scenarios in one batched launch sequence, each
checked against the FP64 oracle's stored sample (tests/golden/make_sweep.py:
its 512 hottest nodes and 32 drawn ones) at the oracle's own step, to the
compensated-FP32 bar of 1e-3 K, and each GPU critical step against the
oracle's."""
import json
import os

import numpy as np
import pytest

from paper_1909_05098_amd import fedfem as ff
from synth import scenarios as sc

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "sweep_oracle.json")


def test_sweep_batched_matches_oracle():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    recs = json.load(open(GOLDEN))["scenarios"]
    hs = []
    for r in recs:
        s = sc.sweep_scenario(r["j"])
        assert s.n_tets == r["n_tets"] and s.n_nodes == r["n_nodes"]
        h = ff.Handle(s.xyz, s.tets, s.materials, s.T0, s.dir_nodes, s.dir_T,
                      dt=r["dt"], precision=ff.FP32C)
        h.precompute()
        lam = h.info()["lambda_geometry"]
        assert lam >= (1 - 1e-4) * r["lambda_geometry"], r["j"]
        assert lam <= (1 + 1e-3) * r["lambda_geometry"], r["j"]
        h.set_gaussian_sources(s.sources, s.source_mode)
        hs.append(h)
    b = ff.Batch(hs)
    b.run([r["n_steps"] for r in recs])
    worst, peak = 0.0, 0.0
    for r, h in zip(recs, hs):
        T = h.read_T()
        err = float(np.max(np.abs(T[np.asarray(r["idx"])] - np.asarray(r["T"]))))
        worst = max(worst, err)
        peak = max(peak, r["T_max"])
        assert abs(T.max() - r["T_max"]) <= 0.1, r["j"]
    print(f"[parity] sweep: {len(recs)} scenarios batched, graph {b.last_ms():.2f} ms, "
          f"worst sampled max|dT| = {worst:.3e} K (hottest scenario {peak:.1f} C)",
          flush=True)
    assert worst <= 1e-3
    b.close()
    for h in hs:
        h.close()
