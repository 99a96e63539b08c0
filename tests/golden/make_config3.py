"""Write tests/golden/config3_oracle.json from the FP64 CPU oracle only.

Workload: the 75x50x40 mm jittered ellipsoid at h = 0.6 mm (17.45M tets),
temperature-dependent properties, two seeded Gaussian sources, handed over in
seeded random order.  The oracle finds its own critical step (Lanczos on the
assembled geometry pencil, Eq 9), uses dt = 0.9 dt_cr, runs 1000 steps and
stores a seeded sample of nodal temperatures (the 512 hottest nodes plus 3584
uniformly drawn ones), in the caller's node order.

Run from the repository root:  python tests/golden/make_config3.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import dense  # noqa: E402
from synth import scenarios as sc  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config3_oracle.json")


def main(n_steps=1000):
    t0 = time.time()
    s = sc.config3("random", n_steps=n_steps)
    m = oracle.build_model(s)
    tets64 = m.tets.astype(np.int64)
    A, vol = dense.element_matrices(m.xyz, tets64)
    Vi = dense.lumped_volume(m.N, tets64, vol)
    lam = dense.geometry_lambda_from(m.N, tets64, A, Vi, m.is_dir, method="sparse")
    del A, vol, Vi
    print(f"lambda {lam:.9e} after {time.time() - t0:.0f} s", flush=True)
    dt_cr, lam_max = dense.critical_dt_from_lambda(lam, m.mat)
    dt = 0.9 * dt_cr
    m.dt = dt
    q = m.source(s.sources, s.source_mode)
    T = m.run(m.initial(37.0), n_steps, q)
    rng = np.random.default_rng(np.random.SeedSequence([sc.SEED_ROOT, 3, 99]))
    hot = np.argsort(T)[-512:]
    rest = rng.choice(np.setdiff1d(np.arange(m.N), hot), 3584, replace=False)
    idx = np.sort(np.concatenate([hot, rest]))
    rec = {
        "about": "FP64 CPU oracle, config 3 (h=0.6 mm ellipsoid, random order), "
                 "written by tests/golden/make_config3.py",
        "n_nodes": int(m.N), "n_tets": int(m.E), "n_steps": int(n_steps),
        "lambda_geometry": float(lam), "dt_cr": float(dt_cr), "dt": float(dt),
        "source_total_W": float(q.sum()), "T_max": float(T.max()),
        "T_sum": float(T.sum()), "idx": idx.tolist(), "T": T[idx].tolist(),
        "oracle_threads": oracle.max_threads(),
        "seconds": time.time() - t0,
    }
    with open(OUT, "w") as f:
        json.dump(rec, f)
    print(f"wrote {OUT}: lambda={lam:.9e} dt={dt:.9g} Tmax={T.max():.4f} "
          f"({time.time() - t0:.0f} s)")


if __name__ == "__main__":
    main()
