"""Write tests/golden/hex_ellipsoid_oracle.json from the FP64 CPU oracle only.

Workload: the 75x50x40 mm jittered ellipsoid at h = 0.6 mm as eight-node
reduced-integration hexahedra (2.91M elements), temperature-dependent
properties, two seeded Gaussian sources converted at the nodes, handed over
in seeded random node, element and corner order.  The oracle finds its own
critical step (largest eigenvalue of the assembled geometry pencil, Eq 9),
uses dt = 0.9 dt_cr, runs 1000 steps and stores a seeded sample of nodal
temperatures (the 512 hottest nodes plus 3584 uniformly drawn ones), in the
caller's node order.

Run from the repository root:  python tests/golden/make_hex_ellipsoid.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import hex as ohx  # noqa: E402
from oracle.dense import critical_dt_from_lambda  # noqa: E402
from synth import scenarios as sc  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "hex_ellipsoid_oracle.json")


def main(n_steps=1000):
    t0 = time.time()
    s = sc.hex_ellipsoid("random", n_steps=n_steps)
    m = ohx.HexModel(s.xyz, s.tets, oracle.mat_vector(s.materials), s.dir_nodes, s.dir_T)
    lam = m.geometry_lambda("sparse")
    print(f"lambda {lam:.9e} after {time.time() - t0:.0f} s", flush=True)
    dt_cr, _ = critical_dt_from_lambda(lam, m.m)
    m.dt = 0.9 * dt_cr
    q = m.source_nodal(s.sources)
    T = m.initial(s.T0)
    for n in range(n_steps):
        T = m.step(T, q)
        if (n + 1) % 100 == 0:
            print(f"step {n + 1}: Tmax {T.max():.4f} ({time.time() - t0:.0f} s)", flush=True)
    rng = np.random.default_rng(np.random.SeedSequence([sc.SEED_ROOT, 5, 99]))
    hot = np.argsort(T)[-512:]
    rest = rng.choice(np.setdiff1d(np.arange(m.N), hot), 3584, replace=False)
    idx = np.sort(np.concatenate([hot, rest]))
    rec = {
        "about": "FP64 CPU oracle, eight-node hexahedra on the h=0.6 mm ellipsoid "
                 "(random order), written by tests/golden/make_hex_ellipsoid.py",
        "n_nodes": int(m.N), "n_hexes": int(len(m.hexes)), "n_steps": int(n_steps),
        "lambda_geometry": float(lam), "dt_cr": float(dt_cr), "dt": float(m.dt),
        "source_total_W": float(q.sum()), "T_max": float(T.max()),
        "T_sum": float(T.sum()), "idx": idx.tolist(), "T": T[idx].tolist(),
        "seconds": time.time() - t0,
    }
    with open(OUT, "w") as f:
        json.dump(rec, f)
    print(f"wrote {OUT}: lambda={lam:.9e} dt={m.dt:.9g} Tmax={T.max():.4f} "
          f"({time.time() - t0:.0f} s)")


if __name__ == "__main__":
    main()
