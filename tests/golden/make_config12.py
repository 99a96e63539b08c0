"""Write tests/golden/config1_oracle.json and config2_oracle.json from the
FP64 CPU oracle only.

Config 1: the 1 cm cube as a 10 x 10 x 10 Kuhn lattice (6000 tets), constant
properties, Dirichlet 37 C on the surface, nodal-sampled Gaussian source,
300 s.  The oracle's dense eigenvalue gives dt_cr (Eq 9); n = ceil(300 s /
(0.9 dt_cr)) steps of 300 s / n.  Every nodal temperature is stored.

Config 2: the 75 x 50 x 40 mm ellipsoid as a jittered lattice at h = 1.2 mm
(2.18M tets), temperature-dependent k(T) and c(T), one consistent Gaussian
source, 600 s at the oracle's own step (Lanczos on the assembled pencil).
A seeded sample of 4096 nodal temperatures is stored (the 512 hottest plus
3584 drawn ones).

Run from the repository root:  python tests/golden/make_config12.py
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

HERE = os.path.dirname(os.path.abspath(__file__))


def config1():
    t0 = time.time()
    s = sc.config1()
    m = oracle.build_model(s)
    lam = m.geometry_lambda(method="dense")
    dt_cr, _ = dense.critical_dt_from_lambda(lam, m.mat)
    n, dt = sc.steps_for(s.t_end, dt_cr)
    m.dt = dt
    q = m.source(s.sources, s.source_mode)
    T = m.run(m.initial(37.0), n, q)
    rec = {"about": "FP64 CPU oracle, config 1 (1 cm Kuhn cube, 6000 tets), every node, "
                    "written by tests/golden/make_config12.py",
           "n_nodes": int(m.N), "n_tets": int(m.E), "n_steps": int(n),
           "lambda_geometry": float(lam), "dt_cr": float(dt_cr), "dt": float(dt),
           "T_max": float(T.max()), "T": [float(v) for v in T],
           "seconds": time.time() - t0}
    path = os.path.join(HERE, "config1_oracle.json")
    with open(path, "w") as f:
        json.dump(rec, f)
    print(f"wrote {path}: n={n} dt={dt:.9g} Tmax={T.max():.6f}", flush=True)


def config2():
    t0 = time.time()
    s = sc.config2()
    m = oracle.build_model(s)
    lam = m.geometry_lambda()
    dt_cr, _ = dense.critical_dt_from_lambda(lam, m.mat)
    n, dt = sc.steps_for(s.t_end, dt_cr)
    print(f"config 2: lambda {lam:.9e}, n={n} after {time.time() - t0:.0f} s", flush=True)
    m.dt = dt
    q = m.source(s.sources, s.source_mode)
    T = m.run(m.initial(37.0), n, q)
    rng = np.random.default_rng(np.random.SeedSequence([sc.SEED_ROOT, 2, 99]))
    hot = np.argsort(T)[-512:]
    rest = rng.choice(np.setdiff1d(np.arange(m.N), hot), 3584, replace=False)
    idx = np.sort(np.concatenate([hot, rest]))
    rec = {"about": "FP64 CPU oracle, config 2 (h=1.2 mm ellipsoid), written by "
                    "tests/golden/make_config12.py",
           "n_nodes": int(m.N), "n_tets": int(m.E), "n_steps": int(n),
           "lambda_geometry": float(lam), "dt_cr": float(dt_cr), "dt": float(dt),
           "source_total_W": float(q.sum()), "T_max": float(T.max()),
           "idx": idx.tolist(), "T": T[idx].tolist(),
           "oracle_threads": oracle.max_threads(), "seconds": time.time() - t0}
    path = os.path.join(HERE, "config2_oracle.json")
    with open(path, "w") as f:
        json.dump(rec, f)
    print(f"wrote {path}: n={n} dt={dt:.9g} Tmax={T.max():.4f} ({time.time() - t0:.0f} s)")


if __name__ == "__main__":
    config1()
    config2()
