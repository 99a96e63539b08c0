"""Write tests/golden/sweep_oracle.json from the FP64 CPU oracle only.

Workload: the 256-scenario planning sweep (seeded ellipsoids with semi-axes
30-80 mm and 20k-400k tets, per-scenario k0, perfusion, source power, width
and position, temperature-dependent properties, 300 s each).  For every
scenario the oracle finds its own critical step (Eq 9, Lanczos on the
assembled pencil), takes n = ceil(300 s / (0.9 dt_cr)) steps of 300 s / n and
stores a seeded sample of nodal temperatures: the 512 hottest nodes (where
the heating, and so any error of the time stepping, concentrates) plus 32
uniformly drawn ones, to 1e-9 K.

Run from the repository root:  python tests/golden/make_sweep.py
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

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sweep_oracle.json")


def one(j):
    s = sc.sweep_scenario(j)
    m = oracle.build_model(s)
    lam = m.geometry_lambda()
    dt_cr, _ = dense.critical_dt_from_lambda(lam, m.mat)
    n, dt = sc.steps_for(s.t_end, dt_cr)
    m.dt = dt
    q = m.source(s.sources, s.source_mode)
    T = m.run(m.initial(37.0), n, q)
    rng = np.random.default_rng(np.random.SeedSequence([sc.SEED_ROOT, 4, j, 99]))
    hot = np.argsort(T)[-512:]
    rest = rng.choice(np.setdiff1d(np.arange(m.N), hot), 32, replace=False)
    idx = np.sort(np.concatenate([hot, rest]))
    return {"j": j, "n_nodes": int(m.N), "n_tets": int(m.E), "lambda_geometry": float(lam),
            "dt_cr": float(dt_cr), "dt": float(dt), "n_steps": int(n),
            "T_max": float(T.max()), "idx": idx.tolist(),
            "T": [round(float(v), 9) for v in T[idx]]}


def main(count=256):
    t0 = time.time()
    recs = []
    for j in range(count):
        recs.append(one(j))
        if j % 16 == 15:
            print(f"{j + 1} scenarios, {time.time() - t0:.0f} s", flush=True)
    with open(OUT, "w") as f:
        json.dump({"about": "FP64 CPU oracle, planning sweep, written by "
                            "tests/golden/make_sweep.py", "scenarios": recs}, f)
    print(f"wrote {OUT} ({time.time() - t0:.0f} s)")


if __name__ == "__main__":
    main()
