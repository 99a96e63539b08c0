"""Write tests/golden/config3_dose_oracle.json from the FP64 CPU oracle only.

The config-3 run of tests/golden/make_config3.py (the 17.45M-tet ellipsoid at
h = 0.6 mm, random order, the oracle's own step from config3_oracle.json,
1000 steps) with the CEM43 thermal dose accumulated at every node from the
start of the run (oracle/dose.py).  Stores the dose and temperature at the
same 4096 sampled nodes as config3_oracle.json, in the caller's node order.

Run from the repository root, after make_config3.py:
    python tests/golden/make_config3_dose.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import dose  # noqa: E402
from synth import scenarios as sc  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "config3_dose_oracle.json")


def main():
    t0 = time.time()
    g = json.load(open(os.path.join(HERE, "config3_oracle.json")))
    s = sc.config3("random", n_steps=g["n_steps"])
    m = oracle.build_model(s)
    m.dt = g["dt"]
    q = m.source(s.sources, s.source_mode)
    idx = np.asarray(g["idx"])

    def step(T, n):
        if (n + 1) % 100 == 0:
            print(f"step {n + 1} ({time.time() - t0:.0f} s)", flush=True)
        return m.run(T, 1, q)

    T, D = dose.accumulate(step, m.initial(37.0), g["n_steps"], m.dt, dose.cem43_rate)
    rec = {
        "about": "FP64 CPU oracle, config 3 with the CEM43 dose, written by "
                 "tests/golden/make_config3_dose.py",
        "n_nodes": int(m.N), "n_tets": int(m.E), "n_steps": int(g["n_steps"]),
        "dt": float(m.dt), "model": "cem43", "idx": idx.tolist(),
        "T": T[idx].tolist(), "dose": D[idx].tolist(),
        "dose_max": float(D.max()), "seconds": time.time() - t0,
    }
    with open(OUT, "w") as f:
        json.dump(rec, f)
    print(f"wrote {OUT}: max T diff vs config3 golden "
          f"{np.max(np.abs(T[idx] - np.asarray(g['T']))):.3e}, dose max {D.max():.4e} "
          f"({time.time() - t0:.0f} s)")


if __name__ == "__main__":
    main()
