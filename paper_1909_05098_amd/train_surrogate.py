"""Train the surrogate on FED-FEM runs of the planning-sweep generator and
evaluate it on held-out seeds.

    python -m paper_1909_05098_amd.train_surrogate --train 4096 --test 512 \
        --out surrogate_g64.npy --summary summary.json

Scenario j of the generator (synth.scenarios.sweep_scenario) is a seeded
ellipsoid mesh with temperature-dependent properties and one Gaussian
source; FED-FEM runs it to 300 s in batched launches and the result is
resampled onto the 64^3 voxel frame.  Training seeds are 0 .. train-1,
held-out seeds test_seed0 .. test_seed0 + test - 1.  Meshes are built by a
pool of host processes forked before the GPU is touched.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


def log(msg):
    print(f"[train] {msg}", file=sys.stderr, flush=True)


def _gen(j):
    from synth import scenarios as sc
    return sc.sweep_scenario(j)


def fem_dataset(pool, ids, G, fr, chunk, tag):
    """FED-FEM fields of scenarios `ids` on the grid (device tensors) and the
    samples (host float64 [S, 12])."""
    import torch
    from . import surrogate_pipeline as pl
    S = len(ids)
    T = torch.empty((S, G, G, G), dtype=torch.float32, device="cuda")
    M = torch.empty((S, G, G, G), dtype=torch.uint8, device="cuda")
    rows = []
    t0 = time.perf_counter()
    chunks = [ids[i:i + chunk] for i in range(0, S, chunk)]
    pending = pool.map_async(_gen, chunks[0])
    for c, ch in enumerate(chunks):
        scns = pending.get()
        if c + 1 < len(chunks):
            pending = pool.map_async(_gen, chunks[c + 1])
        rows += [pl.sample_row(s) for s in scns]
        i0 = c * chunk
        pl.fem_on_grid(scns, T[i0:i0 + len(ch)], M[i0:i0 + len(ch)], G, fr)
        torch.cuda.synchronize()
        log(f"{tag}: {i0 + len(ch)}/{S} scenarios on the grid "
            f"({time.perf_counter() - t0:.1f} s)")
    return np.array(rows), T, M, time.perf_counter() - t0


def evaluate(net, samples, T, M, phys, G, fr, batch):
    """Per-scenario max |T_surrogate - T_FED-FEM| over the mesh's voxels."""
    import torch
    from . import surrogate as sg
    from . import surrogate_pipeline as pl
    S = samples.shape[0]
    pred = torch.empty((S, G, G, G), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pl.predict(net, samples, phys, pred, batch, G, fr)
    torch.cuda.synchronize()
    t_inf = time.perf_counter() - t0
    err = torch.empty(S, dtype=torch.float32, device="cuda")
    sg.max_error(G, pred, T, M, err, torch.cuda.current_stream().cuda_stream)
    P = pl.peak_scale(samples, phys)
    return err.cpu().numpy().astype(np.float64), P, t_inf


def error_summary(err, P, tol):
    q = np.quantile(err, [0.5, 0.9, 0.99])
    rel = err / P
    return {"max_abs_err_K": {"median": float(q[0]), "p90": float(q[1]), "p99": float(q[2]),
                              "max": float(err.max())},
            "max_err_over_peak": {"median": float(np.median(rel)), "max": float(rel.max())},
            "fraction_within_tol": float(np.mean(err <= tol)),
            "peak_K": {"min": float(P.min()), "median": float(np.median(P)),
                       "max": float(P.max())}}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--train", type=int, default=4096)
    ap.add_argument("--test", type=int, default=512)
    ap.add_argument("--test-seed0", type=int, default=10000)
    ap.add_argument("--grid", type=int, default=64)
    ap.add_argument("--epochs", type=int, default=12)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--focus", type=float, default=20.0)
    ap.add_argument("--chunk", type=int, default=256)
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--init", default=None, help="start from these parameters (.npy)")
    ap.add_argument("--out", required=True, help="trained parameters (.npy)")
    ap.add_argument("--summary", default=None, help="JSON summary file")
    args = ap.parse_args()

    from multiprocessing import get_context
    pool = get_context("fork").Pool(args.workers)  # before any GPU use

    import torch
    assert torch.cuda.is_available(), "training needs a GPU"
    torch.cuda.set_device(0)
    from . import surrogate as sg
    from . import surrogate_pipeline as pl

    G = args.grid
    fr = pl.frame(G)
    phys = pl.phys_of(_gen(0).materials)
    rows, T, M, t_data = fem_dataset(pool, list(range(args.train)), G, fr, args.chunk, "train")
    rows_t, Tt, Mt, t_data_t = fem_dataset(
        pool, list(range(args.test_seed0, args.test_seed0 + args.test)), G, fr, args.chunk,
        "test")
    pool.close()
    samples = torch.tensor(rows, device="cuda")
    samples_t = torch.tensor(rows_t, device="cuda")

    net = sg.Net(G, args.batch, seed=args.seed)
    if args.init:
        pl.load_params(net, args.init)
    err0, P0, _ = evaluate(net, samples_t, Tt, Mt, phys, G, fr, args.batch)
    log(f"before training: held-out median max|dT| {np.median(err0):.3f} K")
    t0 = time.perf_counter()
    hist = pl.train(net, samples, T, M, phys, args.epochs, args.batch, args.lr, G, fr,
                    seed=args.seed, focus=args.focus, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    pl.save_params(net, args.out)
    err, P, t_inf = evaluate(net, samples_t, Tt, Mt, phys, G, fr, args.batch)
    err_tr, P_tr, _ = evaluate(net, samples[:args.test], T[:args.test], M[:args.test], phys,
                               G, fr, args.batch)
    # the prior alone (network output zero) as the no-learning baseline
    zero = sg.Net(G, args.batch, seed=args.seed)
    zero.set_params(np.zeros(zero.n_params, dtype=np.float32))
    err_p, _, _ = evaluate(zero, samples_t, Tt, Mt, phys, G, fr, args.batch)
    out = {"grid": G, "train_scenarios": args.train, "test_scenarios": args.test,
           "epochs": args.epochs, "batch": args.batch, "lr": args.lr, "focus": args.focus,
           "dataset_s": round(t_data + t_data_t, 1), "train_s": round(t_train, 1),
           "train_sample_steps_per_s": round(args.epochs * (args.train // args.batch)
                                             * args.batch / t_train, 1),
           "loss_per_epoch": [float(x) for x in hist],
           "heldout_inference_s": round(t_inf, 3),
           "heldout": error_summary(err, P, pl.TOL_K),
           "train_subset": error_summary(err_tr, P_tr, pl.TOL_K),
           "heldout_prior_only": error_summary(err_p, P, pl.TOL_K),
           "heldout_untrained": error_summary(err0, P0, pl.TOL_K)}
    log(json.dumps(out, indent=1))
    if args.summary:
        with open(args.summary, "w") as f:
            json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
