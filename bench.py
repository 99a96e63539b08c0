#!/usr/bin/env python3
"""FED-FEM bio-heat benchmark on one MI355X.

Workload (default): the 75x50x40 mm jittered-lattice ellipsoid at h = 0.6 mm
(17.45M linear tets, 2.98M nodes), temperature-dependent k(T) and c(T), two
seeded Gaussian sources, compensated FP32 time stepping, nodes and elements
renumbered along a Morton curve by the library (``--order random`` keeps the
seeded random input order).  One benchmark step is one explicit time step
(element loads, assembly, nodal update) over the whole mesh.  The timed
region runs exactly --steps steps from the initial state as captured HIP
graphs; the result after them is checked against the FP64 oracle's stored
sample of the same run when one exists for the workload.

Prints one JSON line: element-updates/s, the roofline of the dominant kernel
(algorithmic bytes / measured kernel time, against 8 TB/s), and the FP64 CPU
oracle timed on a bounded sample of the same workload on the host cores.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = ("tet-element updates/s + achieved HBM GB/s; scenarios/s plain vs "
          "batched/surrogate")
GOLDEN3 = os.path.join(ROOT, "tests", "golden", "config3_oracle.json")
PMC_SUMMARY = os.path.join(ROOT, "profiles", "elem_loads_config3_pmc.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_1909_05098_amd", "csrc", "kernels_step.hip")
TUNE_CACHE = os.path.join(os.environ.get("TMPDIR", "/tmp"), "fedfem_tune_cache.txt")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_sha():
    return hashlib.sha1(open(KERNEL_SRC, "rb").read()).hexdigest()[:12]


def read_traffic(n_tets):
    """HBM bytes per element-kernel launch from the committed PMC summary,
    if it was taken on the current kernel source; else None."""
    if not os.path.exists(PMC_SUMMARY):
        return None
    text = open(PMC_SUMMARY).read()
    vals = dict(re.findall(r"^(\w+)\s*=\s*(\S+)\s*$", text, flags=re.M))
    try:
        if vals.get("kernel_source_sha1") != kernel_sha():
            return None
        if int(vals["n_tets"]) != n_tets:
            return None
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(scn, dt, q_params, seconds):
    """The FP64 oracle as it stands, on the first steps of the same run."""
    import oracle
    t0 = time.perf_counter()
    m = oracle.build_model(scn)
    m.dt = dt
    q = m.source(q_params, scn.source_mode)
    setup = time.perf_counter() - t0
    T = m.initial(37.0)
    steps = 0
    t0 = time.perf_counter()
    while True:
        T = m.run(T, 5, q)
        steps += 5
        el = time.perf_counter() - t0
        if el >= seconds or steps >= 400:
            break
    return {"value": scn.n_tets * steps / el, "unit": "element-updates/s",
            "cores": oracle.max_threads(), "kind": "oracle",
            "sample": (f"FP64 oracle, {steps} steps of the same mesh, sources "
                       f"and dt from the initial state ({el:.1f} s timed, "
                       f"{setup:.1f} s untimed setup), OpenMP threads = "
                       f"{oracle.max_threads()}")}


def _gen_sweep_one(j):
    from synth import scenarios as sc
    return sc.sweep_scenario(j)


def gen_sweep(count, workers):
    """Seeded planning-sweep scenarios, built on host cores before any GPU
    use in this process (the pool forks)."""
    from multiprocessing import get_context
    with get_context("fork").Pool(workers) as pool:
        return pool.map(_gen_sweep_one, range(count))


def run_sweep(scns, autotune=True):
    """Scenarios/s for the planning sweep: plain per-scenario use of the
    library versus one batched graph launch, on the same GPU."""
    import numpy as np
    from paper_1909_05098_amd import fedfem as ff
    from synth import scenarios as sc

    def handle(s):
        h = ff.Handle(s.xyz, s.tets, s.materials, s.T0, s.dir_nodes, s.dir_T,
                      dt=-0.9, precision=ff.FP32C)
        if autotune:
            h.autotune(TUNE_CACHE, for_batch=True)
        h.precompute()
        h.set_gaussian_sources(s.sources, s.source_mode)
        _, dtcr = h.dt()
        n, dt = sc.steps_for(s.t_end, dtcr)
        h.set_dt(dt)
        return h, n

    # tune each mesh-size class once (untimed); both legs then hit the cache
    t_tune = 0.0
    if autotune:
        t0 = time.perf_counter()
        for s in scns:
            h = ff.Handle(s.xyz, s.tets, s.materials, s.T0, s.dir_nodes, s.dir_T,
                          dt=-0.9, precision=ff.FP32C)
            h.autotune(TUNE_CACHE, for_batch=True)
            h.close()
        t_tune = time.perf_counter() - t0
        log(f"sweep autotune (all size classes) {t_tune:.2f} s")
    # plain: create -> precompute -> step -> read, one scenario at a time
    plain_T, ns = [], []
    t_all = t_steps = 0.0
    for s in scns:
        t0 = time.perf_counter()
        h, n = handle(s)
        t1 = time.perf_counter()
        h.step(n)
        plain_T.append(h.read_T())
        t2 = time.perf_counter()
        h.close()
        t_all += t2 - t0
        t_steps += t2 - t1
        ns.append(n)
    log(f"sweep plain: {len(scns)} scenarios in {t_all:.2f} s ({t_steps:.2f} s stepping)")
    # batched: all handles, one captured launch sequence
    t0 = time.perf_counter()
    hs = [handle(s)[0] for s in scns]
    t1 = time.perf_counter()
    b = ff.Batch(hs)
    t2 = time.perf_counter()
    b.run(ns)
    t3 = time.perf_counter()
    dT = max(float(np.max(np.abs(h.read_T() - T))) for h, T in zip(hs, plain_T))
    first_graph_ms = b.last_ms()
    # steady state: the same launch sequence again (graph already captured)
    b.run(ns)
    graph_ms = b.last_ms()
    t4 = time.perf_counter()
    b.close()
    for h in hs:
        h.close()
    S = len(scns)
    upd = float(sum(s.n_tets * n for s, n in zip(scns, ns)))
    log(f"sweep batched: precompute {t1 - t0:.2f} s, batch create {t2 - t1:.2f} s, "
        f"first run {t3 - t2:.3f} s, graph {graph_ms:.2f} ms")
    return {"workload": f"planning sweep: {S} seeded ellipsoids, 20k-400k tets, "
                        f"TD properties, 300 s each, FP32C",
            "scenarios": S, "element_updates": upd,
            "steps_min_max": [int(min(ns)), int(max(ns))],
            "plain_scenarios_per_s": round(S / t_all, 2),
            "plain_scenarios_per_s_excl_precompute": round(S / t_steps, 2),
            "batched_scenarios_per_s": round(S / (graph_ms * 1e-3), 1),
            "batched_scenarios_per_s_incl_precompute": round(S / ((t1 - t0) + (t2 - t1) + (t3 - t2)), 2),
            "batched_graph_ms": round(graph_ms, 3),
            "autotune_s_untimed": round(t_tune, 2),
            "batched_first_run_ms": round(first_graph_ms, 3),
            "batched_element_updates_per_s": round(upd / (graph_ms * 1e-3), 1),
            "max_abs_dT_batched_vs_plain_K": dT}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--order", choices=["morton", "random"], default="morton")
    ap.add_argument("--h", type=float, default=0.6e-3)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--max-nodes", type=int, default=0)
    ap.add_argument("--xcd", type=int, default=0)
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the given/default layout options instead of "
                         "letting the library's autotuner choose")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--kernel-steps", type=int, default=20)
    ap.add_argument("--sweep", type=int, default=256,
                    help="planning-sweep scenarios for the batched leg (0 = skip)")
    ap.add_argument("--copy-calib-gib", type=float, default=0.0,
                    help="also run a plain device copy of this size (for "
                         "counter calibration) and exit")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build runs on one GPU only; a multi-GPU run "
              "(--gpus N>1) is not provided.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    sweep_scns = None
    if args.sweep and not args.copy_calib_gib:
        t0 = time.perf_counter()
        sweep_scns = gen_sweep(args.sweep, min(16, os.cpu_count() or 1))
        log(f"sweep meshes: {len(sweep_scns)} scenarios "
            f"({sum(s.n_tets for s in sweep_scns)} tets, {time.perf_counter() - t0:.1f} s)")
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    if args.copy_calib_gib > 0:
        n = int(args.copy_calib_gib * (1 << 30)) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calib_bytes_each_way": 4 * n, "launches": 3}))
        return

    from paper_1909_05098_amd import fedfem as ff
    from synth import scenarios as sc

    t0 = time.perf_counter()
    scn = sc.config3("random", h=args.h, n_steps=args.steps)
    log(f"mesh {scn.n_tets} tets {scn.n_nodes} nodes ({time.perf_counter() - t0:.1f} s)")
    golden = None
    if abs(args.h - 0.6e-3) < 1e-12 and os.path.exists(GOLDEN3):
        golden = json.load(open(GOLDEN3))
        if golden["n_tets"] != scn.n_tets:
            golden = None
    # the oracle's own critical step where it is stored; else the library's
    dt_spec = golden["dt"] if golden else -0.9
    h = ff.Handle(scn.xyz, scn.tets, scn.materials, scn.T0, scn.dir_nodes,
                  scn.dir_T, dt=dt_spec, precision=ff.FP32C,
                  reorder=(args.order == "morton"), tile_elems=args.tile,
                  threads=args.threads, max_tile_nodes=args.max_nodes,
                  xcd=bool(args.xcd))
    tuned = None
    if not args.no_autotune:
        t0 = time.perf_counter()
        tuned = h.autotune(TUNE_CACHE)
        log(f"autotune {time.perf_counter() - t0:.2f} s -> {tuned}")
    t0 = time.perf_counter()
    h.precompute()
    t_pre = time.perf_counter() - t0
    info = h.info()
    dt, dt_cr = h.dt()
    log(f"precompute {t_pre:.2f} s, dt={dt:.6g} dt_cr={dt_cr:.6g}, tiles="
        f"{info['n_tiles']} partials={info['n_partials']} "
        f"lanczos={info['lanczos_iterations']}")
    h.set_gaussian_sources(scn.sources, ff.SOURCE_CONSISTENT)
    state0, _, _ = h.read_state()
    h.prepare(args.steps)
    if args.warmup:
        h.step(args.warmup)
    h.write_state(state0, 0.0, 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h.step(args.steps)
    torch.cuda.synchronize()
    t_run = time.perf_counter() - t0
    log(f"timed {args.steps} steps in {t_run * 1e3:.2f} ms")
    E, N = scn.n_tets, scn.n_nodes
    value = E * args.steps / t_run
    ms_step = t_run * 1e3 / args.steps
    max_err = None
    if golden and golden["n_steps"] == args.steps:
        T = h.read_T()
        idx = np.asarray(golden["idx"])
        max_err = float(np.max(np.abs(T[idx] - np.asarray(golden["T"]))))
        log(f"max|T - T_oracle| on {len(idx)} sampled nodes = {max_err:.3e} K")
    # per-kernel durations with HIP events on the handle's stream
    elem_ms, node_ms = h.time_kernels(args.kernel_steps)
    elem_bytes = 40.0 * E   # 4 x i32 connectivity + 6 x f32 coefficients
    node_bytes = 24.0 * N   # T hi/lo read+write, 1/V_i, source
    kern = {"elem_loads": (elem_ms, elem_bytes), "node_update": (node_ms, node_bytes)}
    dom = max(kern, key=lambda k: kern[k][0])
    ms, by = kern[dom]
    achieved = by / (ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4),
                "traffic": read_traffic(E) if dom == "elem_loads" else None,
                "algorithmic_bytes_per_launch": by, "avg_launch_ms": round(ms, 5)}
    other = [k for k in kern if k != dom][0]
    step_gbps = (elem_bytes + node_bytes) / (ms_step * 1e-3) / 1e9
    h.close()
    batched = run_sweep(sweep_scns, not args.no_autotune) if sweep_scns else None
    cpu = None
    if not args.no_cpu:
        log("timing the FP64 CPU oracle on a bounded sample")
        cpu = cpu_baseline(scn, dt, scn.sources, args.cpu_seconds)
        cpu["value"] = round(cpu["value"], 1)
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "element-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"ellipsoid 75x50x40 mm, jittered Kuhn lattice "
                               f"h={args.h * 1e3:g} mm, TD k(T) c(T), two "
                               f"Gaussian sources, {args.order} order",
                   "n_tets": E, "n_nodes": N, "dt_s": dt,
                   "precision": "f32 element loop, compensated f32 hi/lo nodal state, f64 precompute",
                   "tile_elems": info["tile_elems"], "threads": info["threads"],
                   "autotuned": tuned is not None,
                   "parallelism": "1 GPU"},
        "roofline": roofline,
        "other_kernel": {"kernel": other, "avg_launch_ms": round(kern[other][0], 5),
                         "achieved_GBps": round(kern[other][1] / (kern[other][0] * 1e-3) / 1e9, 1)},
        "step_GBps_algorithmic": round(step_gbps, 1),
        "max_abs_dT_vs_oracle_K": max_err,
        "precompute_s": round(t_pre, 3),
        "batched": batched,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
