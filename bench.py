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
Beside it: the planning sweep (256 seeded scenarios, one at a time versus one
batched launch) and the learned surrogate on 512 held-out scenarios (FED-FEM
one at a time and batched, the network alone, and the network with its
FED-FEM spot check and fallback), each with scenarios/s and its error
against FED-FEM; and the same ellipsoid meshed with eight-node
reduced-integration hexahedra (element-updates/s, its element kernel's
roofline, its parity against the oracle's stored run).
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
GOLDEN_HEX = os.path.join(ROOT, "tests", "golden", "hex_ellipsoid_oracle.json")
GOLDEN_DOSE = os.path.join(ROOT, "tests", "golden", "config3_dose_oracle.json")
GOLDEN1 = os.path.join(ROOT, "tests", "golden", "config1_oracle.json")
GOLDEN2 = os.path.join(ROOT, "tests", "golden", "config2_oracle.json")
GOLDEN_SWEEP = os.path.join(ROOT, "tests", "golden", "sweep_oracle.json")
PMC_SUMMARY = os.path.join(ROOT, "profiles", "elem_loads_config3_pmc.txt")
PMC_SUMMARY_HEX = os.path.join(ROOT, "profiles", "elem_loads_hex_ellipsoid_pmc.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_1909_05098_amd", "csrc", "kernels_step.hip")
TUNE_CACHE = os.path.join(os.environ.get("TMPDIR", "/tmp"), "fedfem_tune_cache.txt")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_sha():
    return hashlib.sha1(open(KERNEL_SRC, "rb").read()).hexdigest()[:12]


def read_traffic(n_elems, tile_elems, threads, xcd, summary=PMC_SUMMARY, count="n_tets"):
    """HBM bytes per element-kernel launch from the committed PMC summary,
    if it was taken on the current kernel source and on this layout (tile
    size, workgroup size, XCD remap); else None."""
    if not os.path.exists(summary):
        return None
    text = open(summary).read()
    vals = dict(re.findall(r"^(\w+)\s*=\s*(\S+)\s*$", text, flags=re.M))
    try:
        if vals.get("kernel_source_sha1") != kernel_sha():
            return None
        if int(vals[count]) != n_elems:
            return None
        key = f"traffic_bytes_per_launch_te{tile_elems}_th{threads}_xcd{xcd}"
        return float(vals[key]) if key in vals else None
    except (KeyError, ValueError):
        return None


def check_vs_golden(h, state0, golden, n_tets):
    """Rewind the handle to its initial state, run the stored oracle run's
    step count (untimed) and return max |T - T_oracle| over its sampled
    nodes (every node when the record holds no sample)."""
    import numpy as np
    if not golden or golden.get("n_tets", golden.get("n_hexes")) != n_tets:
        return None
    h.write_state(state0, 0.0, 0)
    h.step(golden["n_steps"])
    T = h.read_T()
    ref = np.asarray(golden["T"])
    if "idx" in golden:
        T = T[np.asarray(golden["idx"])]
    return float(np.max(np.abs(T - ref)))


def load_golden(path, key, value):
    if not os.path.exists(path):
        return None
    g = json.load(open(path))
    return g if g.get(key) == value else None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _oracle_steps(m, q, seconds, chunk=5, cap=400):
    """Steps of the oracle model from its initial state until `seconds` have
    passed (or `cap` steps); returns (steps, elapsed seconds)."""
    T = m.initial(37.0)
    steps = 0
    t0 = time.perf_counter()
    while True:
        T = m.run(T, chunk, q)
        steps += chunk
        el = time.perf_counter() - t0
        if el >= seconds or steps >= cap:
            return steps, el


def cpu_baseline(scn, dt, q_params, seconds, sweep_scns=None, sweep_seconds=8.0):
    """The FP64 oracle as it stands, on the host cores: the first steps of
    the same config-3 run on all cores (up to 16 OpenMP threads) and on one
    thread, and, when given, whole planning-sweep scenarios (critical step,
    source and every step, as the oracle computes them) for a bounded
    number of seconds."""
    import oracle
    from oracle import dense
    from synth import scenarios as sc
    t0 = time.perf_counter()
    m = oracle.build_model(scn)
    m.dt = dt
    q = m.source(q_params, scn.source_mode)
    setup = time.perf_counter() - t0
    threads = oracle.max_threads()
    steps, el = _oracle_steps(m, q, seconds)
    m.n_threads = 1
    steps1, el1 = _oracle_steps(m, q, seconds / 2, chunk=1, cap=100)
    del m  # the sweep models below name their thread count (the last one set stays)
    out = {"value": round(scn.n_tets * steps / el, 1), "unit": "element-updates/s",
           "cores": threads, "kind": "oracle",
           "sample": (f"FP64 oracle, {steps} steps of the same mesh, sources "
                      f"and dt from the initial state ({el:.1f} s timed, "
                      f"{setup:.1f} s untimed setup), OpenMP threads = {threads}"),
           "value_1thread": round(scn.n_tets * steps1 / el1, 1),
           "sample_1thread": f"{steps1} steps on one thread ({el1:.1f} s timed)",
           "cpu_model": cpu_model(), "os_cpu_count": os.cpu_count()}
    if sweep_scns:
        done, upd = 0, 0.0
        t0 = time.perf_counter()
        for s in sweep_scns:
            om = oracle.build_model(s, n_threads=threads)
            dt_cr, _ = dense.critical_dt_from_lambda(om.geometry_lambda(), om.mat)
            n, om.dt = sc.steps_for(s.t_end, dt_cr)
            om.run(om.initial(37.0), n, om.source(s.sources, s.source_mode))
            done += 1
            upd += float(s.n_tets) * n
            if time.perf_counter() - t0 >= sweep_seconds:
                break
        el = time.perf_counter() - t0
        out["sweep"] = {"scenarios_per_s": round(done / el, 3),
                        "element_updates_per_s": round(upd / el, 1), "cores": threads,
                        "sample": f"the first {done} planning-sweep scenarios, each from "
                                  f"mesh to final field ({el:.1f} s)"}
    return out


def run_dose(h, state0, args, E, N, ms_plain):
    """The same config-3 run with the CEM43 thermal dose fused into the
    nodal update: step time, the node kernel with and without it, and the
    dose against the oracle's stored sample of the same run."""
    import numpy as np
    import torch
    from paper_1909_05098_amd import fedfem as ff
    _, node_plain = h.time_kernels(args.kernel_steps)
    h.set_dose(ff.DOSE_CEM43)
    h.write_state(state0, 0.0, 0)
    h.prepare(args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h.step(args.steps)
    torch.cuda.synchronize()
    t_run = time.perf_counter() - t0
    _, node_ms = h.time_kernels(args.kernel_steps)
    # untimed: the stored oracle run's step count from the initial state,
    # with the accumulator restarted (setting the model zeroes it)
    rel = dT = None
    g = load_golden(GOLDEN_DOSE, "n_tets", E)
    if g:
        h.write_state(state0, 0.0, 0)
        h.set_dose(ff.DOSE_CEM43)
        h.step(g["n_steps"])
        idx = np.asarray(g["idx"])
        ref = np.asarray(g["dose"])
        rel = float(np.max(np.abs(h.read_dose()[idx] - ref) / ref))
        dT = float(np.max(np.abs(h.read_T()[idx] - np.asarray(g["T"]))))
        log(f"dose: max relative error on {len(idx)} sampled nodes = {rel:.3e} "
            f"after {g['n_steps']} steps (max|dT| {dT:.3e} K)")
    h.set_dose(ff.DOSE_OFF)
    # node pass bytes: T hi/lo read and write, u, q, and the FP64 dose read
    # and written
    node_bytes = 40.0 * N
    ms_step = t_run * 1e3 / args.steps
    return {"model": "CEM43 (Sapareto-Dewey), FP64 per node, fused into the nodal update",
            "steps": args.steps, "ms_per_step": round(ms_step, 5),
            "ms_per_step_without_dose": round(ms_plain, 5),
            "value": round(E * args.steps / t_run, 1), "unit": "element-updates/s",
            "node_update": {"avg_launch_ms": round(node_ms, 5),
                            "avg_launch_ms_without_dose": round(node_plain, 5),
                            "achieved_GBps": round(node_bytes / (node_ms * 1e-3) / 1e9, 1),
                            "algorithmic_bytes_per_launch": node_bytes},
            "max_rel_dose_error_vs_oracle": rel, "max_abs_dT_vs_oracle_K": dT,
            "oracle_check": (f"{g['n_steps']} steps from the initial state, untimed, "
                             f"{len(g['idx'])} sampled nodes") if g else None}


def run_hex(args):
    """The same ellipsoid as eight-node hexahedra (2.91M elements, 2.99M
    nodes): element-updates/s over --steps captured steps, the element
    kernel's roofline, the result against the oracle's stored sample of the
    same run, and the FP64 oracle timed on a few steps."""
    import numpy as np
    from paper_1909_05098_amd import fedfem as ff
    from synth import scenarios as sc

    t0 = time.perf_counter()
    scn = sc.hex_ellipsoid("random", h=args.h, n_steps=args.steps)
    log(f"hex mesh {scn.n_tets} hexahedra {scn.n_nodes} nodes ({time.perf_counter() - t0:.1f} s)")
    golden = None
    if os.path.exists(GOLDEN_HEX):
        golden = json.load(open(GOLDEN_HEX))
        if golden["n_hexes"] != scn.n_tets:
            golden = None
    h = ff.Handle(scn.xyz, scn.tets, scn.materials, scn.T0, scn.dir_nodes, scn.dir_T,
                  dt=golden["dt"] if golden else -0.9, precision=ff.FP32C,
                  reorder=(args.order == "morton"), tile_elems=args.hex_tile,
                  threads=args.hex_threads, xcd=bool(args.hex_xcd))
    tuned = None
    if not args.no_autotune:
        t0 = time.perf_counter()
        tuned = h.autotune(TUNE_CACHE)
        log(f"hex autotune {time.perf_counter() - t0:.2f} s -> {tuned}")
    t0 = time.perf_counter()
    h.precompute()
    t_pre = time.perf_counter() - t0
    info = h.info()
    xcd = int(tuned["xcd"]) if tuned is not None else int(bool(args.hex_xcd))
    dt, dt_cr = h.dt()
    log(f"hex precompute {t_pre:.2f} s, dt={dt:.6g} dt_cr={dt_cr:.6g}, tiles={info['n_tiles']}")
    h.set_gaussian_sources(scn.sources, ff.SOURCE_NODAL)
    import torch
    stream = torch.cuda.Stream()
    h.set_stream(stream.cuda_stream)
    state0, _, _ = h.read_state()
    h.prepare(args.steps)
    if args.warmup:
        h.step(args.warmup)
    h.write_state(state0, 0.0, 0)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    h.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    t_run = time.perf_counter() - t0
    ev_ms_step = ev0.elapsed_time(ev1) / args.steps
    E, N = scn.n_tets, scn.n_nodes
    # as for the tetrahedral leg: the element kernel's share of the timed
    # steps is the step time by HIP events less the node pass timed alone
    elem_iso_ms, node_ms = h.time_kernels(args.kernel_steps)
    elem_ms = ev_ms_step - node_ms
    max_err = check_vs_golden(h, state0, golden, E)
    if max_err is not None:
        log(f"hex: max|T - T_oracle| on {len(golden['idx'])} sampled nodes after "
            f"{golden['n_steps']} steps = {max_err:.3e} K")
    h.close()
    # algorithmic bytes per hexahedron: the six f32 entries of its 3 x 3
    # matrix S (A_e = Xi^T S Xi) and eight 32-bit node ids (the layout stores
    # 16-bit tile-local ids)
    elem_bytes = 56.0 * E
    node_bytes = 24.0 * N
    achieved = elem_bytes / (elem_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": "elem_loads_hex", "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4),
                "traffic": read_traffic(E, info["tile_elems"], info["threads"], xcd,
                                        PMC_SUMMARY_HEX, "n_hexes"),
                "algorithmic_bytes_per_launch": elem_bytes, "avg_launch_ms": round(elem_ms, 5),
                "avg_launch_ms_how": ("timed steps by HIP events on the kernels' stream, "
                                      "less the node pass timed alone"),
                "avg_launch_ms_alone": round(elem_iso_ms, 5),
                "frac_alone": round(elem_bytes / (elem_iso_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)}
    cpu = None
    if not args.no_cpu:
        from oracle import hex as ohx
        import oracle
        t0 = time.perf_counter()
        m = ohx.HexModel(scn.xyz, scn.tets, oracle.mat_vector(scn.materials),
                         scn.dir_nodes, scn.dir_T, dt=dt)
        q = m.source_nodal(scn.sources)
        setup = time.perf_counter() - t0
        T = m.initial(scn.T0)
        t0 = time.perf_counter()
        T = m.run(T, args.hex_cpu_steps, q)
        el = time.perf_counter() - t0
        cpu = {"value": round(E * args.hex_cpu_steps / el, 1), "unit": "element-updates/s",
               "cores": 1, "kind": "oracle",
               "sample": f"FP64 NumPy hexahedral oracle, {args.hex_cpu_steps} steps of the "
                         f"same mesh from the initial state ({el:.1f} s timed, {setup:.1f} s "
                         f"untimed setup)"}
    return {"workload": f"ellipsoid 75x50x40 mm as eight-node reduced-integration "
                        f"hexahedra, jittered lattice h={args.h * 1e3:g} mm, TD k(T) c(T), "
                        f"two Gaussian sources (nodal), {args.order} order",
            "n_hexes": E, "n_nodes": N, "steps": args.steps, "dt_s": dt,
            "value": round(E * args.steps / t_run, 1), "unit": "element-updates/s",
            "ms_per_step": round(t_run * 1e3 / args.steps, 5),
            "ms_per_step_hip_events": round(ev_ms_step, 5),
            "tile_elems": info["tile_elems"], "threads": info["threads"], "xcd": xcd,
            "roofline": roofline,
            "node_update": {"avg_launch_ms": round(node_ms, 5),
                            "achieved_GBps": round(node_bytes / (node_ms * 1e-3) / 1e9, 1)},
            "max_abs_dT_vs_oracle_K": max_err,
            "oracle_check": (f"{golden['n_steps']} steps from the initial state, untimed, "
                             f"{len(golden['idx'])} sampled nodes") if golden else None,
            "precompute_s": round(t_pre, 3), "cpu_baseline": cpu}


def run_other_order(scn, golden, args):
    """Config 3 in the order the headline did not use: with the library's
    Morton renumbering when the headline kept the seeded random input order,
    else the random input order as handed over (library default tiles, no
    autotuning, since the autotuner would pick the renumbered layout).
    --steps timed steps, kernel times by HIP events, and the stored oracle
    run checked after rewinding."""
    import torch
    from paper_1909_05098_amd import fedfem as ff
    morton = args.order != "morton"
    h = ff.Handle(scn.xyz, scn.tets, scn.materials, scn.T0, scn.dir_nodes, scn.dir_T,
                  dt=golden["dt"] if golden else -0.9, precision=ff.FP32C, reorder=morton)
    t0 = time.perf_counter()
    h.precompute()
    t_pre = time.perf_counter() - t0
    info = h.info()
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
    elem_ms, node_ms = h.time_kernels(args.kernel_steps)
    err = check_vs_golden(h, state0, golden, scn.n_tets)
    h.close()
    E, N = scn.n_tets, scn.n_nodes
    log(f"{'morton' if morton else 'random'} order: {t_run * 1e3 / args.steps:.4f} ms/step, "
        f"element kernel {elem_ms:.4f} ms, node pass {node_ms:.4f} ms, max|dT| {err}")
    return {"order": "morton" if morton else "random",
            "value": round(E * args.steps / t_run, 1), "unit": "element-updates/s",
            "ms_per_step": round(t_run * 1e3 / args.steps, 5),
            "tile_elems": info["tile_elems"], "threads": info["threads"],
            "max_tile_nodes": info["max_tile_nodes"], "n_tiles": info["n_tiles"],
            "n_partials": info["n_partials"],
            "elem_loads": {"avg_launch_ms": round(elem_ms, 5),
                           "achieved_GBps": round(40.0 * E / (elem_ms * 1e-3) / 1e9, 1)},
            "node_update": {"avg_launch_ms": round(node_ms, 5),
                            "achieved_GBps": round(24.0 * N / (node_ms * 1e-3) / 1e9, 1)},
            "max_abs_dT_vs_oracle_K": err, "precompute_s": round(t_pre, 3)}


def run_config12(args):
    """Configs 1 and 2, whole runs at the oracle's own step, in FP64 and in
    compensated FP32: element-updates/s of the captured steps and the error
    against the oracle's stored result (every node of config 1, 4096
    sampled nodes of config 2)."""
    import numpy as np
    import torch
    from paper_1909_05098_amd import fedfem as ff
    from synth import scenarios as sc
    out = {}
    for name, make, path in (("config1", sc.config1, GOLDEN1), ("config2", sc.config2, GOLDEN2)):
        s = make()
        g = load_golden(path, "n_tets", s.n_tets)
        if g is None:
            continue
        rec = {"workload": ("1 cm cube, 10^3 Kuhn cubes, constant properties, nodal "
                            "Gaussian source, 300 s" if name == "config1" else
                            "ellipsoid 75x50x40 mm, jittered lattice h=1.2 mm, TD k(T) "
                            "c(T), consistent Gaussian source, 600 s"),
               "n_tets": s.n_tets, "n_nodes": s.n_nodes, "steps": g["n_steps"],
               "dt_s": g["dt"]}
        T_prec = {}
        for prec, label in ((ff.FP64, "fp64"), (ff.FP32C, "fp32c")):
            h = ff.Handle(s.xyz, s.tets, s.materials, s.T0, s.dir_nodes, s.dir_T,
                          dt=g["dt"], precision=prec)
            h.precompute()
            h.set_gaussian_sources(s.sources, s.source_mode)
            state0, _, _ = h.read_state()
            h.prepare(g["n_steps"])
            h.step(min(args.warmup, g["n_steps"]) if args.warmup else 0)
            h.write_state(state0, 0.0, 0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h.step(g["n_steps"])
            torch.cuda.synchronize()
            t_run = time.perf_counter() - t0
            T = h.read_T()
            if "idx" in g:
                T = T[np.asarray(g["idx"])]
            T_prec[label] = T
            err = float(np.max(np.abs(T - np.asarray(g["T"]))))
            elem_ms, node_ms = h.time_kernels(args.kernel_steps)
            h.close()
            rec[label] = {"value": round(s.n_tets * g["n_steps"] / t_run, 1),
                          "unit": "element-updates/s",
                          "ms_per_step": round(t_run * 1e3 / g["n_steps"], 5),
                          "elem_loads_ms": round(elem_ms, 5), "node_update_ms": round(node_ms, 5),
                          "max_abs_dT_vs_oracle_K": err}
            log(f"{name} {label}: {t_run * 1e3 / g['n_steps']:.4f} ms/step, max|dT| {err:.3e} K")
        rec["max_abs_dT_fp32c_vs_fp64_K"] = float(np.max(np.abs(T_prec["fp32c"] - T_prec["fp64"])))
        out[name] = rec
    return out


def _gen_sweep_one(j):
    from synth import scenarios as sc
    return sc.sweep_scenario(j)


def _gen_sweep_one_v2(j):
    from synth import scenarios as sc
    return sc.sweep_scenario(j, mesh_variant=2)


def gen_sweep(ids, workers, variant=1):
    """Seeded planning-sweep scenarios, built on host cores before any GPU
    use in this process (the pool forks); variant 2 re-seeds only the
    interior-node jitter of each mesh."""
    from multiprocessing import get_context
    with get_context("fork").Pool(workers) as pool:
        return pool.map(_gen_sweep_one if variant == 1 else _gen_sweep_one_v2, list(ids))


def run_sweep(scns, autotune=True, recs=None):
    """Scenarios/s for the planning sweep: plain per-scenario use of the
    library versus one batched graph launch, on the same GPU."""
    import numpy as np
    from paper_1909_05098_amd import fedfem as ff
    from synth import scenarios as sc

    # with the oracle's stored runs of these scenarios, both legs take the
    # oracle's own step and step count, so the results can be checked
    # against it; otherwise each handle's own critical step
    if recs is not None and [r["j"] for r in recs[:len(scns)]] != list(range(len(scns))):
        recs = None
    rec_of = (lambda i: recs[i]) if recs is not None else (lambda i: None)  # noqa: E731

    def handle(i, s):
        r = rec_of(i)
        h = ff.Handle(s.xyz, s.tets, s.materials, s.T0, s.dir_nodes, s.dir_T,
                      dt=r["dt"] if r else -0.9, precision=ff.FP32C)
        if autotune:
            h.autotune(TUNE_CACHE, for_batch=True)
        h.precompute()
        h.set_gaussian_sources(s.sources, s.source_mode)
        if r:
            return h, r["n_steps"]
        _, dtcr = h.dt()
        n, dt = sc.steps_for(s.t_end, dtcr)
        h.set_dt(dt)
        return h, n

    def oracle_err(i, T):
        r = rec_of(i)
        if not r:
            return None
        return float(np.max(np.abs(T[np.asarray(r["idx"])] - np.asarray(r["T"]))))

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
    for i, s in enumerate(scns):
        t0 = time.perf_counter()
        h, n = handle(i, s)
        t1 = time.perf_counter()
        h.step(n)
        plain_T.append(h.read_T())
        t2 = time.perf_counter()
        h.close()
        t_all += t2 - t0
        t_steps += t2 - t1
        ns.append(n)
    log(f"sweep plain: {len(scns)} scenarios in {t_all:.2f} s ({t_steps:.2f} s stepping)")
    # batched: all handles (precompute overlapped on host threads), one
    # captured launch sequence
    t0 = time.perf_counter()
    hs = []
    for i, s in enumerate(scns):
        r = rec_of(i)
        h = ff.Handle(s.xyz, s.tets, s.materials, s.T0, s.dir_nodes, s.dir_T,
                      dt=r["dt"] if r else -0.9, precision=ff.FP32C)
        if autotune:
            h.autotune(TUNE_CACHE, for_batch=True)
        hs.append(h)
    ff.precompute_many(hs)
    for i, (h, s) in enumerate(zip(hs, scns)):
        h.set_gaussian_sources(s.sources, s.source_mode)
        if not rec_of(i):
            h.set_dt(sc.steps_for(s.t_end, h.dt()[1])[1])
    t1 = time.perf_counter()
    b = ff.Batch(hs)
    t2 = time.perf_counter()
    b.run(ns)
    t3 = time.perf_counter()
    batched_T = [h.read_T() for h in hs]
    dT = max(float(np.max(np.abs(Tb - T))) for Tb, T in zip(batched_T, plain_T))
    e_b = [oracle_err(i, T) for i, T in enumerate(batched_T)]
    e_p = [oracle_err(i, T) for i, T in enumerate(plain_T)]
    e_b = max(e_b) if recs is not None else None
    e_p = max(e_p) if recs is not None else None
    if e_b is not None:
        log(f"sweep: worst sampled max|T - T_oracle| batched {e_b:.3e} K, plain {e_p:.3e} K")
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
            "max_abs_dT_batched_vs_plain_K": dT,
            "max_abs_dT_batched_vs_oracle_K": e_b, "max_abs_dT_plain_vs_oracle_K": e_p,
            "oracle_check": ("every scenario at the oracle's own step, its 512 hottest "
                             "and 32 drawn nodes, worst over scenarios")
                            if recs is not None else None}


def forward_flops(G):
    """Multiply-adds x 2 of one forward pass of the surrogate on a G^3 grid."""
    from paper_1909_05098_amd import surrogate as sg
    f = sum(2 * 27 * ci * co * (G >> lv) ** 3 for (_, ci, co), lv in zip(sg.LAYERS, sg.LEVEL))
    return f + 2 * 32 * G ** 3


def run_surrogate(scns, weights, net_batch=16, check_batch=64, scns_b=None):
    """Scenarios/s of FED-FEM (one at a time, batched) and of the trained
    surrogate (raw, and with the 1/16 FED-FEM spot check and fallback) on
    held-out scenarios, with each path's error against FED-FEM on the grid."""
    import numpy as np
    import torch
    from paper_1909_05098_amd import surrogate as sg
    from paper_1909_05098_amd import surrogate_pipeline as pl

    S, G = len(scns), pl.GRID
    fr = pl.frame(G)
    phys = pl.phys_of(scns[0].materials)
    stream = torch.cuda.current_stream().cuda_stream
    samples = torch.tensor(np.array([pl.sample_row(s) for s in scns]), device="cuda")
    f32, u8 = torch.float32, torch.uint8

    def field():
        return torch.empty((S, G, G, G), dtype=f32, device="cuda")

    def errors(Tp, T, M):
        e = torch.empty(S, dtype=f32, device="cuda")
        sg.max_error(G, Tp, T, M, e, stream)
        return e.cpu().numpy().astype(np.float64)

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, r

    T, M = field(), torch.empty((S, G, G, G), dtype=u8, device="cuda")
    t_batched, _ = timed(lambda: pl.fem_on_grid(scns, T, M, G, fr))
    log(f"surrogate leg: FED-FEM batched {S} scenarios {t_batched:.2f} s")
    T1, M1 = field(), torch.empty_like(M)
    t_plain, _ = timed(lambda: pl.fem_on_grid(scns, T1, M1, G, fr, batched=False))
    d_plain = float(errors(T1, T, M).max())
    del T1, M1
    log(f"surrogate leg: FED-FEM plain {t_plain:.2f} s (max diff to batched {d_plain:.2e} K)")
    net = sg.Net(G, net_batch, seed=0)
    pl.load_params(net, weights)
    pred = field()
    pl.predict(net, samples[:net_batch], phys, pred[:net_batch], net_batch, G, fr)  # warm-up
    t_raw, _ = timed(lambda: pl.predict(net, samples, phys, pred, net_batch, G, fr))
    e_raw = errors(pred, T, M)
    zero = sg.Net(G, net_batch, seed=0)
    zero.set_params(np.zeros(zero.n_params, dtype=np.float32))
    pl.predict(zero, samples, phys, pred, net_batch, G, fr)
    e_prior = errors(pred, T, M)
    zero.close()
    out = field()
    t_fb, stats = timed(lambda: pl.infer_with_fallback(net, scns, samples, phys, out,
                                                        batch=check_batch, grid=G, fr=fr,
                                                        net_batch=net_batch))
    e_fb = errors(out, T, M)
    log(f"surrogate leg: raw {t_raw:.3f} s, with fallback {t_fb:.2f} s, "
        f"fallback batches {stats['fallback_batches']}/{stats['batches']}")
    # the same spot check at looser bounds
    loose = {}
    for tol in (1.0, 2.0):
        t_l, st = timed(lambda: pl.infer_with_fallback(net, scns, samples, phys, out,
                                                        batch=check_batch, grid=G, fr=fr,
                                                        net_batch=net_batch, tol=tol))
        e_l = errors(out, T, M)
        loose[f"{tol:g}K"] = {"fallback_batches": st["fallback_batches"],
                              "batches": st["batches"],
                              "scenarios_per_s": round(S / t_l, 2),
                              "max_abs_dT_K_median": round(float(np.median(e_l)), 3),
                              "max_abs_dT_K_max": round(float(e_l.max()), 3)}
        log(f"surrogate leg: spot check at {tol:g} K: fallback batches "
            f"{st['fallback_batches']}/{st['batches']}, {S / t_l:.1f} scen/s")
    # FED-FEM on a second mesh of every scenario (same parameters and
    # elements, another jitter seed) against the first: how far a prediction
    # that does not see the mesh can be expected to land
    spread = None
    if scns_b is not None:
        TB, MB = field(), torch.empty_like(M)
        pl.fem_on_grid(scns_b, TB, MB, G, fr)
        e_sp = errors(TB, T, M)
        spread = {"median": round(float(np.median(e_sp)), 3),
                  "p90": round(float(np.quantile(e_sp, 0.9)), 3),
                  "max": round(float(e_sp.max()), 3),
                  "within_K": {f"{t:g}": round(float(np.mean(e_sp <= t)), 4)
                               for t in (0.5, 1.0, 2.0)},
                  "same_voxels": bool(torch.equal(M, MB))}
        del TB, MB
        log(f"surrogate leg: FED-FEM mesh-to-mesh spread median {spread['median']} K, "
            f"p90 {spread['p90']} K")
    # training throughput of the same network (a fresh copy, 12 steps timed)
    tr = sg.Net(G, 8, seed=1)
    tr.set_stream(stream)
    ws = pl.Workspace(8, G)
    idx = torch.arange(8, device="cuda")

    def train_steps(n):
        for _ in range(n):
            sg.rasterize(G, fr, samples[:8], phys, ws.X, ws.prior, ws.scale, stream)
            sg.target(G, ws.prior, ws.scale, T.index_select(0, idx), M.index_select(0, idx),
                      37.0, ws.target, ws.maskf, pl.FOCUS, stream)
            tr.loss_backward(ws.X, ws.target, ws.maskf)
            tr.adam_step(1e-4)

    train_steps(2)
    t_tr, _ = timed(lambda: train_steps(12))
    tr.close()
    net.close()
    ff_flops = forward_flops(G)
    q = lambda e: {"median": round(float(np.median(e)), 3),  # noqa: E731
                   "p90": round(float(np.quantile(e, 0.9)), 3), "max": round(float(e.max()), 3)}
    return {"workload": f"learned surrogate on a {G}^3 frame (2.5 mm voxels), {S} held-out "
                        f"planning-sweep seeds 10000..{10000 + S - 1}, 300 s heating",
            "scenarios": S,
            "fedfem_plain_scenarios_per_s": round(S / t_plain, 2),
            "fedfem_batched_scenarios_per_s": round(S / t_batched, 2),
            "surrogate_raw_scenarios_per_s": round(S / t_raw, 1),
            "surrogate_with_fallback_scenarios_per_s": round(S / t_fb, 2),
            "gain_raw_vs_batched": round(t_batched / t_raw, 1),
            "gain_with_fallback_vs_batched": round(t_batched / t_fb, 3),
            "spot_check_tol_K": pl.TOL_K, "fallback_batches": stats["fallback_batches"],
            "batches": stats["batches"], "fedfem_runs_in_surrogate_path": stats["fedfem_runs"],
            "max_abs_dT_K": {"surrogate_raw": q(e_raw), "prior_only": q(e_prior),
                             "with_fallback": q(e_fb), "fedfem_plain_vs_batched": d_plain},
            "surrogate_raw_within_K": {f"{t:g}": round(float(np.mean(e_raw <= t)), 4)
                                       for t in (0.5, 1.0, 2.0)},
            "spot_check_looser": loose,
            "fedfem_mesh_to_mesh_max_abs_dT_K": spread,
            "forward_TFLOPs": round(ff_flops * S / t_raw / 1e12, 1),
            "forward_mfma_frac_bf16": round(ff_flops * S / t_raw / 1e12 / 2500.0, 4),
            "train_sample_steps_per_s": round(12 * 8 / t_tr, 1),
            "train_TFLOPs": round(3 * ff_flops * 12 * 8 / t_tr / 1e12, 1)}


def run_network_only(steps, batch=8, grid=64):
    """Only the surrogate network's kernels, for profiling them: `steps`
    forward passes and `steps` training steps (loss, backward, Adam) at
    `batch` samples of the held-out sweep's parameters (no FED-FEM run;
    target zero, unit weights).  Prints the network's TFLOP/s."""
    import numpy as np
    import torch
    from paper_1909_05098_amd import surrogate as sg
    from paper_1909_05098_amd import surrogate_pipeline as pl
    from synth import scenarios as sc
    G = grid
    fr = pl.frame(G)
    rows = []
    for j in range(10000, 10000 + batch):
        p = sc.sweep_params(j)
        rows.append([*p["pos"], p["sigma"], p["q0"], p["k0"], p["omega_b"], *p["axes"],
                     p["h"], 0.0])
    samples = torch.tensor(np.array(rows), device="cuda")
    phys = pl.phys_of(sc.td_materials())
    stream = torch.cuda.current_stream().cuda_stream
    ws = pl.Workspace(batch, G)
    sg.rasterize(G, fr, samples, phys, ws.X, ws.prior, ws.scale, stream)
    ws.target.zero_()
    ws.maskf.fill_(1.0)
    net = sg.Net(G, batch, seed=3)
    net.set_stream(stream)
    net.forward(ws.X, ws.Y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        net.forward(ws.X, ws.Y)
    torch.cuda.synchronize()
    t_f = (time.perf_counter() - t0) / steps
    net.loss_backward(ws.X, ws.target, ws.maskf)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        net.loss_backward(ws.X, ws.target, ws.maskf)
        net.adam_step(1e-4)
    torch.cuda.synchronize()
    t_t = (time.perf_counter() - t0) / steps
    net.close()
    f = forward_flops(G) * batch
    return {"batch": batch, "grid": G, "forward_ms": round(t_f * 1e3, 3),
            "forward_TFLOPs": round(f / t_f / 1e12, 1),
            "train_step_ms": round(t_t * 1e3, 3), "train_TFLOPs": round(3 * f / t_t / 1e12, 1)}


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
    ap.add_argument("--surrogate", type=int, default=512,
                    help="held-out scenarios for the surrogate leg (0 = skip)")
    ap.add_argument("--surrogate-weights", default=os.path.join(
        ROOT, "paper_1909_05098_amd", "weights", "surrogate_g64.npy"))
    ap.add_argument("--surrogate-only", action="store_true",
                    help="run only the surrogate leg and print its result (for profiling "
                         "its kernels); not a benchmark line")
    ap.add_argument("--network-only", type=int, default=0,
                    help="run only the surrogate network's forward and training kernels "
                         "this many times each (for profiling them); not a benchmark line")
    ap.add_argument("--dose", type=int, default=1,
                    help="also time config 3 with the CEM43 dose (0 to skip)")
    ap.add_argument("--other-order", type=int, default=1,
                    help="also time config 3 in the other element/node order (0 to skip)")
    ap.add_argument("--small", type=int, default=1,
                    help="also time configs 1 and 2 in both precisions (0 to skip)")
    ap.add_argument("--cpu-sweep-seconds", type=float, default=8.0,
                    help="seconds of the CPU oracle on whole sweep scenarios (0 to skip)")
    ap.add_argument("--hex", type=int, default=1,
                    help="also run the hexahedral ellipsoid (0 to skip)")
    ap.add_argument("--hex-only", action="store_true",
                    help="run only the hexahedral ellipsoid leg")
    ap.add_argument("--hex-tile", type=int, default=0)
    ap.add_argument("--hex-threads", type=int, default=0)
    ap.add_argument("--hex-xcd", type=int, default=0)
    ap.add_argument("--hex-cpu-steps", type=int, default=4)
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
    if args.sweep and not (args.copy_calib_gib or args.surrogate_only or args.hex_only
                           or args.network_only):
        t0 = time.perf_counter()
        sweep_scns = gen_sweep(range(args.sweep), min(16, os.cpu_count() or 1))
        log(f"sweep meshes: {len(sweep_scns)} scenarios "
            f"({sum(s.n_tets for s in sweep_scns)} tets, {time.perf_counter() - t0:.1f} s)")
    sur_scns = sur_scns_b = None
    if args.surrogate and not args.copy_calib_gib and not args.hex_only and not args.network_only:
        t0 = time.perf_counter()
        sur_scns = gen_sweep(range(10000, 10000 + args.surrogate), min(16, os.cpu_count() or 1))
        sur_scns_b = gen_sweep(range(10000, 10000 + args.surrogate),
                               min(16, os.cpu_count() or 1), variant=2)
        log(f"surrogate held-out meshes: {len(sur_scns)}, twice ({time.perf_counter() - t0:.1f} s)")
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
    if args.network_only:
        print(json.dumps({"network": run_network_only(args.network_only)}), flush=True)
        return
    if args.surrogate_only:
        print(json.dumps({"surrogate": run_surrogate(sur_scns, args.surrogate_weights,
                                                         scns_b=sur_scns_b)}),
              flush=True)
        return
    if args.hex_only:
        print(json.dumps({"hex": run_hex(args)}), flush=True)
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
    xcd = int(tuned["xcd"]) if tuned is not None else int(bool(args.xcd))
    dt, dt_cr = h.dt()
    log(f"precompute {t_pre:.2f} s, dt={dt:.6g} dt_cr={dt_cr:.6g}, tiles="
        f"{info['n_tiles']} partials={info['n_partials']} "
        f"lanczos={info['lanczos_iterations']}")
    h.set_gaussian_sources(scn.sources, ff.SOURCE_CONSISTENT)
    # the handle launches on a torch stream, so HIP events recorded on it
    # bracket the timed steps
    stream = torch.cuda.Stream()
    h.set_stream(stream.cuda_stream)
    state0, _, _ = h.read_state()
    h.prepare(args.steps)
    if args.warmup:
        h.step(args.warmup)
    h.write_state(state0, 0.0, 0)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    h.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    t_run = time.perf_counter() - t0
    ev_ms_step = ev0.elapsed_time(ev1) / args.steps
    log(f"timed {args.steps} steps in {t_run * 1e3:.2f} ms ({ev_ms_step:.5f} ms per step "
        f"by HIP events)")
    E, N = scn.n_tets, scn.n_nodes
    value = E * args.steps / t_run
    ms_step = t_run * 1e3 / args.steps
    # each kernel timed alone, back to back, with HIP events on the handle's
    # stream; the element kernel's share of the timed steps is the step time
    # by events less the node pass (launch gaps counted against it)
    elem_iso_ms, node_ms = h.time_kernels(args.kernel_steps)
    elem_ms = ev_ms_step - node_ms
    max_err = check_vs_golden(h, state0, golden, scn.n_tets)
    if max_err is not None:
        log(f"max|T - T_oracle| on {len(golden['idx'])} sampled nodes after "
            f"{golden['n_steps']} steps = {max_err:.3e} K")
    # algorithmic bytes per element-update of the stencil: six f32 coefficients
    # and four 32-bit node ids (the layout itself stores 10- or 16-bit
    # tile-local ids)
    elem_bytes = 40.0 * E
    node_bytes = 24.0 * N   # T hi/lo read+write, 1/V_i, source
    kern = {"elem_loads": (elem_ms, elem_bytes), "node_update": (node_ms, node_bytes)}
    dom = max(kern, key=lambda k: kern[k][0])
    ms, by = kern[dom]
    achieved = by / (ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4),
                "traffic": (read_traffic(E, info["tile_elems"], info["threads"], xcd)
                            if dom == "elem_loads" else None),
                "algorithmic_bytes_per_launch": by, "avg_launch_ms": round(ms, 5),
                "avg_launch_ms_how": ("timed steps by HIP events on the kernels' stream, "
                                      "less the node pass timed alone"
                                      if dom == "elem_loads" else "timed alone, back to back"),
                "avg_launch_ms_alone": round(elem_iso_ms if dom == "elem_loads" else ms, 5),
                "frac_alone": round(by / ((elem_iso_ms if dom == "elem_loads" else ms) * 1e-3)
                                    / 1e9 / HBM_PEAK_GBPS, 4)}
    other = [k for k in kern if k != dom][0]
    step_gbps = (elem_bytes + node_bytes) / (ms_step * 1e-3) / 1e9
    dose_leg = run_dose(h, state0, args, E, N, ms_step) if args.dose else None
    h.close()
    order_leg = run_other_order(scn, golden, args) if args.other_order else None
    small = run_config12(args) if args.small else None
    sweep_recs = None
    if sweep_scns and os.path.exists(GOLDEN_SWEEP):
        sweep_recs = json.load(open(GOLDEN_SWEEP))["scenarios"]
        if len(sweep_recs) < len(sweep_scns):
            sweep_recs = None
    batched = run_sweep(sweep_scns, not args.no_autotune, sweep_recs) if sweep_scns else None
    surrogate = run_surrogate(sur_scns, args.surrogate_weights, scns_b=sur_scns_b) \
        if sur_scns else None
    if surrogate is not None:
        # the network alone at batch 8 (20 forward passes, 20 training steps):
        # its kernels' rate without the rasteriser, decoder and resampler
        surrogate["network_batch8"] = run_network_only(20)
        log(f"surrogate network alone at batch 8: {surrogate['network_batch8']}")
    hexleg = run_hex(args) if args.hex else None
    cpu = None
    if not args.no_cpu:
        log("timing the FP64 CPU oracle on a bounded sample")
        cpu = cpu_baseline(scn, dt, scn.sources, args.cpu_seconds,
                           sweep_scns if args.cpu_sweep_seconds > 0 else None,
                           args.cpu_sweep_seconds)
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "element-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5), "ms_per_step_hip_events": round(ev_ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"ellipsoid 75x50x40 mm, jittered Kuhn lattice "
                               f"h={args.h * 1e3:g} mm, TD k(T) c(T), two "
                               f"Gaussian sources, {args.order} order",
                   "n_tets": E, "n_nodes": N, "dt_s": dt,
                   "precision": "f32 element loop, compensated f32 hi/lo nodal state, f64 precompute",
                   "tile_elems": info["tile_elems"], "threads": info["threads"],
                   "xcd": xcd,
                   "autotuned": tuned is not None,
                   "parallelism": "1 GPU"},
        "roofline": roofline,
        "other_kernel": {"kernel": other, "avg_launch_ms": round(kern[other][0], 5),
                         "achieved_GBps": round(kern[other][1] / (kern[other][0] * 1e-3) / 1e9, 1)},
        "step_GBps_algorithmic": round(step_gbps, 1),
        "max_abs_dT_vs_oracle_K": max_err,
        "oracle_check": (f"{golden['n_steps']} steps from the initial state, untimed, "
                         f"{len(golden['idx'])} sampled nodes (512 hottest, 3584 drawn)")
                        if golden else None,
        "precompute_s": round(t_pre, 3),
        "other_order": order_leg,
        "configs_1_2": small,
        "batched": batched,
        "surrogate": surrogate,
        "dose": dose_leg,
        "hex": hexleg,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
