"""Surrogate workflow around the library: FED-FEM temperature fields on a
voxel grid as training data, training with the library's forward / backward /
Adam kernels, and inference with a FED-FEM spot check and fallback.

Python only sequences library calls here (and indexes device tensors); every
numerical step -- FED-FEM precompute and stepping, resampling, rasterising,
the network, the loss, the error judge -- runs in the library's kernels.

Scenarios are duck-typed: any object with the attributes xyz, tets,
materials, T0, dir_nodes, dir_T, sources, source_mode, t_end, h, semi_axes
(the ellipsoid centred on the origin) and one Gaussian source row
(cx, cy, cz, sigma, Q0) with the perfusion rate in materials.w_b / rho_b.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import fedfem as ff
from . import surrogate as sg

GRID = 64
FRAME_EDGE = 0.16      # m: the voxel frame, centred on the ellipsoid
T_HEAT = 300.0         # s
RHO_B = 1000.0         # kg/m^3, blood density behind w_b = omega_b rho_b
SPOT_FRACTION = 16     # one scenario in 16 of each inference batch is checked
TOL_K = 0.5            # spot-check bound on max |dT_surrogate - dT_FED-FEM|
FOCUS = 20.0           # loss weight 1 + FOCUS prior / P: leans on the heated region


def frame(grid=GRID, edge=FRAME_EDGE):
    h = edge / grid
    return np.array([-0.5 * edge, -0.5 * edge, -0.5 * edge, h])


def phys_of(materials, t_heat=T_HEAT):
    return (materials.rho0, materials.c0, RHO_B * materials.c_b, t_heat)


def sample_row(s):
    """fedsur_sample record of a scenario."""
    cx, cy, cz, sigma, q0 = (float(v) for v in np.asarray(s.sources)[0])
    m = s.materials
    ax, ay, az = s.semi_axes
    return [cx, cy, cz, sigma, q0, m.k0, m.w_b / RHO_B, ax, ay, az, s.h, 0.0]


def steps_for(t_end, dt_cr, fraction=0.9):
    n = max(1, int(math.ceil(t_end / (fraction * dt_cr) - 1e-12)))
    return n, t_end / n


# -- FED-FEM fields on the grid ---------------------------------------------
def fem_handles(scns, tune_cache=None, threads=0):
    """Created and precomputed handles (precompute overlapped on host threads)
    with their sources and step counts."""
    hs, ns = [], []
    for s in scns:
        h = ff.Handle(s.xyz, s.tets, s.materials, s.T0, s.dir_nodes, s.dir_T, dt=-0.9,
                      precision=ff.FP32C)
        if tune_cache:
            h.autotune(tune_cache, for_batch=True)
        hs.append(h)
    ff.precompute_many(hs, threads)
    for h, s in zip(hs, scns):
        h.set_gaussian_sources(s.sources, s.source_mode)
        _, dtcr = h.dt()
        n, dt = steps_for(s.t_end, dtcr)
        h.set_dt(dt)
        ns.append(n)
    return hs, ns


def fem_on_grid(scns, T_out, M_out, grid=GRID, fr=None, tune_cache=None, batched=True):
    """Run FED-FEM for every scenario to its t_end (one batched launch, or
    one scenario at a time) and resample T onto the grid: T_out float32
    [S, G, G, G], M_out uint8 [S, G, G, G] (cuda)."""
    fr = frame(grid) if fr is None else fr
    if batched:
        hs, ns = fem_handles(scns, tune_cache)
        b = ff.Batch(hs)
        b.run(ns)
        b.close()
        for i, h in enumerate(hs):
            sg.resample(h, grid, fr, T_out[i], M_out[i])
            h.close()
    else:
        for i, s in enumerate(scns):
            (h,), (n,) = fem_handles([s], tune_cache)
            h.step(n)
            sg.resample(h, grid, fr, T_out[i], M_out[i])
            h.close()


# -- training -----------------------------------------------------------------
class Workspace:
    """Device buffers for one minibatch of the network's input and target."""

    def __init__(self, batch, grid=GRID):
        G = grid
        dev = "cuda"
        self.X = torch.empty((batch, G, G, G, 8), dtype=torch.bfloat16, device=dev)
        self.prior = torch.empty((batch, G, G, G), dtype=torch.float32, device=dev)
        self.scale = torch.empty(batch, dtype=torch.float32, device=dev)
        self.target = torch.empty((batch, G, G, G), dtype=torch.float32, device=dev)
        self.maskf = torch.empty((batch, G, G, G), dtype=torch.float32, device=dev)
        self.Y = torch.empty((batch, G, G, G), dtype=torch.float32, device=dev)


def train(net, samples, T, M, phys, epochs, batch, lr, grid=GRID, fr=None, seed=0,
          lr_min=1e-5, focus=FOCUS, log=None):
    """Adam on the weighted MSE of (T - T_a - prior) / P over the training
    set (samples float64 cuda [S, 12], T float32 / M uint8 cuda
    [S, G, G, G]; weights 1 + focus prior / P inside the mesh), cosine
    learning-rate decay from lr to lr_min.  Returns per-epoch mean losses."""
    fr = frame(grid) if fr is None else fr
    S = samples.shape[0]
    ws = Workspace(batch, grid)
    stream = torch.cuda.current_stream().cuda_stream
    net.set_stream(stream)
    rng = np.random.default_rng(seed)
    steps_per_epoch = S // batch
    total = epochs * steps_per_epoch
    k = 0
    history = []
    for ep in range(epochs):
        order = torch.tensor(rng.permutation(S), device="cuda")
        acc = 0.0
        t0 = time.perf_counter()
        for i in range(steps_per_epoch):
            idx = order[i * batch:(i + 1) * batch]
            smp = samples.index_select(0, idx)
            sg.rasterize(grid, fr, smp, phys, ws.X, ws.prior, ws.scale, stream)
            sg.target(grid, ws.prior, ws.scale, T.index_select(0, idx), M.index_select(0, idx),
                      37.0, ws.target, ws.maskf, focus, stream)
            acc += net.loss_backward(ws.X, ws.target, ws.maskf)
            rate = lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * k / max(1, total)))
            net.adam_step(rate)
            k += 1
        history.append(acc / steps_per_epoch)
        if log:
            log(f"epoch {ep + 1}/{epochs}: loss {history[-1]:.4e} "
                f"({time.perf_counter() - t0:.1f} s)")
    return history


# -- inference ----------------------------------------------------------------
def predict(net, samples, phys, out, batch, grid=GRID, fr=None, ws=None, T_a=37.0):
    """Predicted temperature (float32 cuda [S, G, G, G]) for every sample,
    `batch` at a time."""
    fr = frame(grid) if fr is None else fr
    ws = ws or Workspace(batch, grid)
    stream = torch.cuda.current_stream().cuda_stream
    net.set_stream(stream)
    S = samples.shape[0]
    for i in range(0, S, batch):
        n = min(batch, S - i)
        sg.rasterize(grid, fr, samples[i:i + n], phys, ws.X[:n], ws.prior[:n], ws.scale[:n],
                     stream)
        net.forward(ws.X[:n], out[i:i + n])
        sg.decode(grid, ws.prior[:n], ws.scale[:n], T_a, out[i:i + n], stream)


def peak_scale(samples, phys):
    """P (the prior's centre value) of every sample, by a 1-voxel raster."""
    S = samples.shape[0]
    X = torch.empty((S, 1, 1, 1, 8), dtype=torch.bfloat16, device="cuda")
    scale = torch.empty(S, dtype=torch.float32, device="cuda")
    sg.rasterize(1, np.array([-1.0, -1.0, -1.0, 2.0]), samples, phys, X, None, scale,
                 torch.cuda.current_stream().cuda_stream)
    return scale.cpu().numpy()


def infer_with_fallback(net, scns, samples, phys, out, batch=64, grid=GRID, fr=None,
                        tol=TOL_K, seed=0, tune_cache=None, group_by_peak=True, net_batch=None):
    """Surrogate inference with a FED-FEM spot check per batch.

    Scenarios are put in batches of `batch` (by increasing predicted peak P
    when group_by_peak, so that batches are alike in difficulty).  Each
    batch is predicted by the network; a seeded 1/SPOT_FRACTION of it is
    also run through FED-FEM and compared on the grid.  If any checked
    scenario is off by more than `tol` kelvin (or not finite), the whole
    batch falls back to FED-FEM.  Checked scenarios keep their FED-FEM
    field.  out: float32 cuda [S, G, G, G] temperature (FED-FEM fields are 0
    outside their mesh).  Returns a dict of counts and `from_fedfem`, the
    scenarios whose field came from FED-FEM.
    """
    fr = frame(grid) if fr is None else fr
    S = len(scns)
    order = np.argsort(peak_scale(samples, phys), kind="stable") if group_by_peak \
        else np.arange(S)
    rng = np.random.default_rng(seed)
    net_batch = net_batch or min(batch, net.batch_max)
    ws = Workspace(net_batch, grid)
    G = grid
    n_check = n_fallback_batches = n_fem = 0
    worst_check = 0.0
    from_fem = np.zeros(S, dtype=bool)
    for b0 in range(0, S, batch):
        ids = order[b0:b0 + batch]
        n = len(ids)
        sel = torch.tensor(ids, device="cuda")
        smp = samples.index_select(0, sel)
        pred = torch.empty((n, G, G, G), dtype=torch.float32, device="cuda")
        predict(net, smp, phys, pred, net_batch, grid, fr, ws)
        k = max(1, n // SPOT_FRACTION)
        chk = np.sort(rng.choice(n, k, replace=False))
        Tc = torch.empty((k, G, G, G), dtype=torch.float32, device="cuda")
        Mc = torch.empty((k, G, G, G), dtype=torch.uint8, device="cuda")
        fem_on_grid([scns[ids[j]] for j in chk], Tc, Mc, grid, fr, tune_cache)
        err = torch.empty(k, dtype=torch.float32, device="cuda")
        ci = torch.tensor(chk, device="cuda")
        sg.max_error(grid, pred.index_select(0, ci), Tc, Mc, err,
                     torch.cuda.current_stream().cuda_stream)
        e = err.cpu().numpy()
        n_check += k
        n_fem += k
        worst_check = max(worst_check, float(np.nan_to_num(e, nan=np.inf).max()))
        # checked scenarios take their FED-FEM field (computed anyway)
        pred[ci] = Tc
        from_fem[ids[chk]] = True
        if not np.all(e <= tol):
            n_fallback_batches += 1
            rest = np.setdiff1d(np.arange(n), chk)
            if len(rest):
                Tr = torch.empty((len(rest), G, G, G), dtype=torch.float32, device="cuda")
                Mr = torch.empty((len(rest), G, G, G), dtype=torch.uint8, device="cuda")
                fem_on_grid([scns[ids[j]] for j in rest], Tr, Mr, grid, fr, tune_cache)
                pred[torch.tensor(rest, device="cuda")] = Tr
                n_fem += len(rest)
                from_fem[ids[rest]] = True
        out[sel] = pred
    return {"scenarios": S, "batches": (S + batch - 1) // batch,
            "fallback_batches": n_fallback_batches, "spot_checks": n_check,
            "fedfem_runs": n_fem, "worst_spot_check_K": worst_check, "from_fedfem": from_fem}


def save_params(net, path):
    np.save(path, net.get_params(), allow_pickle=False)


def load_params(net, path):
    net.set_params(np.load(path, allow_pickle=False))
