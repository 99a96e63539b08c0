"""Batched execution: many scenarios of the planning sweep advanced by one
graph launch must give exactly what per-handle stepping gives, and match the
FP64 oracle per scenario."""
import numpy as np
import pytest

import oracle
from oracle import dense
from paper_1909_05098_amd import fedfem as ff
from synth import scenarios as sc

pytestmark = pytest.mark.gpu

SMALL = [5, 8, 9, 13, 16, 30]


@pytest.fixture(scope="module")
def scenarios():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    out = []
    for j in SMALL:
        s = sc.sweep_scenario(j)
        om = oracle.build_model(s)
        dtcr, _ = dense.critical_dt_from_lambda(om.geometry_lambda(), om.mat)
        n, dt = sc.steps_for(s.t_end, dtcr)
        om.dt = dt
        q = om.source(s.sources, s.source_mode)
        out.append((s, om, q, n, dt))
    return out


def make(s, dt, **opt):
    h = ff.Handle(s.xyz, s.tets, s.materials, s.T0, s.dir_nodes, s.dir_T, dt=dt,
                  precision=ff.FP32C, **opt)
    h.precompute()
    h.set_gaussian_sources(s.sources, s.source_mode)
    return h


def test_batch_equals_single_and_oracle(scenarios):
    hb = [make(s, dt) for s, _, _, _, dt in scenarios]
    hs = [make(s, dt) for s, _, _, _, dt in scenarios]
    ns = np.array([n for _, _, _, n, _ in scenarios])
    b = ff.Batch(hb)
    b.run(ns)
    print(f"[batch] {len(hb)} scenarios, steps {ns.tolist()}, graph {b.last_ms():.3f} ms",
          flush=True)
    worst = 0.0
    for (s, om, q, n, dt), h1, h2 in zip(scenarios, hb, hs):
        h2.step(n)
        Tb = h1.read_T()
        assert np.array_equal(h1.read_state()[0], h2.read_state()[0]), s.name
        assert h1.time()[1] == n
        T_ref = om.run(om.initial(37.0), n, q)
        err = float(np.max(np.abs(Tb - T_ref)))
        worst = max(worst, err)
        print(f"[parity] batch {s.name}: n={n} tets={s.n_tets} peak={T_ref.max():.2f} "
              f"max|dT|={err:.3e} K", flush=True)
    assert worst <= 1e-3
    # a second run continues from the end state; one scenario stays put
    ns2 = ns // 3
    ns2[2] = 0
    before = hb[2].read_state()[0]
    b.run(ns2)
    for h1, h2, k in zip(hb, hs, ns2):
        h2.step(int(k))
        assert np.array_equal(h1.read_state()[0], h2.read_state()[0])
    assert np.array_equal(hb[2].read_state()[0], before)
    b.close()


def test_batch_of_packed_and_16_bit_corner_ids(scenarios):
    """Scenarios whose tiles exceed 1024 nodes keep 16-bit corner ids; a batch
    mixing them with packed scenarios expands the packed ones and must still
    equal per-handle stepping bit for bit."""
    wide = dict(reorder=False, tile_elems=4096)
    picks = [(scenarios[k], wide if k % 2 else {}) for k in range(4)]
    hb = [make(s, dt, **o) for (s, _, _, _, dt), o in picks]
    hs = [make(s, dt, **o) for (s, _, _, _, dt), o in picks]
    nodes = [h.info()["max_tile_nodes"] for h in hb]
    print(f"[batch] max tile nodes {nodes}", flush=True)
    assert any(m > 1024 for m in nodes) and any(m <= 1024 for m in nodes)
    ns = np.array([n // 2 for (_, _, _, n, _), _ in picks])
    b = ff.Batch(hb)
    b.run(ns)
    for h1, h2, k in zip(hb, hs, ns):
        h2.step(int(k))
        assert np.array_equal(h1.read_state()[0], h2.read_state()[0])
    b.close()
    for h in hb + hs:
        h.close()


def test_batch_rejects_mixed_or_unprepared(scenarios):
    s, _, _, _, dt = scenarios[0]
    h = make(s, dt)
    h64 = ff.Handle(s.xyz, s.tets, s.materials, s.T0, s.dir_nodes, s.dir_T, dt=dt,
                    precision=ff.FP64)
    h64.precompute()
    with pytest.raises(ff.FedFemError) as ei:
        ff.Batch([h, h64])
    assert ei.value.code == ff.E_INVALID
    raw = ff.Handle(s.xyz, s.tets, s.materials, s.T0, s.dir_nodes, s.dir_T, dt=dt)
    with pytest.raises(ff.FedFemError) as ei:
        ff.Batch([h, raw])
    assert ei.value.code == ff.E_NOT_PRECOMPUTED
    with pytest.raises(ff.FedFemError):
        ff.Batch([h, h])


def test_batch_run_refuses_schedule_or_dose_set_after_create(scenarios):
    """A schedule or dose model set on a member after fedfem_batch_create
    would be ignored by the lockstep launches: the run refuses it
    (FEDFEM_E_STATE) and advances no scenario."""
    (s0, _, _, n0, dt0), (s1, _, _, n1, dt1) = scenarios[:2]
    h0, h1 = make(s0, dt0), make(s1, dt1)
    b = ff.Batch([h0, h1])
    for setter, clear in ((lambda h: h.set_schedule(np.ones((1, h.N)), [([0.0], [1.0])]),
                           lambda h: h.set_schedule(None, [])),
                          (lambda h: h.set_dose(ff.DOSE_CEM43),
                           lambda h: h.set_dose(ff.DOSE_OFF))):
        setter(h1)
        with pytest.raises(ff.FedFemError) as ei:
            b.run([n0, n1])
        assert ei.value.code == ff.E_STATE
        assert h0.time()[1] == 0 and h1.time()[1] == 0
        clear(h1)
    b.run([n0, n1])
    assert h0.time()[1] == n0 and h1.time()[1] == n1
    b.close()
    h0.close()
    h1.close()


def test_precompute_many_equals_sequential_and_reports_errors(scenarios):
    """Precompute overlapped on host threads gives every handle exactly what
    its own precompute gives (critical step, then 20 steps bit for bit), and
    a degenerate mesh among them is reported at its own index."""
    seq, par = [], []
    for s, _, _, _, _ in scenarios:
        h = ff.Handle(s.xyz, s.tets, s.materials, s.T0, s.dir_nodes, s.dir_T, dt=-0.9,
                      precision=ff.FP32C)
        h.precompute()
        seq.append(h)
        par.append(ff.Handle(s.xyz, s.tets, s.materials, s.T0, s.dir_nodes, s.dir_T, dt=-0.9,
                             precision=ff.FP32C))
    ff.precompute_many(par, threads=4)
    for (s, _, _, _, _), a, b in zip(scenarios, seq, par):
        assert a.dt() == b.dt()
        for h in (a, b):
            h.set_gaussian_sources(s.sources, s.source_mode)
            h.step(20)
        assert np.array_equal(a.read_state()[0], b.read_state()[0])
    for h in seq + par:
        h.close()
    # a flattened tet in the third scenario
    hs = []
    for k, (s, _, _, _, _) in enumerate(scenarios[:4]):
        xyz = s.xyz.copy()
        if k == 2:
            t = s.tets[11]
            xyz[t[3]] = (xyz[t[0]] + xyz[t[1]] + xyz[t[2]]) / 3.0
        hs.append(ff.Handle(xyz, s.tets, s.materials, s.T0, s.dir_nodes, s.dir_T, dt=-0.9,
                            precision=ff.FP32C))
    with pytest.raises(ff.FedFemError) as ei:
        ff.precompute_many(hs, threads=3)
    assert ei.value.code == ff.E_DEGENERATE
    assert "handle 2:" in str(ei.value)
    for h in hs:
        h.close()


def test_recycled_device_memory_gives_identical_results(scenarios):
    """Handles built on blocks recycled by the library's device cache (left
    dirty by other scenarios) step exactly as on fresh memory."""
    ff.release_cached_memory()

    def run(s):
        h = ff.Handle(s.xyz, s.tets, s.materials, s.T0, s.dir_nodes, s.dir_T, dt=-0.9,
                      precision=ff.FP32C)
        h.precompute()
        h.set_gaussian_sources(s.sources, s.source_mode)
        h.step(30)
        out = (h.dt(), h.read_state()[0])
        h.close()
        return out

    s0 = scenarios[0][0]
    fresh = run(s0)
    for s, _, _, _, _ in scenarios[1:]:
        run(s)  # leaves its blocks, dirty, in the cache
    recycled = run(s0)
    assert fresh[0] == recycled[0]
    assert np.array_equal(fresh[1], recycled[1])
    assert ff.release_cached_memory() > 0
    assert ff.release_cached_memory() == 0


def test_batch_run_with_sources(scenarios):
    """Per-scenario sources given to the batch run replace the handles'
    active sources, as the source argument of fedfem_step does: the batch
    equals each handle stepped alone with the same source; a None entry keeps
    the handle's own; a non-finite source is refused before anything runs."""
    sc3 = scenarios[:3]
    hb = [make(s, dt) for s, _, _, _, dt in sc3]
    hs = [make(s, dt) for s, _, _, _, dt in sc3]
    ns = np.array([40, 25, 60])
    rng = np.random.default_rng(7)
    srcs = [0.5 * q + rng.uniform(0.0, 1e-3, len(q)) for _, _, q, _, _ in sc3]
    srcs[1] = None
    b = ff.Batch(hb)
    before = hb[0].read_source()
    bad = [srcs[0], None, np.full(len(sc3[2][2]), np.nan)]
    with pytest.raises(ff.FedFemError) as ei:
        b.run(ns, bad)
    assert ei.value.code == ff.E_INVALID
    assert all(h.time()[1] == 0 for h in hb)
    assert np.array_equal(hb[0].read_source(), before)   # nothing replaced
    b.run(ns, srcs)
    for h1, h2, n, q in zip(hb, hs, ns, srcs):
        h2.step(int(n), q)
        assert np.array_equal(h1.read_state()[0], h2.read_state()[0])
        if q is not None:
            assert np.max(np.abs(h1.read_source() - q)) <= 1e-6 * np.max(np.abs(q))
    # the sources stay active: a second run without them continues the same way
    b.run(ns)
    for h1, h2, n in zip(hb, hs, ns):
        h2.step(int(n))
        assert np.array_equal(h1.read_state()[0], h2.read_state()[0])
    b.close()
    for h in hb + hs:
        h.close()
