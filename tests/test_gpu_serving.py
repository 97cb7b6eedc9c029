"""Serving: a request gives the same result alone and in a mix (bitwise: the kernels are
deterministic and requests share nothing), admission respects the HBM budget, and HIP-graph
replay of the step chunks reproduces eager stepping."""
import numpy as np
import pytest

from paper_1107_4889_amd import synth

pytestmark = pytest.mark.gpu


def _requests(n, seed=77, steps=(60, 140)):
    from paper_1107_4889_amd.serving import Request

    tr = synth.serving_trace(n, rate_hz=1e6, seed=seed, r_range=(8.0, 12.0), k_range=(3.0, 5.0),
                             h_range=(0.1, 0.3), steps_range=steps)
    reqs = []
    for d in tr:
        cfg = dict(nx=d["nx"], ny=d["ny"], nz=d["nz"], periodic=(0, 0, 1), tau0=0.8,
                   g_ext=(0, 0, 1e-5), storage="f32")
        reqs.append(Request(rid=d["rid"], arrival=0.0, cfg=cfg, solid=d["solid"], R=d["R"],
                            Q=d["Q"], steps=d["steps"]))
    return reqs


def test_alone_equals_mix_and_budget():
    from paper_1107_4889_amd.serving import Server

    reqs = _requests(4)
    assert sum(len(r.R) for r in reqs) > 0
    alone = {}
    for r in reqs:
        res, _ = Server(budget_bytes=8 << 30, chunk_steps=16, digests=True).run([r])
        alone[r.rid] = res[0]
    mixed, _ = Server(budget_bytes=8 << 30, chunk_steps=16, digests=True).run(reqs)
    assert [m.rid for m in mixed] == [r.rid for r in reqs]
    for m in mixed:
        a = alone[m.rid]
        assert m.digest == a.digest and m.mass == a.mass and m.flow_rate == a.flow_rate
        assert m.flags == 0
    # a budget that holds one request at a time serialises them (admission by footprint)
    from paper_1107_4889_amd.serving import Server as S
    one = max(S(1 << 40).footprint(r) for r in reqs)
    res, _ = S(budget_bytes=one, chunk_steps=16, digests=True).run(reqs)
    spans = sorted((r.admitted, r.finished) for r in res)
    for (a0, f0), (a1, f1) in zip(spans, spans[1:]):
        assert a1 >= f0 - 1e-9
    assert {r.rid: r.digest for r in res} == {k: v.digest for k, v in alone.items()}


def test_graph_replay_matches_eager():
    from paper_1107_4889_amd.serving import Server

    reqs = _requests(3, seed=78, steps=(64, 64))
    eager, _ = Server(budget_bytes=8 << 30, chunk_steps=16, digests=True).run(reqs)
    graph, _ = Server(budget_bytes=8 << 30, chunk_steps=16, digests=True, use_graphs=True).run(reqs)
    for e, g in zip(eager, graph):
        assert e.digest == g.digest, (e.rid, e.steps)


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_graph_every_replay_matches_eager(storage):
    """Each replay of a captured 16-step chunk leaves the state an eager 16-step chunk does;
    eager work (observables, syncs) runs between the replays. In BF16 the stochastic rounding's
    step term comes from the device counter, which every replay advances."""
    import hashlib

    import torch

    from paper_1107_4889_amd import lbrbc

    r = _requests(1, seed=79, steps=(64, 64))[0]
    cfg = dict(r.cfg, storage=storage)
    s_e, s_g = torch.cuda.Stream(), torch.cuda.Stream()
    eager = lbrbc.Simulation(cfg, r.solid, R=r.R, Q=r.Q, stream=s_e)
    graph = lbrbc.Simulation(cfg, r.solid, R=r.R, Q=r.Q, stream=s_g)
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.stream(s_g):
        with torch.cuda.graph(g, stream=s_g):
            graph.lb_step(16)
    for rep in range(4):
        eager.lb_step(16)
        with torch.cuda.stream(s_g):
            g.replay()
        torch.cuda.synchronize()
        o_e, o_g = eager.lb_observe(), graph.lb_observe()
        assert o_e.flags == 0 and o_g.flags == 0
        d_e = hashlib.sha1(eager.lb_save()[88:]).hexdigest()
        d_g = hashlib.sha1(graph.lb_save()[88:]).hexdigest()
        assert d_e == d_g, rep
        assert o_e.mass == o_g.mass and o_e.flow_rate == o_g.flow_rate


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_fused_batch_16bit_equals_each_alone(storage):
    """The fused stages of the 16-bit storages (u, sigma and the coverage entries in 16 bits,
    BF16 with its step-salted stochastic rounding) give each context the bits it gets alone."""
    import hashlib

    import torch

    from paper_1107_4889_amd import lbrbc

    reqs = _requests(3, seed=81, steps=(30, 30))
    cases = [(dict(r.cfg, storage=storage, f16_scale=2.0 ** 21), r.solid, r.R, r.Q) for r in reqs]
    nsteps = [24, 36, 30]
    print(f"fused {storage}: {len(cases)} contexts", flush=True)

    def digest(sim):
        return hashlib.sha1(sim.lb_save()[88:]).hexdigest()

    alone = []
    for (cfg, solid, R, Q), n in zip(cases, nsteps):
        sim = lbrbc.Simulation(cfg, solid, R=R, Q=Q)
        sim.lb_step(n)
        sim.lb_sync()
        alone.append(digest(sim))
        del sim
    shared = torch.cuda.Stream()
    sims = [lbrbc.Simulation(cfg, solid, R=R, Q=Q, stream=shared) for cfg, solid, R, Q in cases]
    for sim in sims:
        sim.lb_step(4)
    lbrbc.lb_batch_step(sims, [n - 4 for n in nsteps])
    torch.cuda.synchronize()
    for k, (sim, d) in enumerate(zip(sims, alone)):
        assert sim.lb_observe().flags == 0
        assert digest(sim) == d, k


def test_fused_batch_equals_each_alone():
    """lb_batch_step over contexts on one stream runs each stage as one launch for all of them
    (fused); each context ends bitwise where it ends when stepped alone. The mix has different
    step counts, a context without cells and one large enough to fork onto a side stream when
    stepped alone."""
    import hashlib

    import torch

    from paper_1107_4889_amd import lbrbc

    reqs = _requests(2, seed=80, steps=(40, 40))
    big_solid, big = synth.tube_workload(64, 64, 256, 30.0, hematocrit=0.40, seed=1107)
    bigcfg = dict(nx=64, ny=64, nz=256, periodic=(0, 0, 1), tau0=0.8, g_ext=(0, 0, 1e-6),
                  storage="f32")
    cases = [(r.cfg, r.solid, r.R, r.Q) for r in reqs]
    cases.append((reqs[0].cfg, reqs[0].solid, None, None))          # plasma only
    cases.append((bigcfg, big_solid, big.R, big.Q))                    # >= 2048 cells
    nsteps = [30, 50, 40, 20]

    def digest(sim):
        return hashlib.sha1(sim.lb_save()[88:]).hexdigest()

    alone = []
    for (cfg, solid, R, Q), n in zip(cases, nsteps):
        sim = lbrbc.Simulation(cfg, solid, R=R, Q=Q)
        sim.lb_step(n)
        sim.lb_sync()
        alone.append(digest(sim))
        del sim
    shared = torch.cuda.Stream()
    sims = [lbrbc.Simulation(cfg, solid, R=R, Q=Q, stream=shared) for cfg, solid, R, Q in cases]
    # a few single-context steps first (they leave coverage counts for the fused step to clear)
    for sim in sims:
        sim.lb_step(5)
    lbrbc.lb_batch_step(sims, [n - 5 for n in nsteps])
    torch.cuda.synchronize()
    for k, (sim, d) in enumerate(zip(sims, alone)):
        assert sim.lb_observe().flags == 0
        assert digest(sim) == d, k


def test_fused_server_matches_alone():
    from paper_1107_4889_amd.serving import Server

    reqs = _requests(4, seed=81)
    alone = {}
    for r in reqs:
        res, _ = Server(budget_bytes=8 << 30, chunk_steps=16, digests=True).run([r])
        alone[r.rid] = res[0].digest
    mixed, _ = Server(budget_bytes=8 << 30, chunk_steps=16, digests=True, fused=True).run(reqs)
    for m in mixed:
        assert m.digest == alone[m.rid] and m.flags == 0


def test_interleaved_batch_with_open_boundaries_equals_each_alone():
    """A context with open z faces cannot join a fused launch, so lb_batch_step interleaves the
    contexts step by step on their own streams instead; each still ends bitwise where it ends
    when stepped alone, also when the contexts share one stream."""
    import hashlib

    import torch

    from paper_1107_4889_amd import lbrbc

    reqs = _requests(1, seed=81, steps=(30, 30))
    solid = synth.tube(24, 24, 40, 10.0)
    Q = synth.random_rotations(np.random.default_rng(17), 3).reshape(3, 9)
    R = np.array([[11.5, 11.5, 2.0], [11.5, 11.5, 37.2], [11.0, 12.0, 20.0]])
    open_cfg = dict(nx=24, ny=24, nz=40, periodic=(0, 0, 0), tau0=0.8, open_z=1, rho_in=1.002,
                    rho_out=0.998, storage="f32")
    cases = [(open_cfg, solid, R, Q), (reqs[0].cfg, reqs[0].solid, reqs[0].R, reqs[0].Q)]
    nsteps = [25, 35]
    print("interleaved batch: open-boundary tube with 3 cells beside a periodic request",
          flush=True)

    def digest(sim):
        return hashlib.sha1(sim.lb_save()[88:]).hexdigest()

    alone = []
    for (cfg, sd, Rc, Qc), n in zip(cases, nsteps):
        sim = lbrbc.Simulation(cfg, sd, R=Rc, Q=Qc)
        sim.lb_step(n)
        sim.lb_sync()
        alone.append(digest(sim))
        del sim
    for shared in (False, True):
        one = torch.cuda.Stream()
        sims = [lbrbc.Simulation(cfg, sd, R=Rc, Q=Qc, stream=one if shared else torch.cuda.Stream())
                for cfg, sd, Rc, Qc in cases]
        lbrbc.lb_batch_step(sims, nsteps)
        torch.cuda.synchronize()
        for k, (sim, d) in enumerate(zip(sims, alone)):
            assert sim.lb_observe().flags == 0
            assert digest(sim) == d, (shared, k)
        del sims


def test_served_request_matches_oracle_f64():
    """A request served in the fused mode beside two others, in FP64, ends where the oracle
    ends after the same number of steps: velocity and cells to 1e-10 relative."""
    from oracle import oracle as orc
    from paper_1107_4889_amd.serving import Request, Server

    reqs = _requests(3, seed=82, steps=(40, 60))
    reqs = [Request(**{**r.__dict__, "cfg": dict(r.cfg, storage="f64")}) for r in reqs]
    target = max(reqs, key=lambda r: len(r.R))
    print(f"served request {target.rid}: {target.cfg['nx']}x{target.cfg['ny']}x{target.cfg['nz']}, "
          f"{len(target.R)} cells, {target.steps} steps, FP64", flush=True)
    res, _ = Server(budget_bytes=8 << 30, chunk_steps=16, fused=True, keep_state=True).run(reqs)
    got = {r.rid: r for r in res}[target.rid]
    assert got.flags == 0 and got.steps == target.steps
    ocfg = {k: v for k, v in target.cfg.items() if k != "storage"}
    ref = orc.Oracle(ocfg, target.solid, R=target.R, Q=target.Q)
    assert ref.step(target.steps) == 0
    fl = target.solid.reshape(-1) == 0
    ur = ref.u()[fl]
    assert np.linalg.norm(got.state["u"][fl] - ur) <= 1e-10 * np.linalg.norm(ur)
    Rg, Qg, Vg, Og = got.state["cells"]
    Rr, Qr, Vr, Or = ref.rbc()
    assert np.abs(Rg - Rr).max() < 1e-10 and np.abs(Qg - Qr).max() < 1e-10
    assert np.linalg.norm(Vg - Vr) <= 1e-9 * np.linalg.norm(Vr)


def test_batch_graph_every_replay_matches_eager_fused():
    """lb_batch_capture records 8 fused steps of three contexts on one stream; each of four
    replays, with eager work (observables, a coupling probe that leaves coverage counts set)
    between them, leaves every context bitwise where eager fused batches of 8 steps leave a
    twin, and advances the step counters."""
    import hashlib

    import torch

    from paper_1107_4889_amd import lbrbc

    reqs = _requests(3, seed=83, steps=(64, 64))
    s_g, s_e = torch.cuda.Stream(), torch.cuda.Stream()
    graph_sims = [lbrbc.Simulation(r.cfg, r.solid, R=r.R, Q=r.Q, stream=s_g) for r in reqs]
    eager_sims = [lbrbc.Simulation(r.cfg, r.solid, R=r.R, Q=r.Q, stream=s_e) for r in reqs]
    torch.cuda.synchronize()
    g = lbrbc.BatchGraph(graph_sims, 8)
    assert all(s.lb_observe().step == 0 for s in graph_sims)     # capturing runs nothing

    def digest(sim):
        return hashlib.sha1(sim.lb_save()[88:]).hexdigest()

    for rep in range(4):
        print(f"batch graph replay {rep}", flush=True)
        g.launch()
        lbrbc.lb_batch_step(eager_sims, [8, 8, 8])
        torch.cuda.synchronize()
        for a, b in zip(graph_sims, eager_sims):
            o = a.lb_observe()
            assert o.flags == 0 and o.step == 8 * (rep + 1)
            assert digest(a) == digest(b), rep
        # eager work between replays: a coupling probe leaves the coverage counts set
        graph_sims[rep % 3].rbc_couple()
        eager_sims[rep % 3].rbc_couple()
    del g


def test_fused_server_with_graphs_matches_alone():
    from paper_1107_4889_amd.serving import Server

    reqs = _requests(4, seed=84, steps=(48, 96))
    alone = {}
    for r in reqs:
        res, _ = Server(budget_bytes=8 << 30, chunk_steps=16, digests=True).run([r])
        alone[r.rid] = res[0].digest
    srv = Server(budget_bytes=8 << 30, chunk_steps=16, digests=True, fused=True, use_graphs=True)
    mixed, _ = srv.run(reqs)
    assert srv.graph_launches > 0 and srv.captures > 0
    for m in mixed:
        assert m.digest == alone[m.rid] and m.flags == 0
