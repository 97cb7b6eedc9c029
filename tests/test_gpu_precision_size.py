"""Every storage against the FP64 oracle at the size of the precision-study subsample (64x64x256
tube, R = 30, hematocrit 0.40, 2,881 cells), over 20 coupled steps from rest: the FP64 path to
round-off growth, FP32 within the velocity target 1e-4 and the wall-shear-stress target 1e-3
(relative L2 over the fluid and the wall-adjacent nodes), BF16 with stochastic rounding within
1e-2 and FP16 (scale 2^21) within 2e-3 in velocity, with their wall shear stress reported
against bounds set from the measured errors."""
import numpy as np
import pytest

from paper_1107_4889_amd import synth

pytestmark = pytest.mark.gpu

NX, NY, NZ, STEPS = 64, 64, 256, 20
CFG = dict(nx=NX, ny=NY, nz=NZ, periodic=(0, 0, 1), tau0=0.8, g_ext=(0.0, 0.0, 1e-6),
           f16_scale=2.0 ** 21)


@pytest.fixture(scope="module")
def subsample():
    from oracle import oracle as orc

    solid, pl = synth.tube_workload(NX, NY, NZ, 30.0, hematocrit=0.40, seed=1107)
    print(f"oracle: {NX}x{NY}x{NZ} tube, {len(pl.R)} cells, {STEPS} steps", flush=True)
    o = orc.Oracle({k: v for k, v in CFG.items() if k != "f16_scale"}, solid, R=pl.R, Q=pl.Q)
    assert o.step(STEPS) == 0
    return solid, pl, dict(u=o.u(), rbc=o.rbc(), wss=o.wall_shear_stress())


# storage: (velocity, wall shear stress, cell position) bounds, relative L2 / absolute lu
BOUNDS = {"f64": (1e-10, 1e-9, 1e-10), "f32": (1e-4, 1e-3, 1e-7),
          "bf16": (1e-2, 5e-2, 1e-6), "f16": (2e-3, 1e-2, 1e-6)}


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16", "f16"])
def test_storage_matches_oracle_at_study_size(subsample, storage):
    from paper_1107_4889_amd import lbrbc

    solid, pl, ref = subsample
    print(f"{storage} against the oracle: {NX}x{NY}x{NZ}, {len(pl.R)} cells, {STEPS} steps", flush=True)
    sim = lbrbc.Simulation({**CFG, "storage": storage}, solid, R=pl.R, Q=pl.Q)
    sim.lb_step(STEPS)
    fl = solid.reshape(-1) == 0
    ug = sim.lb_get_fields(f=False, u=True, sigma=False)["u"][fl]
    uo = ref["u"][fl]
    bu, bw, br = BOUNDS[storage]
    eu = np.linalg.norm(ug - uo) / np.linalg.norm(uo)
    node_g, wss_g = sim.lb_wall_shear_stress(False)
    node_o, wss_o = ref["wss"]
    assert np.array_equal(node_g, node_o)
    ew = np.linalg.norm(wss_g - wss_o) / np.linalg.norm(wss_o)
    er = np.abs(sim.rbc_get_state()[0] - ref["rbc"][0]).max()
    print(f"{storage}: u rel L2 {eu:.3e}, WSS rel L2 {ew:.3e}, max |dR| {er:.3e}", flush=True)
    assert eu <= bu and ew <= bw and er <= br


def test_pipelined_steps_bitwise_equal_to_single_steps():
    """With at least 2,048 cells the cells' own work of the next step runs on a second stream
    beside the stream-collide, within one lb_step call; a call joins it back before it returns.
    Every kernel sees the inputs of the serial order, so one call of 12 steps, 12 calls of one
    step and calls of 5 + 7 steps must give the same state bit for bit."""
    from paper_1107_4889_amd import lbrbc

    solid, pl = synth.tube_workload(64, 64, 256, 30.0, hematocrit=0.40, seed=1107)
    assert len(pl.R) >= 2048
    cfg = dict(nx=64, ny=64, nz=256, periodic=(0, 0, 1), tau0=0.8, g_ext=(0, 0, 1e-6))
    print(f"pipelined vs single steps: {len(pl.R)} cells, f32", flush=True)
    runs = []
    for split in ((12,), (1,) * 12, (5, 7)):
        sim = lbrbc.Simulation(dict(cfg, storage="f32"), solid, R=pl.R, Q=pl.Q)
        for n in split:
            sim.lb_step(n)
        sim.lb_sync()
        d = sim.lb_get_fields(f=True, u=True, sigma=True)
        runs.append((d, sim.rbc_get_state(), sim.rbc_get_coupling()))
        del sim
    (d0, s0, c0) = runs[0]
    for d, s, c in runs[1:]:
        for k in ("f", "u", "sigma"):
            assert np.array_equal(d[k], d0[k]), k
        for a, b in zip(s, s0):
            assert np.array_equal(a, b)
        assert np.array_equal(c, c0)
