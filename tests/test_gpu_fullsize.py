"""Parity at the benchmark's full size (128x128x512 tube, R = 60, 19,241 cells): the FP64 path
against the oracle over one coupled step (fields, cells, the node->cell map bit for bit), and
the FP32 configuration the benchmark times checked by properties that hold at any size; the
256x256x1024 study tube by the same properties in the reduced storages."""
import numpy as np
import pytest

from paper_1107_4889_amd import synth

pytestmark = pytest.mark.gpu

NX, NY, NZ, R = 128, 128, 512, 60.0


@pytest.fixture(scope="module")
def tube():
    solid, pl = synth.tube_workload(NX, NY, NZ, R, hematocrit=0.35, seed=1107)
    return solid, pl


def _cfg(**kw):
    d = dict(nx=NX, ny=NY, nz=NZ, periodic=(0, 0, 1), tau0=0.8, g_ext=(0.0, 0.0, 1e-6))
    d.update(kw)
    return d


def test_fullsize_fp64_step_matches_oracle(tube):
    from oracle import oracle as orc
    from paper_1107_4889_amd import lbrbc

    solid, pl = tube
    print(f"full-size parity: {NX}x{NY}x{NZ}, {len(pl.R)} cells", flush=True)
    sim = lbrbc.Simulation(_cfg(storage="f64"), solid, R=pl.R, Q=pl.Q)
    sim.lb_step(1)
    d = sim.lb_get_fields(f=False, u=True, sigma=True)
    Rg, Qg, Vg, Og = sim.rbc_get_state()
    sim.rbc_couple()                     # the map of the state after the step
    moff, mids = sim.rbc_get_map()
    # the 15x15x61 cell grid spans 14 scan chunks of 1024: the multi-block offsets scan
    ncell, coff, cids = sim.rbc_get_cells()
    assert int(np.prod(ncell)) > 2 * 1024
    del sim
    ref = orc.Oracle(_cfg(), solid, R=pl.R, Q=pl.Q)
    assert ref.step(1) == 0
    fl = solid.reshape(-1) == 0
    ur = ref.u()[fl]
    assert np.linalg.norm(d["u"][fl] - ur) <= 1e-10 * np.linalg.norm(ur)
    # sigma after one step is round-off (~1e-17) almost everywhere and ~1e-7 only where the
    # cells push: element-wise bound with an absolute floor far above the round-off
    sr = ref.sigma()[fl]
    assert np.all(np.abs(d["sigma"][fl] - sr) <= 1e-9 * np.abs(sr) + 1e-15)
    Rr, Qr, Vr, Or = ref.rbc()
    assert np.abs(Rg - Rr).max() < 1e-12 and np.abs(Qg - Qr).max() < 1e-12
    assert np.linalg.norm(Vg - Vr) <= 1e-9 * np.linalg.norm(Vr)
    ref.couple()
    roff, rids = ref.node_map()
    assert np.array_equal(moff, roff) and np.array_equal(mids, rids)
    rcoff, rcids = ref.cells()
    assert np.array_equal(coff, rcoff) and np.array_equal(cids, rcids)


def test_fullsize_fp32_bench_config_properties(tube):
    """The configuration bench.py times: mass conserved to FP32 round-off over 200 steps, no
    device fault, cells inside the tube, a positive flow rate along the drive."""
    from paper_1107_4889_amd import lbrbc

    solid, pl = tube
    sim = lbrbc.Simulation(_cfg(storage="f32"), solid, R=pl.R, Q=pl.Q)
    m0 = sim.lb_observe().mass
    sim.lb_step(200)
    o = sim.lb_observe()
    assert o.flags == 0
    assert abs(o.mass - m0) <= 1e-6 * m0
    assert o.flow_rate > 0 and np.isfinite(o.eta_app) and o.eta_app > 0
    Rc = sim.rbc_get_state()[0]
    r = np.hypot(Rc[:, 0] - (NX - 1) / 2, Rc[:, 1] - (NY - 1) / 2)
    assert r.max() < R
    node, wss = sim.lb_wall_shear_stress(False)
    assert len(node) > 0 and np.all(np.isfinite(wss)) and wss.mean() > 0


def test_study_tube_256_properties_in_each_storage():
    """The largest configuration, the 256x256x1024 study tube (R = 120, 80,451 cells by random
    sequential addition), in the three reduced storages over 100 steps: no device fault, mass
    conserved to the storage's round-off, cells inside the tube, a positive flow rate and
    finite wall shear stress."""
    from paper_1107_4889_amd import lbrbc

    nx, ny, nz, Rt = 256, 256, 1024, 120.0
    solid, pl = synth.tube_workload(nx, ny, nz, Rt, hematocrit=0.40, seed=1107, fill=False)
    cfg = dict(nx=nx, ny=ny, nz=nz, periodic=(0, 0, 1), tau0=0.8, g_ext=(0.0, 0.0, 1e-6),
               f16_scale=2.0 ** 21)
    for storage, tol in (("f32", 1e-6), ("bf16", 1e-4), ("f16", 1e-4)):
        print(f"study tube {nx}x{ny}x{nz}, {len(pl.R)} cells, {storage}, 100 steps", flush=True)
        sim = lbrbc.Simulation(dict(cfg, storage=storage), solid, R=pl.R, Q=pl.Q)
        m0 = sim.lb_observe().mass
        sim.lb_step(100)
        o = sim.lb_observe()
        assert o.flags == 0, storage
        assert abs(o.mass - m0) <= tol * m0, (storage, o.mass, m0)
        assert o.flow_rate > 0, storage
        Rc = sim.rbc_get_state()[0]
        r = np.hypot(Rc[:, 0] - (nx - 1) / 2, Rc[:, 1] - (ny - 1) / 2)
        assert r.max() < Rt, storage
        node, wss = sim.lb_wall_shear_stress(False)
        assert len(node) > 0 and np.all(np.isfinite(wss)), storage
        del sim
