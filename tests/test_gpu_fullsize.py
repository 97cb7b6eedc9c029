"""Parity at full size: the 128x128x512 tube (R = 60, 20,150 cells, H = 0.35), FP64 against the
oracle over one coupled step (fields, cells, the node->cell map bit for bit) and FP32 element
by element over three steps, plus properties that hold at any size over 200 FP32 steps; the
256x256x1024 study tube (R = 120, H = 0.40), which the benchmark times, by the same properties in
every storage and against the oracle at sampled cells."""
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


@pytest.fixture(scope="module")
def oracle_runs(tube):
    """The oracle on the full-size tube: the state after 1 step (with the coverage map and cell
    list of that state) and after 3 steps (fields, wall shear stress, coupling, cells)."""
    from oracle import oracle as orc

    solid, pl = tube
    print(f"oracle: {NX}x{NY}x{NZ} tube, {len(pl.R)} cells, 3 steps", flush=True)
    ref = orc.Oracle(_cfg(), solid, R=pl.R, Q=pl.Q)
    assert ref.step(1) == 0
    one = dict(u=ref.u(), sigma=ref.sigma(), rbc=ref.rbc())
    ref.couple()                         # coverage of the state after one step (no time advance)
    one["map"] = ref.node_map()
    one["cells"] = ref.cells()
    assert ref.step(2) == 0
    three = dict(u=ref.u(), sigma=ref.sigma(), rbc=ref.rbc(), wss=ref.wall_shear_stress(),
                 coupling=ref.coupling())
    return one, three


def test_fullsize_fp64_step_matches_oracle(tube, oracle_runs):
    from paper_1107_4889_amd import lbrbc

    solid, pl = tube
    one, _ = oracle_runs
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
    fl = solid.reshape(-1) == 0
    ur = one["u"][fl]
    assert np.linalg.norm(d["u"][fl] - ur) <= 1e-10 * np.linalg.norm(ur)
    # sigma after one step is round-off (~1e-17) almost everywhere and ~1e-7 only where the
    # cells push: element-wise bound with an absolute floor far above the round-off
    sr = one["sigma"][fl]
    assert np.all(np.abs(d["sigma"][fl] - sr) <= 1e-9 * np.abs(sr) + 1e-15)
    Rr, Qr, Vr, Or = one["rbc"]
    assert np.abs(Rg - Rr).max() < 1e-12 and np.abs(Qg - Qr).max() < 1e-12
    assert np.linalg.norm(Vg - Vr) <= 1e-9 * np.linalg.norm(Vr)
    roff, rids = one["map"]
    assert np.array_equal(moff, roff) and np.array_equal(mids, rids)
    rcoff, rcids = one["cells"]
    assert np.array_equal(coff, rcoff) and np.array_equal(cids, rcids)


def test_fullsize_fp32_three_steps_match_oracle(tube, oracle_runs):
    """The FP32 configuration the benchmark's tube runs, element by element against the FP64
    oracle after three coupled steps, at the FP32 tolerances: velocity within 1e-4 of the
    largest |u|, stress and per-node wall shear stress within 1e-3 of their largest values,
    hydrodynamic force and torque within 1e-4 of their largest, and cell positions and
    orientations to 1e-9 (they move by ~1e-6 in three steps)."""
    from paper_1107_4889_amd import lbrbc

    solid, pl = tube
    _, three = oracle_runs
    print(f"full-size FP32 parity: {NX}x{NY}x{NZ}, {len(pl.R)} cells, 3 steps", flush=True)
    sim = lbrbc.Simulation(_cfg(storage="f32"), solid, R=pl.R, Q=pl.Q)
    sim.lb_step(3)
    d = sim.lb_get_fields(f=False, u=True, sigma=True)
    node, wss = sim.lb_wall_shear_stress(False)
    cp = sim.rbc_get_coupling()
    Rg, Qg, Vg, Og = sim.rbc_get_state()
    del sim
    fl = solid.reshape(-1) == 0

    def max_rel(a, b):
        return float(np.abs(a - b).max() / np.abs(b).max())

    assert max_rel(d["u"][fl], three["u"][fl]) <= 1e-4
    assert max_rel(d["sigma"][fl], three["sigma"][fl]) <= 1e-3
    node_r, wss_r = three["wss"]
    assert np.array_equal(node, node_r)
    assert max_rel(wss, wss_r) <= 1e-3
    rcp = three["coupling"]
    assert max_rel(cp[:, 10:13], rcp[:, 10:13]) <= 1e-4          # F^hyd
    assert max_rel(cp[:, 13:16], rcp[:, 13:16]) <= 1e-4          # T^hyd
    Rr, Qr, Vr, Or = three["rbc"]
    assert np.abs(Rg - Rr).max() < 1e-9 and np.abs(Qg - Qr).max() < 1e-9
    assert max_rel(Vg, Vr) <= 1e-4


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
    solid, pl = synth.tube_workload(nx, ny, nz, Rt, hematocrit=0.40, seed=1107)
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


def _wall_points_d3q19(solid):
    """Solid nodes with a fluid D3Q19 neighbour (z periodic), as (m, 3) xyz: the wall mesh
    points of the cell-wall Gay-Berne forces."""
    s = solid.astype(bool)
    near = np.zeros_like(s)
    for dx, dy, dz in [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)
                       if 0 < a * a + b * b + c * c <= 2]:
        sh = np.roll(~s, (dz, dy, dx), axis=(0, 1, 2))
        if dx:
            sh[:, :, 0 if dx > 0 else -1] = False
        if dy:
            sh[:, 0 if dy > 0 else -1, :] = False
        near |= sh
    z, y, x = np.nonzero(s & near)
    return np.stack([x, y, z], 1).astype(np.float64)


def test_study_tube_256_gay_berne_at_sampled_cells():
    """The 256x256x1024 study tube at its full size and cell count: the Gay-Berne force and
    torque (cell-cell and cell-wall) of 64 sampled cells against the oracle's pair function
    summed over every partner within the cut-off, found independently by a KD-tree."""
    from scipy.spatial import cKDTree

    from oracle import oracle as orc
    from paper_1107_4889_amd import lbrbc

    nx, ny, nz, Rt = 256, 256, 1024, 120.0
    solid, pl = synth.tube_workload(nx, ny, nz, Rt, hematocrit=0.40, seed=1107)
    cfg = dict(nx=nx, ny=ny, nz=nz, periodic=(0, 0, 1), tau0=0.8, g_ext=(0.0, 0.0, 1e-6))
    print(f"study tube {nx}x{ny}x{nz}, {len(pl.R)} cells: Gay-Berne at 64 sampled cells", flush=True)
    sim = lbrbc.Simulation(dict(cfg, storage="f32"), solid, R=pl.R, Q=pl.Q)
    F, T = sim.rbc_collide()
    del sim
    rng = np.random.default_rng(11)
    R, Q = pl.R, pl.Q.reshape(-1, 3, 3)
    wall = _wall_points_d3q19(solid)
    # the sample: 32 cells anywhere and the 32 cells nearest the wall
    rr = np.hypot(R[:, 0] - (nx - 1) / 2, R[:, 1] - (ny - 1) / 2)
    idx = np.unique(np.concatenate([rng.choice(len(R), 32, replace=False), np.argsort(-rr)[:32]]))
    box = np.array([4.0 * nx, 4.0 * ny, float(nz)])
    wrap = lambda P: np.stack([P[:, 0] + nx, P[:, 1] + ny, P[:, 2] % nz], 1)  # noqa: E731
    ct = cKDTree(wrap(R), boxsize=box)
    wt = cKDTree(wrap(wall), boxsize=box)
    amax, amin = 4.0, 1.5
    rc_pair = 2 * amax + (2 ** (1 / 6) - 1) * 2 * amin
    rc_wall = np.sqrt(2 * (amax ** 2 + 0.25)) + (2 ** (1 / 6) - 1) * 0.5
    for i in idx:
        Fi, Ti = np.zeros(3), np.zeros(3)
        for j in sorted(ct.query_ball_point(wrap(R[i:i + 1])[0], rc_pair + 1e-9)):
            if j == i:
                continue
            Rj = R[j].copy()
            Rj[2] += nz * np.round((R[i, 2] - Rj[2]) / nz)           # minimum image along z
            st, _, f, ti, _ = orc.gb_pair(cfg, R[i], Q[i].ravel(), Rj, Q[j].ravel())
            assert st == 0
            Fi += f
            Ti += ti
        for k in sorted(wt.query_ball_point(wrap(R[i:i + 1])[0], rc_wall + 1e-9)):
            Wk = wall[k].copy()
            Wk[2] += nz * np.round((R[i, 2] - Wk[2]) / nz)
            st, _, f, ti, _ = orc.gb_pair(cfg, R[i], Q[i].ravel(), Wk, np.eye(3).ravel(), wall=True)
            assert st == 0
            Fi += f
            Ti += ti
        scale = max(np.abs(Fi).max(), 1e-12)
        assert np.abs(F[i] - Fi).max() <= 1e-9 * scale + 1e-15, (i, F[i], Fi)
        Tb = Q[i].T @ Ti
        assert np.abs(T[i] - Tb).max() <= 1e-9 * max(np.abs(Tb).max(), 1e-12) + 1e-15, (i, T[i], Tb)
