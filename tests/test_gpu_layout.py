"""The compact storage layout (only the 64-node row segments that hold fluid are stored, with a
table of the 27 neighbouring segments per stored segment) against the oracle and against the
dense layout. The geometries have rows of several segments ending in a ragged one, periodic
axes that wrap the segment neighbours, cells across the periodic face, open planes, the
overflow (full-tile) map pass, fused batches and checkpoints. Both layouts run the same
per-node arithmetic in the same order, so their fields and cells agree bit for bit."""
import hashlib

import numpy as np
import pytest

from oracle import oracle as orc
from paper_1107_4889_amd import synth

pytestmark = pytest.mark.gpu


def x_tube(nx, ny, nz, r):
    """A tube along x (the axis the segments run along) of radius r in a ny x nz cross-section."""
    z, y = np.meshgrid(np.arange(nz), np.arange(ny), indexing="ij")
    d2 = (y - (ny - 1) / 2.0) ** 2 + (z - (nz - 1) / 2.0) ** 2
    return np.broadcast_to((d2 >= r * r)[:, :, None], (nz, ny, nx)).astype(np.uint8).copy()


def x_tube_case(n_cells=10):
    nx, ny, nz = 150, 22, 22           # segments x0 = 0, 64, 128 (22 nodes: ragged)
    solid = x_tube(nx, ny, nz, 8.5)
    pl = synth.place_cells(solid, synth.AXES, n_cells, seed=21, periodic=(1, 0, 0))
    R = pl.R.copy()
    # a periodic translation along x puts the first cell across the x = 0 face
    R[:, 0] = (R[:, 0] - R[0, 0] + 0.5) % nx
    cfg = dict(nx=nx, ny=ny, nz=nz, periodic=(1, 0, 0), tau0=0.8, g_ext=(2e-6, 0.0, 0.0))
    return cfg, solid, R, pl.Q


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def state(sim):
    d = sim.lb_get_fields(f=True, u=True, sigma=True)
    return d, sim.rbc_get_state(), sim.rbc_get_coupling()


def test_auto_choice_and_footprint():
    from paper_1107_4889_amd import lbrbc

    cfg, solid, R, Q = x_tube_case()
    sims = {lay: lbrbc.Simulation(dict(cfg, storage="f32", layout=lay), solid, R=R, Q=Q) for lay in (0, 1, 2)}
    o = {lay: s.lb_observe() for lay, s in sims.items()}
    rows = (solid == 0).any(-1)
    assert o[0].compact == 1 and o[2].compact == 1 and o[1].compact == 0
    # three column segments per row, stored for the rows that hold fluid
    assert o[2].n_stored == 64 * 3 * int(rows.sum())
    assert o[1].n_stored == solid.size
    for v in o.values():
        assert v.n_fluid == int((solid == 0).sum())


@pytest.mark.parametrize("storage,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_compact_x_tube_matches_oracle(storage, tol):
    from paper_1107_4889_amd import lbrbc

    cfg, solid, R, Q = x_tube_case()
    print(f"x-tube 150x22x22, {len(R)} cells, {storage}: oracle 40 steps", flush=True)
    ref = orc.Oracle(cfg, solid, R=R, Q=Q)
    assert ref.step(40) == 0
    fl = solid.reshape(-1) == 0
    sim = lbrbc.Simulation(dict(cfg, storage=storage, layout=2), solid, R=R, Q=Q)
    sim.lb_step(40)
    d = sim.lb_get_fields()
    ur = ref.u()[fl]
    assert np.linalg.norm(d["u"][fl] - ur) <= tol * np.linalg.norm(ur)
    if storage == "f64":
        assert rel(d["f"][:, fl], ref.f()[:, fl]) < tol
    Rg, Qg, Vg, Og = sim.rbc_get_state()
    Rr, Qr, Vr, Or = ref.rbc()
    assert np.abs(Rg - Rr).max() < tol and np.abs(Qg - Qr).max() < tol
    assert np.linalg.norm(Vg - Vr) <= 10 * tol * np.linalg.norm(Vr)
    assert sim.lb_observe().flags == 0


# BF16 with round-to-nearest: its stochastic rounding draws its bits from the storage index,
# which differs between the layouts (both roundings are exact in expectation)
@pytest.mark.parametrize("storage,extra", [("f64", {}), ("f32", {}), ("bf16", {"bf16_nearest": 1}),
                                           ("f16", {"f16_scale": 2.0 ** 21})])
def test_compact_equals_dense_bitwise(storage, extra):
    from paper_1107_4889_amd import lbrbc

    cfg, solid, R, Q = x_tube_case()
    print(f"x-tube dense vs compact, {storage}", flush=True)
    out = {}
    for lay in (1, 2):
        sim = lbrbc.Simulation(dict(cfg, storage=storage, layout=lay, **extra), solid, R=R, Q=Q)
        sim.lb_step(30)
        out[lay] = state(sim)
        sim.rbc_couple()
        moff, mids = sim.rbc_get_map()
        out[lay] += (moff, mids)
        del sim
    (da, sa, ca, oa, ia), (db, sb, cb, ob, ib) = out[1], out[2]
    for k in ("f", "u", "sigma"):
        assert np.array_equal(da[k], db[k]), k
    for x, y in zip(sa, sb):
        assert np.array_equal(x, y)
    assert np.array_equal(ca, cb)
    assert np.array_equal(oa, ob) and np.array_equal(ia, ib) and len(ia) > 0


def test_compact_overflow_tile_pass_matches_oracle():
    """The smallest candidate capacity sends most cells through the full-tile map pass, which
    looks nodes up through the segment map as well."""
    from paper_1107_4889_amd import lbrbc

    cfg, solid, R, Q = x_tube_case()
    ref = orc.Oracle(cfg, solid, R=R, Q=Q)
    assert ref.step(20) == 0
    sim = lbrbc.Simulation(dict(cfg, storage="f64", layout=2, cand_cap=1), solid, R=R, Q=Q)
    sim.lb_step(20)
    fl = solid.reshape(-1) == 0
    assert rel(sim.lb_get_fields(f=False, sigma=False)["u"][fl], ref.u()[fl]) < 1e-10
    assert np.abs(sim.rbc_get_state()[0] - ref.rbc()[0]).max() < 1e-10


def test_compact_bifurcation_open_planes_wss_and_checkpoint():
    """A Y-bifurcation wider than one segment, with open z faces: the compact layout against
    the dense one (fields, cells, wall-shear-stress nodes), and a checkpoint round trip."""
    from paper_1107_4889_amd import lbrbc

    nx, ny, nz = 96, 40, 64
    solid = synth.y_bifurcation(nx, ny, nz, r_parent=10.0, r_daughter=8.0, z_branch=36.0,
                                angle_deg=35.0)
    pl = synth.place_cells(solid[16:nz - 16], synth.AXES, 12, seed=5, periodic=(0, 0, 0))
    R = pl.R + np.array([0.0, 0.0, 16.0])
    cfg = dict(nx=nx, ny=ny, nz=nz, periodic=(0, 0, 0), tau0=0.8, open_z=1, rho_in=1.002,
               rho_out=0.998, storage="f32")
    sims = {lay: lbrbc.Simulation(dict(cfg, layout=lay), solid, R=R, Q=pl.Q) for lay in (1, 2)}
    assert sims[2].lb_observe().compact == 1
    for s in sims.values():
        s.lb_step(25)
    da, db = sims[1].lb_get_fields(), sims[2].lb_get_fields()
    for k in ("f", "u", "sigma"):
        assert np.array_equal(da[k], db[k]), k
    assert np.array_equal(sims[1].rbc_get_state()[0], sims[2].rbc_get_state()[0])
    na, wa = sims[1].lb_wall_shear_stress()
    nb, wb = sims[2].lb_wall_shear_stress()
    assert np.array_equal(na, nb) and np.array_equal(wa, wb)
    # checkpoint round trip in the compact layout; a dense context refuses it
    sim = sims[2]
    ck = sim.lb_save()
    sim.lb_step(10)
    d1 = hashlib.sha1(sim.lb_save()[88:]).hexdigest()
    sim.lb_load(ck)
    sim.lb_step(10)
    assert hashlib.sha1(sim.lb_save()[88:]).hexdigest() == d1
    with pytest.raises(lbrbc.LbError):
        sims[1].lb_load(ck)


def test_fused_batch_mixed_layouts_equals_each_alone():
    """lb_batch_step fuses contexts of either layout into one launch per stage; each ends
    bitwise where it ends alone. Also through a captured batch graph."""
    import torch

    from paper_1107_4889_amd import lbrbc

    cfg, solid, R, Q = x_tube_case()
    cases = [(dict(cfg, storage="f32", layout=2), solid, R, Q),
             (dict(cfg, storage="f32", layout=1), solid, R, Q),
             (dict(cfg, storage="f32", layout=2), solid, None, None)]

    def digest(sim):
        return hashlib.sha1(sim.lb_save()[88:]).hexdigest()

    alone = []
    for c, s, r, q in cases:
        sim = lbrbc.Simulation(c, s, R=r, Q=q)
        sim.lb_step(16)
        alone.append(digest(sim))
        del sim
    stream = torch.cuda.Stream()
    sims = [lbrbc.Simulation(c, s, R=r, Q=q, stream=stream) for c, s, r, q in cases]
    lbrbc.lb_batch_step(sims, [8, 8, 8])
    g = lbrbc.BatchGraph(sims, 8)
    g.launch()
    torch.cuda.synchronize()
    for k, (sim, d) in enumerate(zip(sims, alone)):
        assert sim.lb_observe().flags == 0
        assert digest(sim) == d, k
    del g


def test_compact_equals_dense_with_moving_walls():
    """The shear cell (moving walls, whose bounce-back term depends on the node's row) stored in
    the compact layout gives the dense layout's bits."""
    import bench
    from paper_1107_4889_amd import lbrbc

    cfg, solid, R, Q = bench.shear_cell_config(0.063, storage="f32", n=(80, 34, 24))
    out = []
    for lay in (1, 2):
        sim = lbrbc.Simulation(dict(cfg, layout=lay), solid, R=R, Q=Q)
        sim.lb_step(200)
        out.append((sim.lb_get_fields(f=True, u=True, sigma=True), sim.rbc_get_state()))
        del sim
    (da, sa), (db, sb) = out
    for k in ("f", "u", "sigma"):
        assert np.array_equal(da[k], db[k]), k
    for x, y in zip(sa, sb):
        assert np.array_equal(x, y)
    assert np.abs(da["u"][:, 0]).max() > 0
