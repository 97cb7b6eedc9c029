"""GPU parity of the open-boundary (pressure-driven) path against the FP64 oracle: a straight
tube and a small Y-bifurcation with inlet z = 0 and outlet z = nz - 1 (non-equilibrium
extrapolation at prescribed densities)."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_1107_4889_amd import synth

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def test_pressure_driven_tube_f64():
    from paper_1107_4889_amd import lbrbc

    nx, ny, nz = 24, 24, 40
    solid = synth.tube(nx, ny, nz, 10.0)
    cfg = dict(nx=nx, ny=ny, nz=nz, periodic=(0, 0, 0), tau0=0.9, open_z=1, rho_in=1.001,
               rho_out=0.999)
    ref = orc.Oracle(cfg, solid)
    assert ref.step(120) == 0
    sim = lbrbc.Simulation(dict(cfg, storage="f64"), solid)
    sim.lb_step(120)
    fl = solid.reshape(-1) == 0
    d = sim.lb_get_fields()
    assert rel(d["u"][fl], ref.u()[fl]) < 1e-11
    assert rel(d["f"][:, fl], ref.f()[:, fl]) < 1e-11
    uz = d["u"][fl][:, 2]
    assert uz.mean() > 0          # flow from the high-density inlet to the outlet


def test_bifurcation_with_cells_f64_and_f32():
    from paper_1107_4889_amd import lbrbc

    nx, ny, nz = 48, 40, 64
    solid = synth.y_bifurcation(nx, ny, nz, r_parent=10.0, r_daughter=8.0, z_branch=36.0)
    # 46% of the 64-node row segments hold fluid: the automatic choice stores the lattice in
    # the compact layout (the tube tests take the dense one)
    segs = np.zeros((nz, ny, 64), dtype=bool)
    segs[:, :, :nx] = solid == 0
    assert segs.any(-1).mean() < 0.6
    # cells away from the open planes (16 lu margin), no periodic axis
    pl = synth.place_cells(solid[16:nz - 16], synth.AXES, 12, seed=5, periodic=(0, 0, 0))
    R = pl.R + np.array([0.0, 0.0, 16.0])
    cfg = dict(nx=nx, ny=ny, nz=nz, periodic=(0, 0, 0), tau0=0.8, open_z=1, rho_in=1.002,
               rho_out=0.998)
    ref = orc.Oracle(cfg, solid, R=R, Q=pl.Q)
    assert ref.step(40) == 0
    fl = solid.reshape(-1) == 0
    sim = lbrbc.Simulation(dict(cfg, storage="f64"), solid, R=R, Q=pl.Q)
    assert sim.lb_observe().compact == 1
    sim.lb_step(40)
    d = sim.lb_get_fields()
    assert rel(d["u"][fl], ref.u()[fl]) < 1e-10
    Rg, Qg, Vg, Og = sim.rbc_get_state()
    Rr, Qr, Vr, Or = ref.rbc()
    assert np.abs(Rg - Rr).max() < 1e-10 and rel(Vg, Vr) < 1e-8
    sim32 = lbrbc.Simulation(dict(cfg, storage="f32"), solid, R=R, Q=pl.Q)
    sim32.lb_step(40)
    u32 = sim32.lb_get_fields(f=False, sigma=False)["u"][fl]
    assert np.linalg.norm(u32 - ref.u()[fl]) / np.linalg.norm(ref.u()[fl]) < 1e-4


@pytest.mark.parametrize("storage,bar", [("bf16", 1e-2), ("f16", 2e-3)])
def test_bifurcation_with_cells_16bit(storage, bar):
    """The open planes and the compact layout in the 16-bit storages (their u, sigma and coverage
    entries in 16 bits), against the FP64 oracle at the 16-bit velocity targets."""
    from paper_1107_4889_amd import lbrbc

    nx, ny, nz = 48, 40, 64
    solid = synth.y_bifurcation(nx, ny, nz, r_parent=10.0, r_daughter=8.0, z_branch=36.0)
    pl = synth.place_cells(solid[16:nz - 16], synth.AXES, 12, seed=5, periodic=(0, 0, 0))
    R = pl.R + np.array([0.0, 0.0, 16.0])
    cfg = dict(nx=nx, ny=ny, nz=nz, periodic=(0, 0, 0), tau0=0.8, open_z=1, rho_in=1.002,
               rho_out=0.998)
    print(f"Y-bifurcation 48x40x64, {len(R)} cells, {storage}: oracle 40 steps", flush=True)
    ref = orc.Oracle(cfg, solid, R=R, Q=pl.Q)
    assert ref.step(40) == 0
    fl = solid.reshape(-1) == 0
    ur = ref.u()[fl]
    for layout in (2, 1):           # compact, then dense
        sim = lbrbc.Simulation(dict(cfg, storage=storage, f16_scale=2.0 ** 21, layout=layout), solid,
                               R=R, Q=pl.Q)
        assert sim.lb_observe().compact == (1 if layout == 2 else 0)
        sim.lb_step(40)
        assert sim.lb_observe().flags == 0
        u = sim.lb_get_fields(f=False, sigma=False)["u"][fl]
        err = np.linalg.norm(u - ur) / np.linalg.norm(ur)
        print(f"{storage}, layout {layout}: u rel L2 {err:.3e}", flush=True)
        assert err < bar
        assert np.abs(sim.rbc_get_state()[0] - ref.rbc()[0]).max() < 1e-5
        del sim


def test_cells_covering_the_open_planes_f64():
    """Cells whose supports cover the inlet and outlet planes and the layers the boundary
    extrapolates from: the boundary kernel reads the coverage counts there after the
    stream-collide and then clears them. Any count left over would double the cells' forcing
    in the next step."""
    from paper_1107_4889_amd import lbrbc

    nx, ny, nz = 24, 24, 40
    solid = synth.tube(nx, ny, nz, 10.0)
    Q = synth.random_rotations(np.random.default_rng(17), 3).reshape(3, 9)
    R = np.array([[11.5, 11.5, 2.0], [11.5, 11.5, 37.2], [11.0, 12.0, 20.0]])
    cfg = dict(nx=nx, ny=ny, nz=nz, periodic=(0, 0, 0), tau0=0.8, open_z=1, rho_in=1.002,
               rho_out=0.998)
    ref = orc.Oracle(cfg, solid, R=R, Q=Q)
    sim = lbrbc.Simulation(dict(cfg, storage="f64"), solid, R=R, Q=Q)
    fl = solid.reshape(-1) == 0
    for _ in range(3):
        assert ref.step(10) == 0
        sim.lb_step(10)
        d = sim.lb_get_fields()
        assert rel(d["u"][fl], ref.u()[fl]) < 1e-10
        assert rel(d["f"][:, fl], ref.f()[:, fl]) < 1e-10
        Rg = sim.rbc_get_state()[0]
        assert np.abs(Rg - ref.rbc()[0]).max() < 1e-10
    # the map of the final state covers nodes of both open planes and both inner layers
    sim.rbc_couple()
    moff = sim.rbc_get_map()[0]
    cnt = np.diff(moff).reshape(nz, ny, nx)
    assert cnt[0].any() and cnt[1].any() and cnt[nz - 2].any() and cnt[nz - 1].any()
