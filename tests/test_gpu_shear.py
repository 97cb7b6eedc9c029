"""Moving walls (the wall-bounded shear cell of the tank-treading experiments, Sec. III): the GPU's
steady plane Couette flow against its exact linear profile, and a cell in the shear cell against
the oracle."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_1107_4889_amd import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("storage,tol", [("f64", 1e-11), ("f32", 2e-5)])
def test_plane_couette_steady_profile(storage, tol):
    from paper_1107_4889_amd import lbrbc

    ny, U, tau = 18, 1e-3, 0.8
    cfg = dict(nx=1, ny=ny, nz=1, periodic=(1, 0, 1), tau0=tau, wall_u_lo=(-U, 0, 0), wall_u_hi=(U, 0, 0),
               storage=storage)
    print(f"plane Couette: {storage}", flush=True)
    sim = lbrbc.Simulation(cfg, synth.slab(1, ny, 1))
    sim.lb_step(40000)
    d = sim.lb_get_fields(f=False, u=True, sigma=True)
    y = np.arange(1, ny - 1)
    assert np.allclose(d["u"][1:ny - 1, 0], U * (2 * y - ny + 1) / (ny - 2), rtol=0, atol=tol * U)
    nu = (tau - 0.5) / 3.0
    assert np.allclose(d["sigma"][1:ny - 1, 3], nu * 2 * U / (ny - 2), rtol=10 * tol)


def test_cell_in_shear_cell_matches_oracle():
    import bench
    from paper_1107_4889_amd import lbrbc

    cfg, solid, R, Q = bench.shear_cell_config(0.063, storage="f64", n=(40, 34, 24))
    print("cell in the shear cell: 40x34x24, 300 steps, FP64 and FP32", flush=True)
    ref = orc.Oracle({k: v for k, v in cfg.items() if k != "storage"}, solid, R=R, Q=Q)
    assert ref.step(300) == 0
    fl = solid.reshape(-1) == 0
    ur = ref.u()[fl]
    Rr, Qr, Vr, Or = ref.rbc()
    ts_ref = ref.coupling()[0, 7:10]
    assert np.abs(ts_ref).max() > 0
    for storage, tol in (("f64", 1e-10), ("f32", 1e-4)):
        sim = lbrbc.Simulation(dict(cfg, storage=storage), solid, R=R, Q=Q)
        sim.lb_step(300)
        u = sim.lb_get_fields(f=False, u=True, sigma=False)["u"][fl]
        assert np.linalg.norm(u - ur) <= tol * np.linalg.norm(ur), storage
        Rg, Qg, Vg, Og = sim.rbc_get_state()
        assert np.abs(Rg - Rr).max() < tol and np.abs(Qg - Qr).max() < tol, storage
        assert np.linalg.norm(Og - Or) <= 10 * tol * np.linalg.norm(Or), storage
        ts = sim.rbc_get_coupling()[0, 7:10]
        assert np.abs(ts - ts_ref).max() <= 10 * tol * np.abs(ts_ref).max(), storage
        del sim


@pytest.mark.parametrize("storage,bar,ts_bar", [("bf16", 1e-2, 5e-2), ("f16", 2e-3, 1e-2)])
def test_cell_in_shear_cell_16bit(storage, bar, ts_bar):
    """Moving walls and a tumbling cell in the 16-bit storages (u, sigma and the coverage entries in
    16 bits; the stress torque reads the 16-bit sigma) against the FP64 oracle, at the 16-bit
    velocity targets and the WSS bars for the stress torque."""
    import bench
    from paper_1107_4889_amd import lbrbc

    cfg, solid, R, Q = bench.shear_cell_config(0.063, storage="f64", n=(40, 34, 24))
    print(f"cell in the shear cell: 40x34x24, 300 steps, {storage}", flush=True)
    ref = orc.Oracle({k: v for k, v in cfg.items() if k != "storage"}, solid, R=R, Q=Q)
    assert ref.step(300) == 0
    fl = solid.reshape(-1) == 0
    ur = ref.u()[fl]
    sim = lbrbc.Simulation(dict(cfg, storage=storage, f16_scale=2.0 ** 21), solid, R=R, Q=Q)
    sim.lb_step(300)
    assert sim.lb_observe().flags == 0
    u = sim.lb_get_fields(f=False, u=True, sigma=False)["u"][fl]
    err = np.linalg.norm(u - ur) / np.linalg.norm(ur)
    ts_ref = ref.coupling()[0, 7:10]
    ts = sim.rbc_get_coupling()[0, 7:10]
    ts_err = np.abs(ts - ts_ref).max() / np.abs(ts_ref).max()
    print(f"{storage}: u rel L2 {err:.3e}, T^S rel {ts_err:.3e}", flush=True)
    assert err < bar and ts_err < ts_bar
    # the cell is carried by the shear flow: its position error is the velocity error integrated
    # over 300 steps (BF16 measured 5e-5 lu)
    assert np.abs(sim.rbc_get_state()[0] - ref.rbc()[0]).max() < 1e-3
