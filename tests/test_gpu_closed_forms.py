"""GPU checks against hand-derived values and forced paths: the stress torque T^S of Eq. 16
in the four-node closed form, a singular Gay-Berne overlap raised during a step, and the
full-tile map pass (the overflow path of the one-wavefront pass) against the oracle."""
import math

import numpy as np
import pytest

from oracle import oracle as orc
from paper_1107_4889_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lb():
    from paper_1107_4889_amd import lbrbc
    return lbrbc


def _periodic(n, **kw):
    d = dict(nx=n, ny=n, nz=n, periodic=(1, 1, 1), tau0=1.0, wall_particles=0)
    d.update(kw)
    return d


@pytest.mark.parametrize("storage,tol", [("f64", 1e-13), ("f32", 2e-6)])
@pytest.mark.parametrize("alpha,comp,s", [(0.04, 4, 1e-3), (0.063, 5, -2.5e-4)])
def test_stress_torque_four_node_closed_form(lb, storage, tol, alpha, comp, s):
    """xi = (1, 1, 1/2), axis-aligned, centre (x0 + 1/2, y0 + 1/2, z0): four support nodes with
    dhat = 1/4 and n^ = -(sgn dx, sgn dy, 0)/sqrt 2, so a uniform shear stress s in the xz (yz)
    plane gives T^S = alpha sqrt(2)/4 s (0, -1, 0) ((1, 0, 0)); S = 1/8 (derivation in the
    oracle pin of the same name)."""
    n = 24
    print(f"T^S closed form: {storage}, alpha {alpha}, component {comp}", flush=True)
    sim = lb.Simulation(_periodic(n, storage=storage, alpha=alpha, xi=(1.0, 1.0, 0.5)),
                        np.zeros((n, n, n), np.uint8), R=np.array([[7.5, 8.5, 6.0]]),
                        Q=np.eye(3).reshape(1, 9))
    sig = np.zeros((n ** 3, 6))
    sig[:, comp] = s
    sim.lb_set_fields(sigma=sig)
    sim.rbc_couple()
    cp = sim.rbc_get_coupling()[0]
    k = math.sqrt(2.0) / 4.0 * alpha * s
    ref = np.array([0.0, -k, 0.0]) if comp == 4 else np.array([k, 0.0, 0.0])
    assert cp[0] == pytest.approx(0.125, rel=tol)
    assert np.abs(cp[7:10] - ref).max() <= tol * abs(k)


def test_overlap_raised_during_a_step(lb):
    """Two cells moved by rbc_set_state to 2 lu apart side by side along a long axis: the
    Gay-Berne range there is 8, so rho = (2 - 8 + 3)/3 < 0. The step's Gay-Berne pass raises
    LB_EOVERLAP at the next synchronising call, and the context refuses further steps."""
    n = 32
    R0 = np.array([[8.0, 16.0, 16.0], [24.0, 16.0, 16.0]])
    Q = np.tile(np.eye(3).reshape(1, 9), (2, 1))
    sim = lb.Simulation(_periodic(n, storage="f64"), np.zeros((n, n, n), np.uint8), R=R0, Q=Q)
    sim.lb_step(2)
    sim.lb_sync()                                   # well apart: no fault
    print("overlap during a step: two cells 2 lu apart", flush=True)
    sim.rbc_set_state(np.array([[15.0, 16.0, 16.0], [17.0, 16.0, 16.0]]), Q)
    sim.lb_step(1)
    with pytest.raises(lb.LbError) as e:
        sim.lb_sync()
    assert e.value.status == lb.LB_EOVERLAP
    with pytest.raises(lb.LbError) as e:
        sim.lb_step(1)
    assert e.value.status == lb.LB_ESTATE


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16", "f16"])
def test_full_tile_map_pass_matches_oracle(lb, storage):
    """cand_cap = 1 (raised to tile_max^2 = 289 for xi = (4, 4, 1.5)) is below every cell's
    candidate count here (each covers more than 289 nodes, checked from the oracle's map), so
    every cell of the 32x32x64 tube takes the full-tile pass: the map bit-exact and the coupling
    sums, spread force and local relaxation time equal to the oracle's and to the one-wavefront
    pass's (up to the summation order). In the 16-bit storages the fields handed over are rounded
    to 16 bits and the coverage entries are 16-bit, so the sums follow the oracle to the 16-bit
    velocity targets and the spread force to the entries' rounding."""
    solid, pl = synth.tube_workload(32, 32, 64, 14.0, n_cells=200, seed=1107)
    cfg = dict(nx=32, ny=32, nz=64, periodic=(0, 0, 1), tau0=1.0, g_ext=(0, 0, 1e-6))
    ref = orc.Oracle(cfg, solid, R=pl.R, Q=pl.Q)
    assert ref.step(5) == 0
    ref.couple()
    roff, rids = ref.node_map()
    covered = np.bincount(rids, minlength=len(pl.R))
    assert covered.min() > 17 * 17, covered.min()
    rcp = ref.coupling()
    Rr, Qr, Vr, Or = ref.rbc()
    out = {}
    for cap in (0, 1):
        print(f"full-tile map pass: {storage}, cand_cap {cap}, {len(pl.R)} cells", flush=True)
        sim = lb.Simulation(dict(cfg, storage=storage, cand_cap=cap, f16_scale=2.0 ** 21), solid, R=Rr, Q=Qr,
                            V=Vr, Om=Or)
        sim.lb_set_fields(f=ref.f(), u=ref.u(), sigma=ref.sigma())
        sim.rbc_couple()
        moff, mids = sim.rbc_get_map()
        out[cap] = (moff, mids, sim.rbc_get_coupling(), sim.lb_get_fields(f=False, u=False, sigma=False,
                                                                         g=True, relax=True))
        del sim
    moff, mids, cp, fld = out[1]
    assert np.array_equal(moff, roff) and np.array_equal(mids, rids)
    assert np.array_equal(out[0][0], moff) and np.array_equal(out[0][1], mids)
    tol = {"f64": 1e-11, "f32": 2e-5, "bf16": 1e-2, "f16": 2e-3}[storage]
    tol_g = {"f64": 1e-11, "f32": 2e-5}.get(storage, 1e-3)
    for a, b in ((0, 1), (1, 4), (4, 7), (7, 10), (10, 13), (13, 16)):
        scale = np.abs(rcp[:, a:b]).max()
        assert np.abs(cp[:, a:b] - rcp[:, a:b]).max() <= tol * scale, (a, b)
    g_ref = ref.force()
    assert np.abs(fld["g"] - g_ref).max() <= tol_g * np.abs(g_ref).max()
    assert np.abs(fld["relax"] - ref.relax()).max() <= tol_g
    # the two passes sum the same terms (in a different order)
    cp0 = out[0][2]
    tol2 = 1e-13 if storage == "f64" else 1e-6
    for a, b in ((0, 1), (1, 4), (4, 7), (7, 10), (10, 13), (13, 16)):
        assert np.abs(cp0[:, a:b] - cp[:, a:b]).max() <= tol2 * np.abs(cp[:, a:b]).max(), (a, b)
