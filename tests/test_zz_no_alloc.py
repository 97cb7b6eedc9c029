"""The entry point that allocates nothing, rbc_collide_static, against rbc_collide: the same
Gay-Berne forces and torques bit for bit, written into caller-owned device arrays, on two
calls in a row, the second on a smaller input (fewer cells and a smaller cell grid)."""
import numpy as np
import pytest

from paper_1107_4889_amd import synth

pytestmark = pytest.mark.gpu


def _case(nx, ny, nz, R, n_cells, seed):
    solid, pl = synth.tube_workload(nx, ny, nz, R, n_cells=n_cells, seed=seed)
    cfg = dict(nx=nx, ny=ny, nz=nz, periodic=(0, 0, 1), tau0=0.8, g_ext=(0, 0, 1e-6), storage="f32")
    return cfg, solid, pl


def test_static_collide_equals_collide_on_two_calls():
    import torch

    from paper_1107_4889_amd import lbrbc

    cases = [_case(64, 64, 256, 30.0, 2881, 1107), _case(32, 32, 64, 14.0, 200, 1107)]
    assert len(cases[1][2].R) < len(cases[0][2].R)
    for k, (cfg, solid, pl) in enumerate(cases):
        print(f"static collide call {k + 1}: {cfg['nx']}x{cfg['ny']}x{cfg['nz']}, {len(pl.R)} cells",
              flush=True)
        sim = lbrbc.Simulation(cfg, solid, R=pl.R, Q=pl.Q)
        sim.lb_step(3)                          # cells moved off their initial placement
        F_ref, T_ref = sim.rbc_collide()
        n = sim.nrbc
        F = torch.full((n, 3), float("nan"), dtype=torch.float64, device="cuda")
        T = torch.full((n, 3), float("nan"), dtype=torch.float64, device="cuda")
        sim.rbc_collide_static(F, T)
        sim.lb_sync()
        assert np.abs(F_ref).max() > 0
        assert np.array_equal(F.cpu().numpy(), F_ref)
        assert np.array_equal(T.cpu().numpy(), T_ref)
        # the context's own state is untouched: its next steps match a twin's
        twin = lbrbc.Simulation(cfg, solid, R=pl.R, Q=pl.Q)
        twin.lb_step(3)
        twin.rbc_collide()
        sim.lb_step(2)
        twin.lb_step(2)
        assert np.array_equal(sim.rbc_get_state()[0], twin.rbc_get_state()[0])
        del sim, twin


def test_static_collide_rejects_bad_arguments():
    from paper_1107_4889_amd import lbrbc

    cfg, solid, pl = _case(32, 32, 64, 14.0, 20, 5)
    sim = lbrbc.Simulation(cfg, solid, R=pl.R, Q=pl.Q)
    st = lbrbc._lib.rbc_collide_static(sim.h, None, None)
    assert st == lbrbc.LB_EINVAL
    assert lbrbc._lib.rbc_collide_static(None, None, None) == lbrbc.LB_EINVAL
