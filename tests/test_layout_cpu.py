"""Host side of the storage layouts (no GPU): the automatic choice, the footprint of the compact
layout, and its validation."""
import numpy as np
import pytest

from paper_1107_4889_amd import synth


def _fp(cfg, solid, n=0):
    from paper_1107_4889_amd import lbrbc
    return lbrbc.lb_query_footprint(lbrbc.make_config(cfg), solid, n)


def test_compact_footprint_follows_the_stored_segments():
    # a Y-bifurcation in its bounding box: few row segments hold fluid
    nx, ny, nz = 192, 192, 256
    solid = synth.y_bifurcation(nx, ny, nz, 24.0, 18.0, 170.0)
    cfg = dict(nx=nx, ny=ny, nz=nz, periodic=(0, 0, 0), tau0=0.8, open_z=1, rho_in=1.001,
               rho_out=0.999, storage="f32")
    dense, compact, auto = (_fp(dict(cfg, layout=k), solid) for k in (1, 2, 0))
    assert auto == compact < dense
    seg = np.zeros((nz, ny, (nx + 63) // 64), dtype=bool)
    for b in range(seg.shape[2]):
        seg[:, :, b] = (solid[:, :, 64 * b:64 * b + 64] == 0).any(-1)
    stored = int(seg.sum())
    # per-node planes: 2 x 19 populations, u (3), sigma (6), spread probes (4), node word and
    # two count planes, 4 bytes each: the footprint scales with the stored slots
    per_slot = (38 + 3 + 6 + 4 + 1 + 2) * 4
    assert abs(dense - per_slot * nx * ny * nz) < 0.02 * dense
    assert abs(compact - per_slot * 64 * stored) < 0.05 * compact + 64 * 1024 ** 2
    assert compact < 0.25 * dense


def test_dense_geometries_stay_dense_and_layout_is_validated():
    from paper_1107_4889_amd import lbrbc
    solid = synth.tube(64, 64, 64, 30.0)
    cfg = dict(nx=64, ny=64, nz=64, periodic=(0, 0, 1), tau0=0.8, storage="f32")
    # 80% of the row segments hold fluid: the automatic choice is dense
    assert _fp(dict(cfg, layout=0), solid) == _fp(dict(cfg, layout=1), solid)
    # a periodic box of fluid: the compact layout stores every segment, plus its tables
    box = np.zeros((64, 16, 64), dtype=np.uint8)
    scfg = dict(cfg, ny=16, periodic=(1, 1, 1))
    assert _fp(dict(scfg, layout=2), box) >= _fp(dict(scfg, layout=1), box)
    for bad in (-1, 3):
        with pytest.raises(lbrbc.LbError) as e:
            _fp(dict(cfg, layout=bad), solid)
        assert "layout" in str(e.value)
