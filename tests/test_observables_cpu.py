"""The host-side structural observables (Sec. III) on configurations whose answers are known by
construction: rouleaux from explicit stacks, the cell-free layer from cells at known radii and
orientations, the radial density from counted annuli, the velocity profile of a parabola."""
import math

import numpy as np
import pytest

from paper_1107_4889_amd import observables as obs

AXES = (4.0, 4.0, 1.5)


def _rot_x(deg):
    c, s = math.cos(math.radians(deg)), math.sin(math.radians(deg))
    return np.array([[1, 0, 0], [0, c, -s], [0, s, c]], dtype=float)


def test_rouleaux_of_explicit_stacks():
    # body axis 3 (the short one) is Q's third column: Q = I stacks the discs along lab z
    I = np.eye(3)
    R, Q = [], []
    for k in range(5):                         # a rouleau of 5, 3.2 lu apart (< 1.25 * 3)
        R.append([10.0, 10.0, 10.0 + 3.2 * k])
        Q.append(I)
    R.append([10.0, 10.0, 10.0 + 3.2 * 4 + 4.0])   # 4.0 apart along the axis: a singleton
    Q.append(I)
    R.append([30.0, 10.0, 10.0])                  # a pair, the second tilted by 15 degrees
    Q.append(I)
    R.append([30.0, 10.0, 13.0])
    Q.append(_rot_x(15.0))
    R.append([30.0, 10.0, 16.0])                  # tilted by 25 degrees from its neighbour
    Q.append(_rot_x(40.0))
    R.append([50.0, 10.0, 10.0])                  # lateral offset 2.5 > 2: separate
    Q.append(I)
    R.append([52.5, 10.0, 12.0])
    Q.append(I)
    R, Q = np.array(R), np.array(Q).reshape(-1, 9)
    labels, sizes = obs.rouleaux(R, Q, AXES)
    assert sorted(sizes.tolist(), reverse=True) == [5, 2, 1, 1, 1, 1]
    assert len(set(labels[:5])) == 1 and labels[5] != labels[0]
    assert labels[6] == labels[7] and labels[8] != labels[7]
    assert labels[9] != labels[10]
    h = obs.rouleaux_histogram(R, Q, AXES)
    assert h[1] == 4 and h[2] == 1 and h[5] == 1 and h.sum() == 6
    # anti-parallel axes stack as well (a disc's axis has no sign)
    Q2 = Q.copy()
    Q2[1] = (I @ np.diag([1.0, -1.0, -1.0])).ravel()
    assert sorted(obs.rouleaux(R, Q2, AXES)[1].tolist(), reverse=True)[0] == 5


def test_rouleaux_across_a_periodic_face():
    I = np.eye(3).ravel()
    R = np.array([[8.0, 8.0, 62.5], [8.0, 8.0, 1.5], [8.0, 8.0, 4.6]])
    Q = np.tile(I, (3, 1))
    assert obs.rouleaux(R, Q, AXES)[1].max() == 2                 # not periodic: 62.5 is far
    sizes = obs.rouleaux(R, Q, AXES, box=(16, 16, 64), periodic=(0, 0, 1))[1]
    assert sizes.tolist() == [3]


def test_cell_free_layer_closed_form():
    # tube axis at (31.5, 31.5); cells with Q = I reach a = 4 radially, cells turned by 90
    # degrees about x reach 1.5 along y
    nx = ny = 64
    c = (nx - 1) / 2.0
    R, Q = [], []
    for k, ang in enumerate(np.linspace(0, 2 * np.pi, 16, endpoint=False)):
        R.append([c + 20.0 * math.cos(ang + 0.1), c + 20.0 * math.sin(ang + 0.1), 4.0 + 8.0 * (k % 3)])
        Q.append(np.eye(3))
    res = obs.cell_free_layer(np.array(R), np.array(Q).reshape(-1, 9), AXES, nx, ny, R_vessel=30.0)
    assert res["mean"] == pytest.approx(6.0, abs=1e-12) and res["min"] == pytest.approx(6.0, abs=1e-12)
    # one cell on the +y axis at r = 25 with its short axis radial: reach 26.5, layer 3.5
    R2 = np.array([[c, c + 25.0, 4.0]])
    Q2 = _rot_x(90.0).reshape(1, 9)
    assert obs.radial_extent(Q2, AXES, np.array([[0.0, 1.0, 0.0]]))[0] == pytest.approx(1.5)
    res2 = obs.cell_free_layer(R2, Q2, AXES, nx, ny, R_vessel=30.0)
    assert res2["min"] == pytest.approx(3.5, abs=1e-12)


def test_cell_radial_density_counts_annuli():
    nx = ny = 40
    nz = 10
    c = (nx - 1) / 2.0
    rng = np.random.default_rng(3)
    r = np.concatenate([5.0 + rng.random(30), 12.0 + rng.random(12)])
    t = rng.random(len(r)) * 2 * np.pi
    R = np.stack([c + r * np.cos(t), c + r * np.sin(t), rng.random(len(r)) * nz], 1)
    dens, edges = obs.cell_radial_density(R, nx, ny, nz, r_max=15.0)
    assert dens[5] == pytest.approx(30 / (math.pi * (36 - 25) * nz))
    assert dens[12] == pytest.approx(12 / (math.pi * (169 - 144) * nz))
    assert np.count_nonzero(dens) == 2


def test_radial_velocity_profile_of_a_parabola():
    nx = ny = 33
    nz = 4
    c = 16.0
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r2 = (x - c) ** 2 + (y - c) ** 2
    solid = (r2 >= 15.0 ** 2).astype(np.uint8)
    u = np.zeros((nx * ny * nz, 3))
    u[:, 2] = np.where(solid.ravel() == 0, 1.0 - r2.ravel() / 225.0, 0.0)
    prof = obs.radial_velocity_profile(u, solid, nx, ny, nz)
    # bin 0 holds only the axis nodes (r = 0; the next nodes sit at r = 1): u = 1 there
    assert prof[0] == pytest.approx(1.0)
    # every bin's mean lies between the parabola's values at its edges
    for k in range(1, 15):
        assert 1.0 - (k + 1) ** 2 / 225.0 <= prof[k] <= 1.0 - k ** 2 / 225.0 + 1e-15
