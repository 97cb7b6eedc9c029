"""Structural observables of the cell suspension (Sec. III), computed on the host from the cell
state and the velocity field that the library returns (rbc_get_state, lb_get_fields).

- Radial velocity profile of a straight tube: u_z averaged over z and angle in 1-lu bins
  (the velocity profiles of Sec. III).
- Radial density of cell centres (the inset of the cell-free-layer figure of Sec. III).
- Cell-free layer: the vessel radius minus the outermost radial extent of the cells, per
  axial slab and angular sector (the cell-free layer of Sec. III).
- Rouleaux cluster-size histogram (the shear-thinning passage of Sec. III). The paper gives no
  criterion; the one used here: two cells are stacked neighbours when their symmetry axes are
  within 20 degrees of each other, their centres are within 1.25 cell thicknesses along the
  mean axis, and their lateral offset is below half a long semi-axis. Rouleaux are the
  connected components of that relation; the histogram counts them by size.
"""
from __future__ import annotations

import numpy as np

ROULEAU_ANGLE_DEG = 20.0
ROULEAU_AXIAL_THICKNESSES = 1.25
ROULEAU_LATERAL_FRACTION = 0.5


def radial_velocity_profile(u: np.ndarray, solid: np.ndarray, nx: int, ny: int, nz: int):
    """Mean u_z over z and angle in 1-lu bins of the distance from the tube axis
    ((nx - 1)/2, (ny - 1)/2), over fluid nodes. u: (N, 3) with N = nx ny nz."""
    uz = u[:, 2].reshape(nz, ny, nx)
    fl = solid.reshape(nz, ny, nx) == 0
    yy, xx = np.mgrid[0:ny, 0:nx]
    r = np.hypot(xx - (nx - 1) / 2.0, yy - (ny - 1) / 2.0)
    b = np.broadcast_to(np.floor(r).astype(int), (nz, ny, nx))[fl]
    num = np.bincount(b, weights=uz[fl])
    cnt = np.bincount(b)
    return num / np.maximum(cnt, 1)


def cell_radial_density(R: np.ndarray, nx: int, ny: int, nz: int, r_max: float, dr: float = 1.0):
    """Number density of cell centres per unit volume in annuli of width dr around the tube axis
    (cells per lattice volume), for r in [0, r_max)."""
    r = np.hypot(R[:, 0] - (nx - 1) / 2.0, R[:, 1] - (ny - 1) / 2.0)
    edges = np.arange(0.0, r_max + dr * 0.5, dr)
    cnt, _ = np.histogram(r, bins=edges)
    vol = np.pi * (edges[1:] ** 2 - edges[:-1] ** 2) * nz
    return cnt / vol, edges


def radial_extent(Q: np.ndarray, axes, direction: np.ndarray) -> np.ndarray:
    """Support half-width of each ellipsoid (semi-axes `axes` in the body frame, orientation
    Q with body axes as columns) along unit lab directions (n, 3): sqrt(n^T Q diag(a^2) Q^T n)."""
    nb = np.einsum("nji,nj->ni", Q.reshape(-1, 3, 3), direction)      # direction in body frame
    return np.sqrt((nb * nb * np.asarray(axes, dtype=float) ** 2).sum(axis=1))


def cell_free_layer(R: np.ndarray, Q: np.ndarray, axes, nx: int, ny: int, R_vessel: float,
                    dz: float = 8.0, sectors: int = 16):
    """Vessel radius minus the outermost radial reach of the cells (centre radius plus the
    ellipsoid's extent along the radial direction), per slab of `dz` along z and each of
    `sectors` angular sectors; the mean and minimum over the occupied bins."""
    d = np.stack([R[:, 0] - (nx - 1) / 2.0, R[:, 1] - (ny - 1) / 2.0, np.zeros(len(R))], axis=1)
    r = np.linalg.norm(d, axis=1)
    nrm = d / np.maximum(r, 1e-12)[:, None]
    outer = r + radial_extent(Q, axes, nrm)
    sl = np.floor(R[:, 2] / dz).astype(int)
    sec = np.floor((np.arctan2(d[:, 1], d[:, 0]) + np.pi) / (2 * np.pi) * sectors).astype(int) % sectors
    key = sl * sectors + sec
    top = {}
    for k, o in zip(key, outer):
        top[k] = max(top.get(k, 0.0), o)
    gaps = R_vessel - np.array(list(top.values()))
    return {"mean": float(gaps.mean()), "min": float(gaps.min())}


def rouleaux(R: np.ndarray, Q: np.ndarray, axes, box=None, periodic=(0, 0, 0)):
    """Rouleaux of the cells under the criterion of the module docstring. Returns (labels,
    sizes): a cluster label per cell and the cluster sizes (index = label)."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    from scipy.spatial import cKDTree

    axes = np.asarray(axes, dtype=float)
    k_short = int(np.argmin(axes))
    thick = 2.0 * axes[k_short]
    lateral = ROULEAU_LATERAL_FRACTION * float(axes.max())
    axial = ROULEAU_AXIAL_THICKNESSES * thick
    cos_max = np.cos(np.radians(ROULEAU_ANGLE_DEG))
    n = len(R)
    if n == 0:
        return np.zeros(0, dtype=int), np.zeros(0, dtype=int)
    sym = Q.reshape(-1, 3, 3)[:, :, k_short]                       # symmetry axes (lab)
    reach = float(np.hypot(axial, lateral))
    P = np.asarray(R, dtype=float).copy()
    if box is not None and any(periodic):
        bs = np.array([box[a] if periodic[a] else 4.0 * box[a] + 4.0 * reach for a in range(3)])
        for a in range(3):
            P[:, a] = P[:, a] % box[a] if periodic[a] else P[:, a] + 2.0 * reach
        tree = cKDTree(P, boxsize=bs)
    else:
        tree = cKDTree(P)
    pr = tree.query_pairs(reach, output_type="ndarray")
    if len(pr):
        i, j = pr[:, 0], pr[:, 1]
        d = R[j] - R[i]
        if box is not None:
            for a in range(3):
                if periodic[a]:
                    d[:, a] -= box[a] * np.round(d[:, a] / box[a])
        c = np.einsum("ij,ij->i", sym[i], sym[j])
        m = np.where(c < 0, -1.0, 1.0)[:, None] * sym[j] + sym[i]    # mean axis (signs aligned)
        m /= np.linalg.norm(m, axis=1, keepdims=True)
        ax = np.abs(np.einsum("ij,ij->i", d, m))
        lat = np.linalg.norm(d - np.einsum("ij,ij->i", d, m)[:, None] * m, axis=1)
        ok = (np.abs(c) >= cos_max) & (ax <= axial) & (lat <= lateral)
        i, j = i[ok], j[ok]
    else:
        i = j = np.zeros(0, dtype=int)
    g = coo_matrix((np.ones(len(i)), (i, j)), shape=(n, n))
    _, labels = connected_components(g, directed=False)
    return labels, np.bincount(labels)


def rouleaux_histogram(R: np.ndarray, Q: np.ndarray, axes, box=None, periodic=(0, 0, 0)):
    """Number of rouleaux of each size S (index S; index 0 unused)."""
    _, sizes = rouleaux(R, Q, axes, box, periodic)
    return np.bincount(sizes) if len(sizes) else np.zeros(1, dtype=int)
