"""Seeded synthetic inputs: vessel geometries and cell placements.

This module is the one thing the HIP path and the CPU oracle both consume. It holds none
of the method's arithmetic (no lattice Boltzmann, no shape function, no forces): it
voxelises simple vessels and places rigid oblate ellipsoids without overlap, from a seed.

Geometry convention: arrays are shaped (nz, ny, nx) so that the flat index is
n = x + nx*(y + ny*z); node (x, y, z) sits at the point (x, y, z); 1 = solid.

Placement rule (place_cells): centres uniform in the fluid region, orientations uniform on
SO(3) (normalised Gaussian quaternions). All cells are first placed by random sequential
addition at half their size, then inflated to full size in steps, each followed by
overlap-removal sweeps that move and turn the cells (synth_pack.c). The overlap measure is
the Perram-Wertheim contact function at lambda = 1/2 of two ellipsoids with shape matrices
A = Q diag(a^2) Q^T, c = r^T (A_i + A_j)^-1 r / 2 (c >= 1: no contact), and for a cell and
a wall mesh point the same function with a sphere of radius a_wall. A placement is accepted
with every pair at c >= 0.98^2 (a slight soft overlap of the kind a small Gay-Berne energy
scale permits) and no cell-wall contact (c >= 1); the few cells still violating either bound
are dropped and the achieved hematocrit is reported.
"""
from __future__ import annotations

import hashlib
import math
import os
import sys
from dataclasses import dataclass

import numpy as np
from scipy.spatial import cKDTree


# ---- geometries ----------------------------------------------------------------------------
def tube(nx: int, ny: int, nz: int, radius: float) -> np.ndarray:
    """Straight tube along z: fluid where (x-cx)^2 + (y-cy)^2 < R^2, c = (n-1)/2."""
    x = np.arange(nx) - (nx - 1) / 2.0
    y = np.arange(ny) - (ny - 1) / 2.0
    r2 = x[None, :] ** 2 + y[:, None] ** 2
    fluid2d = r2 < radius * radius
    return np.broadcast_to(~fluid2d, (nz, ny, nx)).astype(np.uint8).copy()


def slab(nx: int, ny: int, nz: int) -> np.ndarray:
    """Plane channel: solid rows y = 0 and y = ny - 1, fluid elsewhere."""
    s = np.zeros((nz, ny, nx), dtype=np.uint8)
    s[:, 0, :] = 1
    s[:, ny - 1, :] = 1
    return s


def _capsule_fluid(P, a, b, radius):
    """Points within `radius` of the segment a-b. P: (..., 3)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    ab = b - a
    t = np.clip(((P - a) @ ab) / float(ab @ ab), 0.0, 1.0)
    d = P - (a + t[..., None] * ab)
    return (d * d).sum(-1) < radius * radius


def y_bifurcation(nx: int, ny: int, nz: int, r_parent: float, r_daughter: float,
                  z_branch: float, angle_deg: float = 30.0) -> np.ndarray:
    """Parent tube along z from z = 0 to z_branch, two daughters leaving the branch point at
    +/- angle to +z in the x-z plane up to the top face (union of capsules). Voxelised in
    z-slabs, so memory stays bounded at large sizes."""
    cx, cy = (nx - 1) / 2.0, (ny - 1) / 2.0
    th = math.radians(angle_deg)
    L = (nz - 1 - z_branch) / math.cos(th) + r_daughter + 2.0
    solid = np.empty((nz, ny, nx), dtype=np.uint8)
    slab_z = max(1, (1 << 22) // max(1, nx * ny))
    for z0 in range(0, nz, slab_z):
        z1 = min(nz, z0 + slab_z)
        zz, yy, xx = np.meshgrid(np.arange(z0, z1), np.arange(ny), np.arange(nx), indexing="ij")
        P = np.stack([xx, yy, zz], -1).astype(np.float64)
        # parent, extended below the inlet face so the inlet plane is a full disc
        fl = _capsule_fluid(P, (cx, cy, -r_parent - 2.0), (cx, cy, z_branch), r_parent)
        for sgn in (-1.0, 1.0):
            end = (cx + sgn * L * math.sin(th), cy, z_branch + L * math.cos(th))
            fl |= _capsule_fluid(P, (cx, cy, z_branch), end, r_daughter)
        solid[z0:z1] = ~fl
    return solid


def elbow(nx: int, ny: int, nz: int, radius: float, bend_radius: float) -> np.ndarray:
    """Single 90-degree bend: a tube along +z from the bottom face, a quarter torus of
    centre-line radius `bend_radius` in the x-z plane, then a tube along +x to the x face."""
    cy = (ny - 1) / 2.0
    x0 = radius + 2.0
    z0 = nz - 1 - bend_radius - radius - 2.0
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    P = np.stack([xx, yy, zz], -1).astype(np.float64)
    fl = _capsule_fluid(P, (x0, cy, -radius - 2.0), (x0, cy, z0), radius)
    # quarter torus: centre of curvature at (x0 + Rb, cy, z0)
    cxb, czb = x0 + bend_radius, z0
    dx, dz = xx - cxb, zz - czb
    ang_ok = (dx <= 0) & (dz >= 0)
    rho = np.sqrt(dx * dx + dz * dz)
    tor = ((rho - bend_radius) ** 2 + (yy - cy) ** 2) < radius * radius
    fl |= tor & ang_ok
    fl |= _capsule_fluid(P, (x0 + bend_radius, cy, z0 + bend_radius),
                         (nx + radius + 2.0, cy, z0 + bend_radius), radius)
    return (~fl).astype(np.uint8)


# ---- placement -----------------------------------------------------------------------------
def random_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """n rotation matrices uniform on SO(3), (n, 3, 3); columns are the body axes."""
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    M = np.empty((n, 3, 3))
    M[:, 0, 0] = 1 - 2 * (y * y + z * z)
    M[:, 0, 1] = 2 * (x * y - w * z)
    M[:, 0, 2] = 2 * (x * z + w * y)
    M[:, 1, 0] = 2 * (x * y + w * z)
    M[:, 1, 1] = 1 - 2 * (x * x + z * z)
    M[:, 1, 2] = 2 * (y * z - w * x)
    M[:, 2, 0] = 2 * (x * z - w * y)
    M[:, 2, 1] = 2 * (y * z + w * x)
    M[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return M


def boundary_points(solid: np.ndarray, periodic) -> np.ndarray:
    """Solid voxels with a fluid voxel among their 26 neighbours, as (m, 3) xyz."""
    s = solid.astype(bool)
    fl = ~s
    near = np.zeros_like(s)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if dx == dy == dz == 0:
                    continue
                sh = np.roll(fl, (dz, dy, dx), axis=(0, 1, 2))
                # non-periodic axes: rolled-in faces are not neighbours
                for ax, d, per in ((0, dz, periodic[2]), (1, dy, periodic[1]), (2, dx, periodic[0])):
                    if d and not per:
                        idx = [slice(None)] * 3
                        idx[ax] = 0 if d > 0 else -1
                        sh[tuple(idx)] = False
                near |= sh
    z, y, x = np.nonzero(s & near)
    return np.stack([x, y, z], 1).astype(np.float64)


def _min_image(d: np.ndarray, box: np.ndarray, periodic) -> np.ndarray:
    for a in range(3):
        if periodic[a]:
            d[..., a] -= box[a] * np.round(d[..., a] / box[a])
    return d


def _contact(r: np.ndarray, Ai: np.ndarray, Aj: np.ndarray) -> np.ndarray:
    """Perram-Wertheim contact function at lambda = 1/2: r^T (Ai + Aj)^-1 r / 2."""
    H = Ai + Aj
    x = np.linalg.solve(H, r[..., None])[..., 0]
    return 0.5 * (r * x).sum(-1)


@dataclass
class Placement:
    R: np.ndarray          # (n, 3) centres
    Q: np.ndarray          # (n, 9) row-major orientation, columns = body axes
    hematocrit: float      # achieved volume fraction of the fluid region
    s_pair: float          # final pair contact scale (1 = no contact between cells)
    attempts: int


def hematocrit_count(solid: np.ndarray, axes, H: float) -> int:
    v = 4.0 / 3.0 * math.pi * axes[0] * axes[1] * axes[2]
    return int(round(H * float((solid == 0).sum()) / v))


class _Packer:
    """Hard-ellipsoid packing state: overlap tests only, no forces or potentials."""

    def __init__(self, solid, axes, periodic, a_wall, rng):
        nz, ny, nx = solid.shape
        self.box = np.array([nx, ny, nz], dtype=np.float64)
        self.per = tuple(bool(p) for p in periodic)
        self.axes = np.asarray(axes, dtype=np.float64)
        self.S2 = np.diag(self.axes ** 2)
        amax = float(self.axes.max())
        self.r_pair = math.sqrt(4.0 * amax * amax)
        self.r_wall = math.sqrt(2.0 * (amax * amax + a_wall * a_wall))
        self.fluid = solid == 0
        self.rng = rng
        self.a_wall = a_wall
        self.Aw = (a_wall * a_wall) * np.eye(3)
        wall = boundary_points(solid, periodic)
        self.wall_base = wall.copy()
        self.fluid_xyz = np.ascontiguousarray((solid == 0).astype(np.uint8))
        # ghost copies across periodic faces, so a plain (non-periodic) tree answers
        # every query on wrapped centres
        for a in range(3):
            if self.per[a] and len(wall):
                lo = wall[wall[:, a] < self.r_wall + 1].copy()
                lo[:, a] += self.box[a]
                hi = wall[wall[:, a] > self.box[a] - self.r_wall - 1].copy()
                hi[:, a] -= self.box[a]
                wall = np.concatenate([wall, lo, hi])
        self.wall = wall
        self.wtree = cKDTree(wall) if len(wall) else None
        zf, yf, xf = np.nonzero(self.fluid)
        self.lo = np.array([xf.min(), yf.min(), zf.min()], dtype=np.float64) - 0.5
        self.hi = np.array([xf.max(), yf.max(), zf.max()], dtype=np.float64) + 0.5
        for a in range(3):
            if self.per[a]:
                self.lo[a], self.hi[a] = 0.0, self.box[a]

    def shape(self, Q):
        return Q @ self.S2 @ np.transpose(Q, (0, 2, 1))

    def centre_ok(self, c):
        ci = np.floor(c + 0.5).astype(np.int64)
        ok = np.ones(len(c), dtype=bool)
        for a in range(3):
            n = int(self.box[a])
            if self.per[a]:
                ci[:, a] %= n
            else:
                ok &= (ci[:, a] >= 0) & (ci[:, a] < n)
                ci[:, a] = np.clip(ci[:, a], 0, n - 1)
        return ok & self.fluid[ci[:, 2], ci[:, 1], ci[:, 0]]

    def walls_ok(self, c, A, ok, s2=1.0):
        if self.wtree is None:
            return ok
        idx = np.nonzero(ok)[0]
        if not len(idx):
            return ok
        cw = _wrap(c, self.box, self.per)
        d1, _ = self.wtree.query(cw[idx], k=1)
        idx = idx[d1 < self.r_wall]
        k = 64
        while len(idx):
            dist, j = self.wtree.query(cw[idx], k=k, distance_upper_bound=self.r_wall)
            full = np.isfinite(dist[:, -1])
            if full.any() and k < 1024:
                k *= 2
                continue
            rows, cols = np.nonzero(np.isfinite(dist))
            if len(rows):
                d = cw[idx[rows]] - self.wall[j[rows, cols]]
                bad = _contact(d, A[idx[rows]], np.broadcast_to(self.Aw, (len(rows), 3, 3))) < s2
                ok[np.unique(idx[rows[bad]])] = False
            break
        return ok

    def pairs_ok(self, c, A, ok, Rs, As, s2, exclude=None):
        """Reject candidates within contact scale^2 s2 of placed cells (skip `exclude`)."""
        idx = np.nonzero(ok)[0]
        if not len(idx) or not len(Rs):
            return ok
        tree = _tree(Rs, self.box, self.per)
        k = 32
        while True:
            dist, j = tree.query(_tc(c[idx], self.box, self.per), k=min(k, len(Rs)),
                                 distance_upper_bound=self.r_pair)
            if dist.ndim == 1:
                dist, j = dist[:, None], j[:, None]
            if np.isfinite(dist[:, -1]).any() and k < len(Rs):
                k *= 2
                continue
            break
        rows, cols = np.nonzero(np.isfinite(dist))
        jj = j[rows, cols]
        if exclude is not None:
            keep = jj != exclude[idx[rows]]
            rows, jj = rows[keep], jj[keep]
        if len(rows):
            d = _min_image(c[idx[rows]] - Rs[jj], self.box, self.per)
            bad = _contact(d, A[idx[rows]], As[jj]) < s2
            ok[np.unique(idx[rows[bad]])] = False
        return ok

    def min_pair_contact(self, Rs, As):
        if len(Rs) < 2:
            return np.inf
        tree = _tree(Rs, self.box, self.per)
        pr = tree.query_pairs(self.r_pair, output_type="ndarray")
        if not len(pr):
            return np.inf
        d = _min_image(Rs[pr[:, 0]] - Rs[pr[:, 1]], self.box, self.per)
        return float(_contact(d, As[pr[:, 0]], As[pr[:, 1]]).min())


def place_cells(solid: np.ndarray, axes, n_target: int, seed: int, periodic=(0, 0, 1),
                a_wall: float = 0.5, batch: int = 8192, scale0: float = 0.5,
                increments: int = 20, steps_per_increment: int = 100, final_steps: int = 3000,
                s_accept: float = 0.98, s_wall: float = 1.0, target: float = 1.0,
                target_wall: float = 1.02, damp: float = 0.8, verbose: bool = False) -> Placement:
    """Seeded placement at a target count, reached by inflation.

    1. Random sequential addition of all n_target cells with their semi-axes scaled by
       scale0 (a dilute packing: it always fits), orientations uniform on SO(3).
    2. Inflation: the scale grows to 1 in `increments` equal steps; after each one,
       `steps_per_increment` overlap-removal sweeps move and turn the cells, aiming at contact
       `target` between cells and `target_wall` (a little clear of the wall points).
    3. Sweeps at full size until every pair has contact function c >= s_accept^2 and every
       cell-wall contact c >= s_wall^2 (no wall overlap at all: the cell-wall Gay-Berne pair is
       the stiffest of the model, and a cell started inside its range would get kicks the time
       step cannot follow), or `final_steps` sweeps.
    4. Cells still violating either bound are dropped (the achieved hematocrit is reported).

    A sweep is a damped Jacobi projection on the linearised contact function: for each pair
    below the target, c(R_i - R_j) = r^T (A_i + A_j)^-1 r / 2 with x = (A_i + A_j)^-1 r has the
    gradient x with respect to R_i and x cross (A_i x) with respect to a small rotation of cell
    i; the minimum-norm move (rotations weighted by 1/a_max^2) that would lift c to the target
    is split between the two cells, averaged over each cell's contacts, capped, and applied.
    Pure geometry: no forces or potentials of the model."""
    rng = np.random.default_rng(seed)
    pk = _Packer(solid, axes, periodic, a_wall, rng)
    box, per = pk.box, pk.per
    # 1. dilute random sequential addition at scale0
    Rs = np.zeros((0, 3))
    Qs = np.zeros((0, 3, 3))
    attempts = 0
    s2 = scale0 * scale0
    budget = 200 * max(n_target, 1) + 100000
    while len(Rs) < n_target and attempts < budget:
        B = int(min(batch, 4 * (n_target - len(Rs)) + 64))
        c = pk.lo + rng.random((B, 3)) * (pk.hi - pk.lo)
        Qc = random_rotations(rng, B)
        attempts += B
        Ac = s2 * pk.shape(Qc)
        ok = pk.centre_ok(c)
        ok = pk.walls_ok(c, Ac, ok)
        ok = pk.pairs_ok(c, Ac, ok, Rs, s2 * pk.shape(Qs) if len(Qs) else np.zeros((0, 3, 3)), 1.0)
        idx = np.nonzero(ok)[0]
        accepted = []
        if len(idx):
            bt = _tree(c[idx], box, per)
            prs = bt.query_pairs(pk.r_pair, output_type="ndarray")
            conflict = {}
            if len(prs):
                a_, b_ = idx[prs[:, 0]], idx[prs[:, 1]]
                d = _min_image(c[a_] - c[b_], box, per)
                bad = _contact(d, Ac[a_], Ac[b_]) < 1.0
                for x, y in zip(a_[bad], b_[bad]):
                    lo_, hi_ = (x, y) if x < y else (y, x)
                    conflict.setdefault(hi_, []).append(lo_)
            acc = set()
            for k in idx:
                if any(j in acc for j in conflict.get(k, ())):
                    continue
                acc.add(k)
                accepted.append(k)
                if len(Rs) + len(accepted) >= n_target:
                    break
        if accepted:
            acc = np.array(accepted)
            Rs = np.concatenate([Rs, _wrap(c[acc], box, per)])
            Qs = np.concatenate([Qs, Qc[acc]])
    # 2.-3. inflation, then sweeps at full size
    sched = [scale0 + (1.0 - scale0) * (k + 1) / increments for k in range(increments)]
    for sc in sched:
        Rs, Qs, worst, nbad = _sweeps(pk, Rs, Qs, sc, target, target_wall, target, s_wall, damp,
                                      steps_per_increment)
        if verbose:
            print(f"[synth] scale {sc:.3f}: worst pair contact {worst:.4f}, {nbad} violations",
                  file=sys.stderr, flush=True)
    Rs, Qs, worst, nbad = _sweeps(pk, Rs, Qs, 1.0, target, target_wall, s_accept, s_wall, damp,
                                  final_steps)
    if verbose:
        print(f"[synth] final: worst pair contact {worst:.4f}, {nbad} violations", file=sys.stderr,
              flush=True)
    # 4. drop what still violates: cells off the fluid or meeting a wall point, then the cell
    # with most violations in each violating pair
    As = pk.shape(Qs)
    okc = pk.centre_ok(Rs)
    okc = pk.walls_ok(Rs, As, okc, s_wall * s_wall)
    Rs, As, Qs = Rs[okc], As[okc], Qs[okc]
    while len(Rs) > 1:
        tree = _tree(Rs, box, per)
        pr = tree.query_pairs(pk.r_pair, output_type="ndarray")
        if not len(pr):
            break
        d = _min_image(Rs[pr[:, 0]] - Rs[pr[:, 1]], box, per)
        c = _contact(d, As[pr[:, 0]], As[pr[:, 1]])
        bad = c < s_accept * s_accept
        if not bad.any():
            break
        cnt = np.bincount(np.concatenate([pr[bad, 0], pr[bad, 1]]), minlength=len(Rs))
        drop = set()
        for k in np.argsort(c[bad]):
            a_, b_ = pr[bad][k]
            if a_ in drop or b_ in drop:
                continue
            drop.add(a_ if cnt[a_] >= cnt[b_] else b_)
        keep = np.array([k not in drop for k in range(len(Rs))])
        Rs, As, Qs = Rs[keep], As[keep], Qs[keep]
    # orthonormal to rounding (polar factor of the accumulated rotations)
    if len(Qs):
        U, _, Vt = np.linalg.svd(Qs)
        Qs = U @ Vt
    s = min(1.0, math.sqrt(pk.min_pair_contact(Rs, As))) if len(Rs) > 1 else 1.0
    v = 4.0 / 3.0 * math.pi * float(np.prod(pk.axes))
    H = len(Rs) * v / float(pk.fluid.sum())
    return Placement(R=Rs, Q=Qs.reshape(-1, 9), hematocrit=H, s_pair=s, attempts=attempts)


_PACK = None


def _pack_lib():
    """The compiled overlap-removal sweeps (synth_pack.c), built with gcc when missing."""
    global _PACK
    if _PACK is None:
        import ctypes

        here = os.path.dirname(os.path.abspath(__file__))
        so = os.path.join(here, "libsynthpack.so")
        if not os.path.exists(so):
            build_pack(so)
        lib = ctypes.CDLL(so)
        P = ctypes.c_void_p
        lib.pack_sweeps.argtypes = [ctypes.c_int, P, P, P, P, P, P, ctypes.c_int, ctypes.c_double, P,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_int, P]
        lib.pack_sweeps.restype = ctypes.c_int
        _PACK = lib
    return _PACK


def build_pack(so=None):
    """Compile synth_pack.c into libsynthpack.so (gcc, OpenMP; no contraction, so the
    placement is the same on every host)."""
    import subprocess

    here = os.path.dirname(os.path.abspath(__file__))
    so = so or os.path.join(here, "libsynthpack.so")
    tmp = so + f".{os.getpid()}.tmp"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-shared", "-fPIC", "-o", tmp,
                    os.path.join(here, "synth_pack.c"), "-lm"], check=True)
    os.replace(tmp, so)
    return so


def _sweeps(pk: "_Packer", Rs, Qs, scale, t_pair, t_wall, s_acc, s_wacc, damp, nsweeps,
            dmax=0.25, thmax=0.1):
    """Up to nsweeps overlap-removal sweeps at the given scale of the semi-axes (synth_pack.c);
    returns centres, orientations, the smallest pair contact and the violations left."""
    import ctypes

    lib = _pack_lib()
    R = np.ascontiguousarray(Rs, dtype=np.float64).copy()
    Q = np.ascontiguousarray(Qs.reshape(-1, 9), dtype=np.float64).copy()
    dims = np.array([int(b) for b in pk.box], dtype=np.int32)
    per = np.array([1 if p else 0 for p in pk.per], dtype=np.int32)
    wall = np.ascontiguousarray(pk.wall_base, dtype=np.float64)
    axes = np.ascontiguousarray(pk.axes, dtype=np.float64)
    stats = np.zeros(2)
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    lib.pack_sweeps(len(R), p(R), p(Q), p(axes), p(dims), p(per), p(wall), len(wall) if len(R) else 0,
                    pk.a_wall, p(pk.fluid_xyz), scale, t_pair, t_wall, s_acc, s_wacc, damp, dmax,
                    thmax, int(nsweeps), p(stats))
    return R, Q.reshape(-1, 3, 3), float(stats[0]), int(stats[1])


def _wrap(c, box, periodic):
    c = c.copy()
    for a in range(3):
        if periodic[a]:
            c[:, a] %= box[a]
    return c


def _tc(pts, box, periodic):
    """Tree coordinates: wrapped on periodic axes, shifted by +32 on the others."""
    p = _wrap(pts, box, periodic)
    for a in range(3):
        if not periodic[a]:
            p[:, a] += 32.0
    return p


def _tree(pts, box, periodic):
    if any(periodic):
        # cKDTree periodic boxes need every axis; non-periodic axes get a box wide enough
        # that no wrap can bring two points closer than the query radius
        bs = np.array([box[a] if periodic[a] else 4.0 * box[a] + 128.0 for a in range(3)])
        return cKDTree(_tc(pts, box, periodic), boxsize=bs)
    return cKDTree(_tc(pts, box, periodic))


# ---- named workloads -------------------------------------------------------------------------
AXES = (4.0, 4.0, 1.5)
# bump when place_cells changes, so that cached placements are regenerated
PLACEMENT_VERSION = "inflate-v2"


def _cache_dir():
    d = os.environ.get("LBRBC_INPUT_CACHE",
                       os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                                    ".input_cache"))
    return d


def cached_placement(key: str, make):
    """Placement memoised on disk (an .npz per key); regenerated when absent."""
    d = _cache_dir()
    fn = os.path.join(d, hashlib.sha1(key.encode()).hexdigest()[:16] + ".npz")
    if os.path.exists(fn):
        z = np.load(fn)
        return Placement(R=z["R"], Q=z["Q"], hematocrit=float(z["H"]), s_pair=float(z["s"]),
                         attempts=int(z["att"]))
    print(f"[synth] generating placement {key} (cached afterwards in {d})", file=sys.stderr,
          flush=True)
    pl = make()
    try:
        os.makedirs(d, exist_ok=True)
        tmp = fn + f".{os.getpid()}.tmp.npz"
        np.savez(tmp, R=pl.R, Q=pl.Q, H=pl.hematocrit, s=pl.s_pair, att=pl.attempts)
        os.replace(tmp, fn)
    except OSError:
        pass
    return pl


def tube_workload(nx, ny, nz, radius, hematocrit=None, n_cells=None, seed=1107, **kw):
    """Tube geometry plus seeded cells. Returns (solid, Placement)."""
    solid = tube(nx, ny, nz, radius)
    if n_cells is None:
        n_cells = hematocrit_count(solid, AXES, hematocrit or 0.0)
    key = f"tube:{nx}:{ny}:{nz}:{float(radius):g}:{n_cells}:{seed}:{sorted(kw.items())}:{PLACEMENT_VERSION}"
    pl = cached_placement(key, lambda: place_cells(solid, AXES, n_cells, seed,
                                                   periodic=(0, 0, 1), **kw))
    return solid, pl


def bifurcation_workload(nx, ny, nz, r_parent, r_daughter, z_branch, hematocrit, seed=1107,
                         margin=16, **kw):
    """Y-bifurcation with open z faces plus seeded cells kept `margin` nodes away from the
    inlet and outlet planes. The voxelised geometry is memoised beside the placement.
    Returns (solid, Placement)."""
    d = _cache_dir()
    gkey = f"ybif:{nx}:{ny}:{nz}:{float(r_parent):g}:{float(r_daughter):g}:{float(z_branch):g}"
    gfn = os.path.join(d, hashlib.sha1(gkey.encode()).hexdigest()[:16] + ".geom.npz")
    solid = None
    if os.path.exists(gfn):
        z = np.load(gfn)
        solid = np.unpackbits(z["bits"], count=nx * ny * nz).reshape(nz, ny, nx)
    if solid is None:
        solid = y_bifurcation(nx, ny, nz, r_parent, r_daughter, z_branch)
        try:
            os.makedirs(d, exist_ok=True)
            tmp = gfn + f".{os.getpid()}.tmp.npz"
            np.savez_compressed(tmp, bits=np.packbits(solid.ravel()))
            os.replace(tmp, gfn)
        except OSError:
            pass
    n_cells = hematocrit_count(solid, AXES, hematocrit)
    key = f"{gkey}:{n_cells}:{seed}:lid{margin}:{sorted(kw.items())}:{PLACEMENT_VERSION}"

    def make():
        # placed in the vessel closed by solid lids `margin` nodes thick at both z faces: the
        # lids keep cells off the open planes, and every real wall point stays in the test
        closed = solid.copy()
        closed[:margin] = 1
        closed[nz - margin:] = 1
        pl = place_cells(closed, AXES, n_cells, seed, periodic=(0, 0, 0), **kw)
        v = 4.0 / 3.0 * math.pi * float(np.prod(AXES))
        return Placement(R=pl.R, Q=pl.Q, hematocrit=len(pl.R) * v / float((solid == 0).sum()),
                         s_pair=pl.s_pair, attempts=pl.attempts)

    return solid, cached_placement(key, make)


def chevron(nx: int, ny: int, nz: int, radius: float, offset: float) -> np.ndarray:
    """Tube periodic along z with one bend per period: the centre line runs straight from
    (x0, cy, 0) to (x0 + offset, cy, nz/2) and back to (x0, cy, nz), x0 = radius + 2 (union
    of capsules, with the periodic images of both segments)."""
    cy = (ny - 1) / 2.0
    x0 = radius + 2.0
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    P = np.stack([xx, yy, zz], -1).astype(np.float64)
    h = nz / 2.0
    fl = np.zeros((nz, ny, nx), dtype=bool)
    for z0 in (-nz, 0.0, nz):
        fl |= _capsule_fluid(P, (x0, cy, z0), (x0 + offset, cy, z0 + h), radius)
        fl |= _capsule_fluid(P, (x0 + offset, cy, z0 + h), (x0, cy, z0 + nz), radius)
    return (~fl).astype(np.uint8)


def _trace_request(args):
    k, seed, R, L, H, steps, bent = args
    n = int(2 * math.ceil(R) + 4)
    nz = max(L, 24)
    if bent:
        off = float(np.round(0.5 * nz * math.tan(math.radians(10.0))))
        nx = n + int(off)
        solid = chevron(nx, n, nz, R, off)
    else:
        nx = n
        solid = tube(n, n, nz, R)
    n_cells = hematocrit_count(solid, AXES, H)
    key = (f"serve:{seed}:{k}:{nx}:{n}:{nz}:{R:.6f}:{int(bent)}:{n_cells}:"
           f"{PLACEMENT_VERSION}")
    pl = cached_placement(key, lambda: place_cells(solid, AXES, n_cells, seed * 1000 + k,
                                                   periodic=(0, 0, 1)))
    return dict(nx=nx, ny=n, nz=nz, radius=R, bent=bent, solid=solid, R=pl.R, Q=pl.Q,
                hematocrit=pl.hematocrit, target_hematocrit=H)


def serving_trace(n_requests: int, rate_hz: float, seed: int = 2011, r_range=(8.0, 32.0),
                  k_range=(4.0, 16.0), h_range=(0.20, 0.50), steps_range=(500, 5000),
                  bent_fraction: float = 0.0, workers: int = 1):
    """A seeded stream of vessel requests: Poisson arrivals (exponential gaps at `rate_hz`),
    periodic tubes of radius R ~ U(r_range) and length k R with k ~ U(k_range), straight or,
    with probability `bent_fraction`, a chevron with a 20-degree bend; target hematocrit
    ~ U(h_range) (placed by place_cells; the achieved value is returned); steps
    ~ U{steps_range}. Returns a list of dicts in arrival order."""
    rng = np.random.default_rng(seed)
    t = 0.0
    jobs, arrivals = [], []
    for k in range(n_requests):
        t += rng.exponential(1.0 / rate_hz)
        R = float(rng.uniform(*r_range))
        L = int(round(float(rng.uniform(*k_range)) * R))
        H = float(rng.uniform(*h_range))
        steps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        bent = bool(rng.uniform() < bent_fraction)
        jobs.append((k, seed, R, L, H, steps, bent))
        arrivals.append(t)
    if workers > 1 and n_requests > 1:
        from concurrent.futures import ProcessPoolExecutor

        with ProcessPoolExecutor(max_workers=workers) as ex:
            done = list(ex.map(_trace_request, jobs, chunksize=1))
    else:
        done = [_trace_request(j) for j in jobs]
    for j, d, a in zip(jobs, done, arrivals):
        d.update(rid=j[0], arrival=a, steps=j[5])
    return done
