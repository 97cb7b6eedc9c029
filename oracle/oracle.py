"""ctypes binding of the plain FP64 CPU oracle (``lbrbc_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()`` and by
the CPU-baseline leg of ``bench.py``. The product package never imports it. It shares no
code with the HIP library; the only things both sides see are the seeded inputs.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbrbc_oracle.c")
LIB = os.path.join(HERE, "liblbrbc_oracle.so")

ORC_OK, ORC_EINVAL, ORC_ENOMEM, ORC_EUNSTABLE, ORC_EOVERLAP = 0, 1, 2, 4, 5


def build() -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP over nodes/cells)."""
    cmd = ["gcc", "-O2", "-std=gnu99", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-o", LIB, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return LIB


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("periodic", ctypes.c_int * 3),
        ("forcing", ctypes.c_int),
        ("tau0", ctypes.c_double), ("delta_visc", ctypes.c_double), ("kappa", ctypes.c_double),
        ("g_ext", ctypes.c_double * 3),
        ("gammaT", ctypes.c_double), ("gammaR", ctypes.c_double), ("alpha", ctypes.c_double),
        ("mass", ctypes.c_double), ("inertia", ctypes.c_double * 3),
        ("vort_scale", ctypes.c_double),
        ("xi", ctypes.c_double * 3), ("axes", ctypes.c_double * 3), ("eps0", ctypes.c_double),
        ("a_wall", ctypes.c_double), ("sigmin_wall", ctypes.c_double),
        ("wall_particles", ctypes.c_int),
        ("open_z", ctypes.c_int), ("rho_in", ctypes.c_double), ("rho_out", ctypes.c_double),
        ("ext_force", ctypes.c_double * 3), ("ext_torque", ctypes.c_double * 3),
        ("wall_u_lo", ctypes.c_double * 3), ("wall_u_hi", ctypes.c_double * 3),
    ]


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)
_L = ctypes.POINTER(ctypes.c_long)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        L.orc_create.restype = ctypes.c_void_p
        L.orc_create.argtypes = [ctypes.POINTER(Params), ctypes.c_void_p, ctypes.c_int,
                                 _D, _D, _D, _D, _I]
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        for name in ("orc_step",):
            getattr(L, name).argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.orc_couple.argtypes = [ctypes.c_void_p]
        L.orc_collide.argtypes = [ctypes.c_void_p, ctypes.c_int, _D, _D]
        L.orc_set_fields.argtypes = [ctypes.c_void_p, _D, _D, _D]
        L.orc_num_nodes.restype = ctypes.c_long
        L.orc_num_nodes.argtypes = [ctypes.c_void_p]
        L.orc_num_fluid.restype = ctypes.c_long
        L.orc_num_fluid.argtypes = [ctypes.c_void_p]
        for name in ("orc_get_f", "orc_get_u", "orc_get_sigma", "orc_get_force",
                     "orc_get_relax", "orc_get_coupling", "orc_observe", "orc_wall_momentum"):
            getattr(L, name).argtypes = [ctypes.c_void_p, _D]
        L.orc_get_rbc.argtypes = [ctypes.c_void_p, _D, _D, _D, _D]
        L.orc_cell_grid.argtypes = [ctypes.c_void_p, _I, _D]
        L.orc_get_cells.argtypes = [ctypes.c_void_p, _I, _I]
        L.orc_get_map.restype = ctypes.c_long
        L.orc_get_map.argtypes = [ctypes.c_void_p, _I, _I]
        L.orc_num_wall_particles.argtypes = [ctypes.c_void_p]
        L.orc_wall_shear_stress.argtypes = [ctypes.c_void_p, _L, _D]
        L.orc_lattice.argtypes = [_I, _D]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_num_threads.argtypes = []
        L.orc_set_num_threads.restype = None
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        L.orc_peskin.restype = ctypes.c_double
        L.orc_peskin.argtypes = [ctypes.c_double]
        L.orc_feq.restype = ctypes.c_double
        L.orc_feq.argtypes = [ctypes.c_double, _D, ctypes.c_int]
        L.orc_force_term.restype = ctypes.c_double
        L.orc_force_term.argtypes = [ctypes.c_int, ctypes.c_double, _D, _D, ctypes.c_int]
        L.orc_gb_pair.argtypes = [ctypes.POINTER(Params), _D, _D, _D, _D, ctypes.c_int,
                                  _D, _D, _D, _D]
        L.orc_rigid_step.argtypes = [ctypes.POINTER(Params), _D, _D, _D, _D, _D, _D]
        _lib = L
    return _lib


def _p(a: np.ndarray, ct=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def make_params(cfg: dict) -> Params:
    """Build oracle parameters from a plain dict (keys as the struct fields)."""
    P = Params()
    defaults = dict(periodic=(0, 0, 1), forcing=0, tau0=1.0, delta_visc=2.0, kappa=20.0,
                    g_ext=(0.0, 0.0, 0.0), gammaT=0.1, gammaR=0.1, alpha=0.04, mass=10.0,
                    inertia=(1000.0, 1000.0, 1000.0), vort_scale=1.0, xi=(4.0, 4.0, 1.5),
                    axes=(4.0, 4.0, 1.5), eps0=1e-3, a_wall=0.5, sigmin_wall=0.5,
                    wall_particles=1, open_z=0, rho_in=1.0, rho_out=1.0,
                    ext_force=(0.0, 0.0, 0.0), ext_torque=(0.0, 0.0, 0.0),
                    wall_u_lo=(0.0, 0.0, 0.0), wall_u_hi=(0.0, 0.0, 0.0))
    d = dict(defaults)
    d.update(cfg)
    for k, v in d.items():
        if k not in [f[0] for f in Params._fields_]:
            continue
        if isinstance(v, (tuple, list, np.ndarray)):
            arr = getattr(P, k)
            for i, x in enumerate(v):
                arr[i] = x
        else:
            setattr(P, k, v)
    return P


class Oracle:
    """One oracle simulation. ``solid`` is a (nz, ny, nx) uint8 array, 1 = solid."""

    def __init__(self, cfg: dict, solid: np.ndarray, R=None, Q=None, V=None, Om=None):
        self.L = lib()
        self.cfg = dict(cfg)
        self.P = make_params(cfg)
        self.solid = np.ascontiguousarray(solid, dtype=np.uint8).reshape(-1)
        nz, ny, nx = cfg["nz"], cfg["ny"], cfg["nx"]
        assert self.solid.size == nx * ny * nz
        self.N = nx * ny * nz
        n = 0 if R is None else len(R)
        self.nrbc = n
        z3 = np.zeros((max(n, 1), 3))
        self._R = np.ascontiguousarray(R if n else z3, dtype=np.float64)
        self._Q = np.ascontiguousarray(Q if n else np.zeros((1, 9)), dtype=np.float64)
        self._V = np.ascontiguousarray(V if V is not None and n else np.zeros((max(n, 1), 3)),
                                       dtype=np.float64)
        self._O = np.ascontiguousarray(Om if Om is not None and n else np.zeros((max(n, 1), 3)),
                                       dtype=np.float64)
        st = ctypes.c_int(0)
        self.h = self.L.orc_create(ctypes.byref(self.P), self.solid.ctypes.data, n,
                                   _p(self._R), _p(self._Q), _p(self._V), _p(self._O),
                                   ctypes.byref(st))
        self.status = st.value
        if not self.h:
            raise RuntimeError(f"oracle create failed: status {st.value}")

    def __del__(self):
        if getattr(self, "h", None):
            self.L.orc_destroy(self.h)
            self.h = None

    def step(self, n: int = 1) -> int:
        return self.L.orc_step(self.h, n)

    def couple(self) -> int:
        return self.L.orc_couple(self.h)

    def collide(self, brute: bool = False):
        F = np.zeros((max(self.nrbc, 1), 3))
        T = np.zeros((max(self.nrbc, 1), 3))
        st = self.L.orc_collide(self.h, int(brute), _p(F), _p(T))
        return st, F[:self.nrbc], T[:self.nrbc]

    def set_fields(self, f=None, u=None, sigma=None):
        f = None if f is None else np.ascontiguousarray(f, dtype=np.float64)
        u = None if u is None else np.ascontiguousarray(u, dtype=np.float64)
        s = None if sigma is None else np.ascontiguousarray(sigma, dtype=np.float64)
        self.L.orc_set_fields(self.h, None if f is None else _p(f),
                              None if u is None else _p(u), None if s is None else _p(s))

    def _get(self, name, shape):
        a = np.zeros(shape)
        getattr(self.L, name)(self.h, _p(a))
        return a

    def f(self):
        return self._get("orc_get_f", (19, self.N))

    def u(self):
        return self._get("orc_get_u", (self.N, 3))

    def sigma(self):
        return self._get("orc_get_sigma", (self.N, 6))

    def force(self):
        return self._get("orc_get_force", (self.N, 3))

    def relax(self):
        return self._get("orc_get_relax", (self.N,))

    def coupling(self):
        return self._get("orc_get_coupling", (max(self.nrbc, 1), 22))[:self.nrbc]

    def rbc(self):
        n = max(self.nrbc, 1)
        R, Q, V, O = np.zeros((n, 3)), np.zeros((n, 9)), np.zeros((n, 3)), np.zeros((n, 3))
        self.L.orc_get_rbc(self.h, _p(R), _p(Q), _p(V), _p(O))
        k = self.nrbc
        return R[:k], Q[:k], V[:k], O[:k]

    def cell_grid(self):
        nc = (ctypes.c_int * 3)()
        ed = (ctypes.c_double * 3)()
        self.L.orc_cell_grid(self.h, nc, ed)
        return tuple(nc), tuple(ed)

    def cells(self):
        (a, b, c), _ = self.cell_grid()
        off = np.zeros(a * b * c + 1, dtype=np.int32)
        ids = np.zeros(max(self.nrbc, 1), dtype=np.int32)
        self.L.orc_get_cells(self.h, _p(off, ctypes.c_int), _p(ids, ctypes.c_int))
        return off, ids[:self.nrbc]

    def node_map(self):
        n = self.L.orc_get_map(self.h, None, None)
        off = np.zeros(self.N + 1, dtype=np.int32)
        ids = np.zeros(max(n, 1), dtype=np.int32)
        self.L.orc_get_map(self.h, _p(off, ctypes.c_int), _p(ids, ctypes.c_int))
        return off, ids[:n]

    def observe(self) -> dict:
        o = self._get("orc_observe", (9,))
        return dict(mass=o[0], momentum=o[1:4].copy(), flow_rate=o[4], eta_app=o[5],
                    wss_mean=o[6], wss_max=o[7], n_wall_nodes=int(o[8]))

    def wall_shear_stress(self):
        n = self.L.orc_wall_shear_stress(self.h, None, None)
        node = np.zeros(max(n, 1), dtype=np.int64)
        w = np.zeros(max(n, 1))
        self.L.orc_wall_shear_stress(self.h, _p(node, ctypes.c_long), _p(w))
        return node[:n], w[:n]

    def wall_momentum(self):
        return self._get("orc_wall_momentum", (3,))

    def num_fluid(self) -> int:
        return int(self.L.orc_num_fluid(self.h))

    def num_wall_particles(self) -> int:
        return int(self.L.orc_num_wall_particles(self.h))


# ---- primitives -------------------------------------------------------------------------
def lattice():
    c = (ctypes.c_int * 57)()
    w = (ctypes.c_double * 19)()
    lib().orc_lattice(ctypes.cast(c, _I), ctypes.cast(w, _D))
    return np.array(list(c), dtype=np.int64).reshape(19, 3), np.array(list(w))


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    lib().orc_set_num_threads(int(n))


def peskin(r: float) -> float:
    return lib().orc_peskin(float(r))


def feq(rho: float, u, p: int) -> float:
    ua = np.ascontiguousarray(u, dtype=np.float64)
    return lib().orc_feq(rho, _p(ua), p)


def force_term(forcing: int, T: float, g, u, p: int) -> float:
    ga = np.ascontiguousarray(g, dtype=np.float64)
    ua = np.ascontiguousarray(u, dtype=np.float64)
    return lib().orc_force_term(forcing, T, _p(ga), _p(ua), p)


def gb_pair(cfg: dict, Ri, Qi, Rj, Qj, wall: bool = False):
    P = make_params(cfg)
    a = [np.ascontiguousarray(x, dtype=np.float64) for x in (Ri, Qi, Rj, Qj)]
    U = np.zeros(1)
    F, ti, tj = np.zeros(3), np.zeros(3), np.zeros(3)
    st = lib().orc_gb_pair(ctypes.byref(P), _p(a[0]), _p(a[1]), _p(a[2]), _p(a[3]), int(wall),
                           _p(U), _p(F), _p(ti), _p(tj))
    return st, U[0], F, ti, tj


def rigid_step(cfg: dict, R, Q, V, Om, F, T):
    P = make_params(cfg)
    R, Q, V, Om = (np.array(x, dtype=np.float64) for x in (R, Q, V, Om))
    F = np.ascontiguousarray(F, dtype=np.float64)
    T = np.ascontiguousarray(T, dtype=np.float64)
    lib().orc_rigid_step(ctypes.byref(P), _p(R), _p(Q), _p(V), _p(Om), _p(F), _p(T))
    return R, Q, V, Om
