"""Python binding of ``liblbrbc.so`` (argument marshalling only).

Every function here forwards to the C ABI of the same name declared in ``include/lbrbc.h``;
all computation runs in the HIP kernels. PyTorch supplies the device arena (a uint8 tensor)
and the HIP stream. Importing this module fails loudly when the library is not built.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch  # noqa: F401  -- loads PyTorch's HIP runtime first; the library binds to it

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbrbc.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built: run `python -c 'import __graft_entry__ as g; g.build()'`")

_lib = ctypes.CDLL(LIB_PATH)

LB_OK, LB_EINVAL, LB_ENOMEM, LB_EHIP, LB_EUNSTABLE, LB_EOVERLAP, LB_ECAPACITY, LB_ESTATE = range(8)
STATUS = {0: "LB_OK", 1: "LB_EINVAL", 2: "LB_ENOMEM", 3: "LB_EHIP", 4: "LB_EUNSTABLE",
          5: "LB_EOVERLAP", 6: "LB_ECAPACITY", 7: "LB_ESTATE"}
STORAGE = {"f64": 0, "f32": 1, "bf16": 2, "f16": 3}
SYMBOLS = ["lb_query_footprint", "lb_init", "lb_step", "rbc_couple", "rbc_collide", "lb_observe",
           "lb_wall_shear_stress", "lb_apparent_viscosity", "lb_wss_accumulate", "lb_get_fields",
           "lb_set_fields", "rbc_get_state", "rbc_set_state", "rbc_get_coupling", "rbc_get_cells",
           "rbc_get_map", "lb_save", "lb_load", "lb_batch_step", "lb_set_stream", "lb_set_side_stream",
           "rbc_collide_static", "lb_batch_capture", "lb_graph_launch", "lb_graph_destroy",
           "lb_sync",
           "lb_last_error",
           "lb_destroy", "lb_set_timing", "lb_kernel_time", "lb_map_time"]


class LbError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {STATUS.get(status, status)}")
        self.status = status


class lb_config(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("periodic", ctypes.c_int * 3), ("storage", ctypes.c_int), ("f16_scale", ctypes.c_double),
        ("forcing", ctypes.c_int), ("tau0", ctypes.c_double), ("delta_visc", ctypes.c_double),
        ("kappa", ctypes.c_double), ("g_ext", ctypes.c_double * 3),
        ("gammaT", ctypes.c_double), ("gammaR", ctypes.c_double), ("alpha", ctypes.c_double),
        ("mass", ctypes.c_double), ("inertia", ctypes.c_double * 3), ("vort_scale", ctypes.c_double),
        ("xi", ctypes.c_double * 3), ("axes", ctypes.c_double * 3), ("eps0", ctypes.c_double),
        ("a_wall", ctypes.c_double), ("sigmin_wall", ctypes.c_double),
        ("wall_particles", ctypes.c_int), ("open_z", ctypes.c_int),
        ("rho_in", ctypes.c_double), ("rho_out", ctypes.c_double), ("map_cap", ctypes.c_int),
        ("bf16_nearest", ctypes.c_int),
        ("ext_force", ctypes.c_double * 3), ("ext_torque", ctypes.c_double * 3),
        ("wall_u_lo", ctypes.c_double * 3), ("wall_u_hi", ctypes.c_double * 3),
        ("cand_cap", ctypes.c_int), ("layout", ctypes.c_int),
    ]


class lb_rbc(ctypes.Structure):
    _fields_ = [("R", ctypes.c_double * 3), ("Q", ctypes.c_double * 9),
                ("V", ctypes.c_double * 3), ("Omega", ctypes.c_double * 3)]


class lb_observables(ctypes.Structure):
    _fields_ = [("mass", ctypes.c_double), ("momentum", ctypes.c_double * 3),
                ("flow_rate", ctypes.c_double), ("eta_app", ctypes.c_double),
                ("wss_mean", ctypes.c_double), ("wss_max", ctypes.c_double),
                ("wss_time_mean", ctypes.c_double), ("step", ctypes.c_longlong),
                ("flags", ctypes.c_uint), ("n_fluid", ctypes.c_longlong),
                ("n_wall_nodes", ctypes.c_int), ("n_rbc", ctypes.c_int),
                ("compact", ctypes.c_int), ("n_stored", ctypes.c_longlong)]


_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)
_LL = ctypes.POINTER(ctypes.c_longlong)
_SZ = ctypes.POINTER(ctypes.c_size_t)

_sig = {
    "lb_query_footprint": [ctypes.POINTER(lb_config), _P, ctypes.c_int, _SZ],
    "lb_init": [ctypes.POINTER(lb_config), _P, ctypes.POINTER(lb_rbc), ctypes.c_int, _P,
                ctypes.c_size_t, _P, ctypes.POINTER(_P)],
    "lb_step": [_P, ctypes.c_int],
    "lb_set_stream": [_P, _P],
    "lb_set_side_stream": [_P, _P],
    "rbc_couple": [_P],
    "rbc_collide": [_P, _D, _D],
    "rbc_collide_static": [_P, _P, _P],
    "lb_observe": [_P, ctypes.POINTER(lb_observables)],
    "lb_wall_shear_stress": [_P, ctypes.c_int, _D, _LL, _I],
    "lb_apparent_viscosity": [_P, _D],
    "lb_wss_accumulate": [_P, ctypes.c_int],
    "lb_get_fields": [_P, _D, _D, _D, _D, _D],
    "lb_set_fields": [_P, _D, _D, _D],
    "rbc_get_state": [_P, ctypes.POINTER(lb_rbc), ctypes.c_int],
    "rbc_set_state": [_P, ctypes.POINTER(lb_rbc), ctypes.c_int],
    "rbc_get_coupling": [_P, _D, ctypes.c_int],
    "rbc_get_cells": [_P, _I, _I, _I],
    "rbc_get_map": [_P, _I, _I, _LL],
    "lb_save": [_P, _P, _SZ],
    "lb_load": [_P, _P, ctypes.c_size_t],
    "lb_batch_step": [ctypes.POINTER(_P), _I, ctypes.c_int],
    "lb_batch_capture": [ctypes.POINTER(_P), ctypes.c_int, ctypes.c_int, ctypes.POINTER(_P)],
    "lb_graph_launch": [_P],
    "lb_graph_destroy": [_P],
    "lb_sync": [_P],
    "lb_destroy": [_P],
    "lb_set_timing": [_P, ctypes.c_int],
    "lb_kernel_time": [_P, _D, _D],
    "lb_map_time": [_P, _D],
}
for _n, _a in _sig.items():
    _f = getattr(_lib, _n)
    _f.argtypes = _a
    _f.restype = None if _n in ("lb_destroy", "lb_graph_destroy") else ctypes.c_int
_lib.lb_last_error.argtypes = [_P]
_lib.lb_last_error.restype = ctypes.c_char_p


def _d(a):
    return None if a is None else a.ctypes.data_as(_D)


# ---- configuration ----------------------------------------------------------------------------
DEFAULTS = dict(periodic=(0, 0, 1), storage="f32", f16_scale=2.0 ** 21, forcing=0, tau0=0.8,
                delta_visc=2.0, kappa=20.0, g_ext=(0.0, 0.0, 0.0), gammaT=0.1, gammaR=0.1,
                alpha=0.04, mass=10.0, inertia=(1000.0, 1000.0, 1000.0), vort_scale=1.0,
                xi=(4.0, 4.0, 1.5), axes=(4.0, 4.0, 1.5), eps0=1e-3, a_wall=0.5, sigmin_wall=0.5,
                wall_particles=1, open_z=0, rho_in=1.0, rho_out=1.0, map_cap=12,
                bf16_nearest=0, ext_force=(0.0, 0.0, 0.0), ext_torque=(0.0, 0.0, 0.0), cand_cap=0,
                wall_u_lo=(0.0, 0.0, 0.0), wall_u_hi=(0.0, 0.0, 0.0), layout=0)


def make_config(cfg: dict) -> lb_config:
    d = dict(DEFAULTS)
    d.update(cfg)
    c = lb_config()
    for name, _ in lb_config._fields_:
        v = d[name]
        if name == "storage" and isinstance(v, str):
            v = STORAGE[v]
        if isinstance(v, (tuple, list, np.ndarray)):
            arr = getattr(c, name)
            for i, x in enumerate(v):
                arr[i] = x
        else:
            setattr(c, name, v)
    return c


def _cells(R, Q, V=None, Om=None):
    n = 0 if R is None else len(R)
    arr = (lb_rbc * max(n, 1))()
    for i in range(n):
        arr[i].R[:] = [float(x) for x in R[i]]
        arr[i].Q[:] = [float(x) for x in np.asarray(Q[i]).ravel()]
        if V is not None:
            arr[i].V[:] = [float(x) for x in V[i]]
        if Om is not None:
            arr[i].Omega[:] = [float(x) for x in Om[i]]
    return arr, n


def lb_query_footprint(cfg: lb_config, solid: np.ndarray, n_rbc: int) -> int:
    s = np.ascontiguousarray(solid, dtype=np.uint8)
    out = ctypes.c_size_t(0)
    st = _lib.lb_query_footprint(ctypes.byref(cfg), s.ctypes.data, n_rbc, ctypes.byref(out))
    if st:
        msg = _lib.lb_last_error(None)
        raise LbError(st, f"lb_query_footprint ({msg.decode() if msg else ''})")
    return out.value


@dataclass
class Observables:
    mass: float
    momentum: np.ndarray
    flow_rate: float
    eta_app: float
    wss_mean: float
    wss_max: float
    wss_time_mean: float
    step: int
    flags: int
    n_fluid: int
    n_wall_nodes: int
    n_rbc: int
    compact: int = 0
    n_stored: int = 0


class Simulation:
    """One lattice + cells resident on a GPU. Methods map 1:1 onto the C ABI."""

    def __init__(self, cfg: dict, solid: np.ndarray, R=None, Q=None, V=None, Om=None,
                 device: str = "cuda:0", stream=None):
        self.cfg_dict = dict(cfg)
        self.cfg = make_config(cfg)
        self.solid = np.ascontiguousarray(solid, dtype=np.uint8).reshape(-1)
        self.N = int(self.cfg.nx * self.cfg.ny * self.cfg.nz)
        assert self.solid.size == self.N, "solid mask size does not match nx*ny*nz"
        cells, n = _cells(R, Q, V, Om)
        self.nrbc = n
        self.bytes = lb_query_footprint(self.cfg, self.solid, n)
        self.device = torch.device(device)
        self.arena = torch.empty(self.bytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        # the arena comes from torch's caching allocator: tie its reuse to this stream's work
        self.arena.record_stream(self.stream)
        h = _P()
        st = _lib.lb_init(ctypes.byref(self.cfg), self.solid.ctypes.data, cells, n,
                          ctypes.c_void_p(self.arena.data_ptr()), self.bytes,
                          ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if st:
            msg = _lib.lb_last_error(None)
            raise LbError(st, f"lb_init ({msg.decode() if msg else ''})")
        self.h = h

    def __del__(self):
        if getattr(self, "h", None):
            _lib.lb_destroy(self.h)
            self.h = None

    def _chk(self, st, what):
        if st:
            msg = _lib.lb_last_error(self.h)
            raise LbError(st, f"{what} ({msg.decode() if msg else ''})")

    def lb_set_stream(self, stream):
        """Later work of this context goes to `stream` (a torch stream); the caller orders it
        after the work already enqueued."""
        self.stream = stream
        self.arena.record_stream(stream)
        self._chk(_lib.lb_set_stream(self.h, ctypes.c_void_p(stream.cuda_stream)), "lb_set_stream")

    def lb_set_side_stream(self, stream):
        """The cells' concurrent work goes to `stream` (a torch stream, kept alive here), or,
        with None, stays on the main stream."""
        self.side_stream = stream
        if stream is not None:
            self.arena.record_stream(stream)
        self._chk(_lib.lb_set_side_stream(self.h, None if stream is None else ctypes.c_void_p(stream.cuda_stream)),
                  "lb_set_side_stream")

    # -- stepping
    def lb_step(self, n: int = 1):
        self._chk(_lib.lb_step(self.h, n), "lb_step")

    def rbc_couple(self):
        self._chk(_lib.rbc_couple(self.h), "rbc_couple")

    def rbc_collide(self):
        F = np.zeros((max(self.nrbc, 1), 3))
        T = np.zeros((max(self.nrbc, 1), 3))
        self._chk(_lib.rbc_collide(self.h, _d(F), _d(T)), "rbc_collide")
        return F[:self.nrbc], T[:self.nrbc]

    def rbc_collide_static(self, F, T):
        """Gay-Berne forces and torques into device tensors F, T (float64, [n_rbc, 3]) on this
        context's stream, with no device memory of the library's own."""
        self._chk(_lib.rbc_collide_static(self.h, ctypes.c_void_p(F.data_ptr()),
                                          ctypes.c_void_p(T.data_ptr())), "rbc_collide_static")

    def lb_sync(self):
        self._chk(_lib.lb_sync(self.h), "lb_sync")

    # -- observables
    def lb_observe(self) -> Observables:
        o = lb_observables()
        self._chk(_lib.lb_observe(self.h, ctypes.byref(o)), "lb_observe")
        return Observables(o.mass, np.array(o.momentum[:]), o.flow_rate, o.eta_app, o.wss_mean,
                           o.wss_max, o.wss_time_mean, o.step, o.flags, o.n_fluid,
                           o.n_wall_nodes, o.n_rbc, o.compact, o.n_stored)

    def lb_wall_shear_stress(self, time: bool = False):
        n = ctypes.c_int(0)
        self._chk(_lib.lb_wall_shear_stress(self.h, 0, None, None, ctypes.byref(n)), "wss")
        w = np.zeros(max(n.value, 1))
        node = np.zeros(max(n.value, 1), dtype=np.int64)
        self._chk(_lib.lb_wall_shear_stress(self.h, int(time), _d(w), node.ctypes.data_as(_LL),
                                            ctypes.byref(n)), "lb_wall_shear_stress")
        return node[:n.value], w[:n.value]

    def lb_apparent_viscosity(self) -> float:
        e = ctypes.c_double(0)
        self._chk(_lib.lb_apparent_viscosity(self.h, ctypes.byref(e)), "lb_apparent_viscosity")
        return e.value

    def lb_wss_accumulate(self, on: bool):
        self._chk(_lib.lb_wss_accumulate(self.h, int(on)), "lb_wss_accumulate")

    # -- fields and state
    def lb_get_fields(self, f=True, u=True, sigma=True, g=False, relax=False):
        out = {}
        arrs = dict(f=np.zeros((19, self.N)) if f else None, u=np.zeros((self.N, 3)) if u else None,
                    sigma=np.zeros((self.N, 6)) if sigma else None,
                    g=np.zeros((self.N, 3)) if g else None, relax=np.zeros(self.N) if relax else None)
        self._chk(_lib.lb_get_fields(self.h, _d(arrs["f"]), _d(arrs["u"]), _d(arrs["sigma"]),
                                     _d(arrs["g"]), _d(arrs["relax"])), "lb_get_fields")
        for k, v in arrs.items():
            if v is not None:
                out[k] = v
        return out

    def lb_set_fields(self, f=None, u=None, sigma=None):
        f = None if f is None else np.ascontiguousarray(f, dtype=np.float64)
        u = None if u is None else np.ascontiguousarray(u, dtype=np.float64)
        s = None if sigma is None else np.ascontiguousarray(sigma, dtype=np.float64)
        self._chk(_lib.lb_set_fields(self.h, _d(f), _d(u), _d(s)), "lb_set_fields")

    def rbc_get_state(self):
        n = self.nrbc
        arr = (lb_rbc * max(n, 1))()
        self._chk(_lib.rbc_get_state(self.h, arr, n), "rbc_get_state")
        R = np.array([arr[i].R[:] for i in range(n)]).reshape(n, 3)
        Q = np.array([arr[i].Q[:] for i in range(n)]).reshape(n, 9)
        V = np.array([arr[i].V[:] for i in range(n)]).reshape(n, 3)
        O = np.array([arr[i].Omega[:] for i in range(n)]).reshape(n, 3)
        return R, Q, V, O

    def rbc_set_state(self, R, Q, V=None, Om=None):
        arr, n = _cells(R, Q, V, Om)
        self._chk(_lib.rbc_set_state(self.h, arr, n), "rbc_set_state")

    def rbc_get_coupling(self):
        o = np.zeros((max(self.nrbc, 1), 22))
        self._chk(_lib.rbc_get_coupling(self.h, _d(o), self.nrbc), "rbc_get_coupling")
        return o[:self.nrbc]

    def rbc_get_cells(self):
        nc = (ctypes.c_int * 3)()
        self._chk(_lib.rbc_get_cells(self.h, nc, None, None), "rbc_get_cells")
        ncell = tuple(nc)
        off = np.zeros(ncell[0] * ncell[1] * ncell[2] + 1, dtype=np.int32)
        ids = np.zeros(max(self.nrbc, 1), dtype=np.int32)
        self._chk(_lib.rbc_get_cells(self.h, nc, off.ctypes.data_as(_I), ids.ctypes.data_as(_I)),
                  "rbc_get_cells")
        return ncell, off, ids[:self.nrbc]

    def rbc_get_map(self):
        ln = ctypes.c_longlong(0)
        self._chk(_lib.rbc_get_map(self.h, None, None, ctypes.byref(ln)), "rbc_get_map")
        off = np.zeros(self.N + 1, dtype=np.int32)
        ids = np.zeros(max(ln.value, 1), dtype=np.int32)
        self._chk(_lib.rbc_get_map(self.h, off.ctypes.data_as(_I), ids.ctypes.data_as(_I),
                                   ctypes.byref(ln)), "rbc_get_map")
        return off, ids[:ln.value]

    # -- checkpoints
    def lb_save(self) -> bytes:
        n = ctypes.c_size_t(0)
        self._chk(_lib.lb_save(self.h, None, ctypes.byref(n)), "lb_save")
        buf = ctypes.create_string_buffer(n.value)
        self._chk(_lib.lb_save(self.h, buf, ctypes.byref(n)), "lb_save")
        return buf.raw[:n.value]

    def lb_load(self, data: bytes):
        buf = ctypes.create_string_buffer(data, len(data))
        self._chk(_lib.lb_load(self.h, buf, len(data)), "lb_load")

    # -- timing
    def lb_set_timing(self, on: bool):
        self._chk(_lib.lb_set_timing(self.h, int(on)), "lb_set_timing")

    def lb_kernel_time(self):
        a, b = ctypes.c_double(0), ctypes.c_double(0)
        self._chk(_lib.lb_kernel_time(self.h, ctypes.byref(a), ctypes.byref(b)), "lb_kernel_time")
        return a.value, b.value

    def lb_map_time(self) -> float:
        a = ctypes.c_double(0)
        self._chk(_lib.lb_map_time(self.h, ctypes.byref(a)), "lb_map_time")
        return a.value


def lb_batch_step(sims, nsteps):
    arr = (_P * len(sims))(*[s.h for s in sims])
    ns = (ctypes.c_int * len(sims))(*nsteps)
    st = _lib.lb_batch_step(arr, ns, len(sims))
    if st:
        raise LbError(st, "lb_batch_step")


class BatchGraph:
    """A captured sequence of `nsteps` fused steps over fixed contexts (lb_batch_capture);
    launch() enqueues one replay. Keeps the Simulations alive while it exists."""

    def __init__(self, sims, nsteps: int):
        self.sims = list(sims)
        arr = (_P * len(self.sims))(*[x.h for x in self.sims])
        h = _P()
        st = _lib.lb_batch_capture(arr, len(self.sims), int(nsteps), ctypes.byref(h))
        if st:
            msg = _lib.lb_last_error(self.sims[0].h)
            raise LbError(st, f"lb_batch_capture ({msg.decode() if msg else ''})")
        self.h = h
        self.nsteps = int(nsteps)

    def launch(self):
        st = _lib.lb_graph_launch(self.h)
        if st:
            raise LbError(st, "lb_graph_launch")

    def __del__(self):
        if getattr(self, "h", None):
            _lib.lb_graph_destroy(self.h)
            self.h = None
