"""Continuous-batching request loop: many vessel simulations resident on one GPU.

Requests (a vessel, a cell count, a number of steps) arrive over time. A request is admitted
as soon as its HBM footprint fits the budget next to the requests already resident; it then
gets its own arena, its own HIP stream (default priority) and its own context of the C
library. Every scheduler tick enqueues the next chunk of steps of every resident request
with one ``lb_batch_step`` call, which interleaves the requests step by step, so their
kernels overlap on the device. Optionally each request's chunk is captured once into a HIP
graph (through PyTorch's graph API on the request's stream) and replayed. In the fused mode all
requests share one stream and ``lb_batch_step`` runs each stage of a step as one launch over
every resident request (batching at the kernel level); with graphs, the fused chunk of the
current resident set is captured once (``lb_batch_capture``) and replayed with one launch per
chunk until a request joins or leaves. A request finishes
when its last chunk's event has completed; its memory is released and queued requests are
admitted in the same tick. Latency = completion time - arrival time.
"""
from __future__ import annotations

import hashlib
import heapq
import threading
import time
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np
import torch

from . import lbrbc

_CKPT_HEADER = 88     # bytes of the checkpoint header (holds the host step counter)


@dataclass
class Request:
    rid: int
    arrival: float            # seconds after the start of the run
    cfg: dict                 # lattice configuration (lbrbc config keys)
    solid: np.ndarray         # (nz, ny, nx) uint8
    R: np.ndarray             # (n, 3) cell centres
    Q: np.ndarray             # (n, 9) orientations
    steps: int


@dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    finished: float
    steps: int
    n_fluid: int
    n_cells: int
    footprint: int
    flow_rate: float
    eta_app: float
    wss_mean: float
    mass: float
    flags: int
    digest: str = None        # SHA-1 of the final state (populations, fields, cells)
    state: dict = None        # final velocity field and cell state (keep_state=True)

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclass
class _Active:
    req: Request
    sim: lbrbc.Simulation
    stream: torch.cuda.Stream
    admitted: float
    done_steps: int = 0
    events: list = field(default_factory=list)
    graph: object = None
    graph_steps: int = 0


class Server:
    """Admission by footprint, interleaved batched steps, completion by events."""

    def __init__(self, budget_bytes: int, chunk_steps: int = 50, use_graphs: bool = False,
                 device: str = "cuda:0", max_inflight_chunks: int = 2, digests: bool = False,
                 max_active: int = 64, progress=None, fused: bool = False, keep_state: bool = False):
        if use_graphs and chunk_steps % 2:
            raise ValueError("graph chunks need an even step count (A/B buffers)")
        self.fused = fused
        # fused mode with graphs: one captured chunk per composition of the resident set
        self._bgraph = None
        self._bkey = None
        self._old_graphs: list = []    # (graph, event after its last replay): freed once done
        self.captures = 0
        self.graph_launches = 0
        self.eager_chunks = 0
        self.shared_stream = torch.cuda.Stream(device=device) if fused else None
        self.budget = int(budget_bytes)
        self.chunk = int(chunk_steps)
        self.use_graphs = use_graphs
        self.device = device
        # the fused mode keeps more chunks queued, so set-up and read-back on the host never
        # leave the device idle
        self.max_inflight = max(max_inflight_chunks, 4) if fused else max_inflight_chunks
        self.digests = digests
        self.keep_state = keep_state
        self.max_active = int(max_active)
        self.progress = progress       # called with each Result as it retires
        self.queue: list = []          # (arrival, rid, Request)
        self.active: dict = {}
        self.used = 0
        self.results: list = []
        self.t0 = None
        self._fp: dict = {}
        self.pending: list = []      # (request, footprint, future of its set-up)
        self.pool = ThreadPoolExecutor(max_workers=1)
        # A stream capture must not overlap a set-up on the worker thread: the set-up allocates
        # device memory and synchronises, which can invalidate the capture. A capture runs only
        # when it gets this lock at once; otherwise the chunk runs without a graph.
        self._capture_lock = threading.Lock()

    # -- admission ------------------------------------------------------------------------
    def footprint(self, req: Request) -> int:
        """HBM bytes of the request (computed once per request: it builds the geometry)."""
        fp = self._fp.get(req.rid)
        if fp is None:
            c = lbrbc.make_config(req.cfg)
            fp = lbrbc.lb_query_footprint(c, np.ascontiguousarray(req.solid).reshape(-1), len(req.R))
            self._fp[req.rid] = fp
        return fp

    def submit(self, req: Request):
        heapq.heappush(self.queue, (req.arrival, req.rid, req))

    def _now(self) -> float:
        return time.perf_counter() - self.t0

    def _setup(self, req: Request):
        """Context of a request on its own stream (lb_init waits for that stream only)."""
        with self._capture_lock:
            stream = torch.cuda.Stream(device=self.device)
            sim = lbrbc.Simulation(req.cfg, req.solid, R=req.R if len(req.R) else None,
                                   Q=req.Q if len(req.R) else None, device=self.device,
                                   stream=stream)
        return sim, stream

    def _admit(self):
        """Admit arrived requests in order while the budget and the slot count allow. The
        memory is reserved at once; the set-up (host geometry build and the context's first
        kernels) runs on a worker thread, so the loop keeps the device fed meanwhile."""
        while self.queue:
            arrival, rid, req = self.queue[0]
            if arrival > self._now():
                break
            fp = self.footprint(req)
            if fp > self.budget:
                raise ValueError(f"request {rid} needs {fp} B, more than the whole budget")
            if (self.used + fp > self.budget or
                    len(self.active) + len(self.pending) >= self.max_active):
                break                                   # first come, first served
            heapq.heappop(self.queue)
            self.used += fp
            self.pending.append((req, fp, self.pool.submit(self._setup, req)))
        # contexts whose set-up has finished join the resident set (in admission order)
        while self.pending and self.pending[0][2].done():
            req, fp, fut = self.pending.pop(0)
            sim, stream = fut.result()
            if self.fused:
                # steps go to the shared stream; set-up and read-back stay on `stream`
                sim.lb_set_stream(self.shared_stream)
            self.active[req.rid] = _Active(req, sim, stream, self._now())
            self.active[req.rid].footprint = fp

    # -- stepping -------------------------------------------------------------------------
    def _graph_for(self, a: _Active) -> bool:
        """Capture `chunk` steps of this request once (even count: the A/B parity returns).
        False, and nothing captured, while a set-up is running."""
        if not self._capture_lock.acquire(blocking=False):
            return False
        try:
            g = torch.cuda.CUDAGraph()
            with torch.cuda.stream(a.stream):
                with torch.cuda.graph(g, stream=a.stream):
                    a.sim.lb_step(self.chunk)
        finally:
            self._capture_lock.release()
        a.graph = g
        a.graph_steps = self.chunk
        return True

    def _enqueue(self):
        if self.fused:
            return self._enqueue_fused()
        eager, counts = [], []
        for a in self.active.values():
            left = a.req.steps - a.done_steps
            if left <= 0 or len(a.events) >= self.max_inflight:
                continue
            n = min(self.chunk, left)
            a.done_steps += n
            if self.use_graphs and n == self.chunk and (a.graph is not None or self._graph_for(a)):
                with torch.cuda.stream(a.stream):
                    a.graph.replay()
                ev = torch.cuda.Event()
                ev.record(a.stream)
                a.events.append(ev)
            else:
                eager.append(a)
                counts.append(n)
        if eager:
            lbrbc.lb_batch_step([a.sim for a in eager], counts)
            for a in eager:
                ev = torch.cuda.Event()
                ev.record(a.stream)
                a.events.append(ev)

    def _enqueue_fused(self):
        """One chunk of every resident request with steps left, as one fused batch: with graphs,
        a replay of the chunk captured for this composition of the resident set (captured anew
        when the composition changes), else the launches themselves."""
        todo = [a for a in self.active.values()
                if a.req.steps - a.done_steps > 0 and len(a.events) < self.max_inflight]
        if not todo:
            return
        counts = [min(self.chunk, a.req.steps - a.done_steps) for a in todo]
        key = tuple(a.req.rid for a in todo)
        if (self.use_graphs and all(n == self.chunk for n in counts) and
                (key == self._bkey or self._capture_batch(todo, key))):
            self._bgraph.launch()
            self.graph_launches += 1
        else:
            lbrbc.lb_batch_step([a.sim for a in todo], counts)
            self.eager_chunks += 1
        ev = torch.cuda.Event()
        ev.record(self.shared_stream)
        for a, n in zip(todo, counts):
            a.done_steps += n
            a.events.append(ev)

    def _capture_batch(self, todo, key) -> bool:
        """Capture the chunk for this composition of the resident set; False, and nothing
        captured, while a set-up is running."""
        if not self._capture_lock.acquire(blocking=False):
            return False
        try:
            self._drop_graph()
            self._bgraph = lbrbc.BatchGraph([a.sim for a in todo], self.chunk)
        finally:
            self._capture_lock.release()
        self._bkey = key
        self.captures += 1
        return True

    def _drop_graph(self):
        """Retire the current batch graph; it is freed once its last replay has finished
        (its contexts stay alive until then)."""
        if self._bgraph is not None:
            ev = torch.cuda.Event()
            ev.record(self.shared_stream)
            self._old_graphs.append((self._bgraph, ev))
        self._bgraph = None
        self._bkey = None
        self._old_graphs = [(g, e) for g, e in self._old_graphs if not e.query()]

    def _retire(self):
        for rid in list(self.active):
            a = self.active[rid]
            while a.events and a.events[0].query():
                a.events.pop(0)
            if a.done_steps >= a.req.steps and not a.events:
                if self.fused:
                    # its last chunk is complete: read it back off the shared stream
                    a.sim.lb_set_stream(a.stream)
                a.stream.synchronize()
                o = a.sim.lb_observe()
                digest = hashlib.sha1(a.sim.lb_save()[_CKPT_HEADER:]).hexdigest() if self.digests else None
                state = None
                if self.keep_state:
                    state = dict(u=a.sim.lb_get_fields(f=False, u=True, sigma=False)["u"],
                                 cells=a.sim.rbc_get_state() if a.sim.nrbc else None)
                res = Result(
                    rid=rid, arrival=a.req.arrival, admitted=a.admitted, finished=self._now(),
                    steps=a.req.steps, n_fluid=int(o.n_fluid), n_cells=int(o.n_rbc),
                    footprint=a.footprint, flow_rate=o.flow_rate, eta_app=o.eta_app,
                    wss_mean=o.wss_mean, mass=o.mass, flags=int(o.flags), digest=digest, state=state)
                self.results.append(res)
                if self.progress:
                    self.progress(res)
                self.used -= a.footprint
                a.graph = None
                if self._bkey is not None and rid in self._bkey:
                    self._drop_graph()           # it refers to this context
                del a.sim
                del self.active[rid]

    def run(self, requests, realtime: bool = True):
        """Replay the requests' arrivals in wall-clock time and serve them to completion."""
        for r in requests:
            self.submit(r if realtime else Request(**{**r.__dict__, "arrival": 0.0}))
        self.t0 = time.perf_counter()
        try:
            while self.queue or self.active or self.pending:
                if self.active:
                    self._enqueue()
                    self._retire()
                self._admit()
                if not self.active and not self.pending and self.queue:
                    wait = self.queue[0][0] - self._now()
                    if wait > 0:
                        time.sleep(min(wait, 0.01))
                time.sleep(0)
        finally:
            self.pool.shutdown(wait=True)
        makespan = self._now()
        self._drop_graph()
        torch.cuda.synchronize()
        self._old_graphs = []
        return sorted(self.results, key=lambda r: r.rid), makespan


def summary(results, makespan: float) -> dict:
    lat = np.array([r.latency for r in results])
    work = sum(r.n_fluid * r.steps for r in results)
    return {
        "requests": len(results),
        "p50_latency_s": float(np.percentile(lat, 50)) if len(lat) else None,
        "p99_latency_s": float(np.percentile(lat, 99)) if len(lat) else None,
        "aggregate_mlups": work / makespan / 1e6 if makespan > 0 else None,
        "makespan_s": makespan,
        "failed": int(sum(1 for r in results if r.flags)),
    }
