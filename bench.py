#!/usr/bin/env python
"""Benchmark of the coupled plasma / rigid-RBC time step on one MI355X.

Workload (default): the largest single-GPU configuration, a straight tube of radius 120 lu
along z in a 256x256x1024 box (periodic in z, body-force driven g = 1e-6, T0 = 0.8), with
184,341 cells of semi-axes (4, 4, 1.5) placed from seed 1107 at hematocrit 0.40 (the achieved
count is reported), FP32 shifted populations with FP32 arithmetic. One step = every stage of
the hot path: rigid-body first half, cell list, coverage map, interpolation, Gay-Berne forces,
rigid-body second half, fused spreading + stream-collide. --workload tube128 times the
128x128x512 tube (R = 60, hematocrit 0.35), bif384 the Y-bifurcation.

Prints one JSON line: MLUPS of the whole step (fluid-node updates per second), the
stream-collide kernel's roofline against HBM (algorithmic bytes per launch over its mean
HIP-event duration on the library's stream), the request-latency part of the metric (p50/p99
latency and aggregate MLUPS of a seeded stream of 256 vessel requests served with fused
launches; --no-serving skips it), and the FP64 CPU oracle timed on a bounded sample of the
same workload.

Other modes: --serve (a serving line of its own), --precision (reduced-precision storage
against FP64 on the same GPU), --copy-calibration (HBM counter calibration).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
STORAGE_BYTES = {"f64": 8, "f32": 4, "bf16": 2, "f16": 2}
LAYOUTS = {"auto": 0, "dense": 1, "compact": 2}


def kernel_source_hash() -> str:
    h = hashlib.sha1()
    for f in ("lb_kernels.hip", "lbrbc_device.h"):
        h.update(open(os.path.join(ROOT, "paper_1107_4889_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:12]


def measured_traffic(workload: str, storage: str, layout: str):
    """HBM bytes per stream-collide launch from the committed rocprofv3 counter summary,
    or None when the kernel source changed since the counters were taken."""
    fn = os.path.join(ROOT, "profiles", f"traffic_stream_collide_{workload}_{storage}_{layout}.json")
    if not os.path.exists(fn):
        return None
    d = json.load(open(fn))
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d.get("bytes_per_launch")


# The map pass's algorithmic bytes per cell: for each covered node (391.6 per cell on average
# for the (4, 4, 1.5) support over sampled orientations and offsets) its node word (4 B), u (3
# elements), its coverage count read and written (8 B), the slot id (4 B) and the entry (raw,
# grad raw: 4 elements); for each inside node (191.9 per cell) sigma (6 elements). Elements are
# in the compute precision, 16 bits for the 16-bit storages.
MAP_COVERED_PER_CELL, MAP_INSIDE_PER_CELL = 391.6, 191.9


def map_bytes_per_cell(storage: str) -> float:
    # v: the element of u, sigma and the coverage entries (the compute precision; 16 bits for
    # the 16-bit storages)
    v = {"f64": 8, "f32": 4}.get(storage, 2)
    return MAP_COVERED_PER_CELL * (4 + 3 * v + 8 + 4 + 4 * v) + MAP_INSIDE_PER_CELL * 6 * v


def map_pass_record(storage: str, n_cells: int, map_ms: float):
    """The map pass (one launch per step): its mean duration from HIP events and its
    algorithmic bytes (map_bytes_per_cell x cells) over that duration."""
    if n_cells == 0 or map_ms <= 0:
        return None
    b = map_bytes_per_cell(storage) * n_cells
    return {"ms_per_launch": round(map_ms, 5), "algorithmic_bytes_per_cell": round(map_bytes_per_cell(storage), 1),
            "hbm_gbs_algorithmic": round(b / (map_ms * 1e-3) / 1e9, 1),
            "frac": round(b / (map_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}


def workload(name: str, storage: str):
    from paper_1107_4889_amd import synth

    if name == "tube128":
        nx, ny, nz, R, H, T0 = 128, 128, 512, 60.0, 0.35, 0.8
        solid, pl = synth.tube_workload(nx, ny, nz, R, hematocrit=H, seed=1107)
    elif name == "tube128_h0":
        # the same tube without cells (the zero-hematocrit twin of the relative viscosity)
        nx, ny, nz, R, H, T0 = 128, 128, 512, 60.0, 0.0, 0.8
        solid, pl = synth.tube_workload(nx, ny, nz, R, n_cells=0, seed=1107)
    elif name == "tube256":
        # the 256x256x1024 study tube at hematocrit 0.40
        nx, ny, nz, R, H, T0 = 256, 256, 1024, 120.0, 0.40, 0.8
        solid, pl = synth.tube_workload(nx, ny, nz, R, hematocrit=H, seed=1107)
    elif name == "bif384":
        # Y-bifurcation 384x384x768, parent R = 48 on the axis up to z = 512, daughters R = 36
        # at +/-30 degrees to the top face; pressure-driven (open z faces, rho 1 +/- 1e-3);
        # cells at hematocrit 0.45, 16 nodes clear of the open planes
        nx, ny, nz, H, T0 = 384, 384, 768, 0.45, 0.8
        solid, pl = synth.bifurcation_workload(nx, ny, nz, 48.0, 36.0, 512.0, H, seed=1107)
        cfg = dict(nx=nx, ny=ny, nz=nz, periodic=(0, 0, 0), tau0=T0, g_ext=(0.0, 0.0, 0.0),
                   open_z=1, rho_in=1.001, rho_out=0.999, storage=storage, f16_scale=2.0 ** 21)
        desc = (f"Y-bifurcation {nx}x{ny}x{nz} (parent R=48 to z=512, daughters R=36 at "
                f"+/-30 deg), open z faces rho 1 +/- 1e-3, {len(pl.R)} cells "
                f"(H={pl.hematocrit:.3f}, target {H}), {storage} shifted storage, T0={T0}")
        return cfg, solid, pl, desc
    elif name == "tube32":
        nx, ny, nz, R, H, T0 = 32, 32, 64, 14.0, None, 1.0
        solid, pl = synth.tube_workload(nx, ny, nz, R, n_cells=110, seed=1107)
    else:
        raise SystemExit(f"unknown workload {name}")
    cfg = dict(nx=nx, ny=ny, nz=nz, periodic=(0, 0, 1), tau0=T0, g_ext=(0.0, 0.0, 1e-6),
               storage=storage, f16_scale=2.0 ** 21)
    desc = (f"tube {nx}x{ny}x{nz} R={R:g} periodic z, {len(pl.R)} cells (H={pl.hematocrit:.3f}"
            f"{'' if H is None else f', target {H}'}), {storage} shifted storage, T0={T0}, g=1e-6")
    return cfg, solid, pl, desc


def cpu_baseline(cfg, solid, pl, n_fluid: int, hematocrit=None, steps: int = 1):
    """The FP64 oracle, as it stands, on a bounded sample of the timed workload, with all host
    threads and with one. A tube workload is sampled as the 64x64x256 tube of radius 30 at the
    same hematocrit (the subsample of the precision study); other workloads run one step of
    themselves."""
    from oracle import oracle as orc
    from paper_1107_4889_amd import synth

    ocfg = {k: v for k, v in cfg.items() if k not in ("storage", "f16_scale")}
    if hematocrit is not None:
        solid, pl = synth.tube_workload(64, 64, 256, 30.0, hematocrit=hematocrit, seed=1107)
        ocfg = dict(ocfg, nx=64, ny=64, nz=256)
        n_fluid = int((solid == 0).sum())
        what = (f"{steps} coupled step(s) of the 64x64x256 tube of radius 30 at the workload's "
                f"hematocrit {hematocrit} ({n_fluid} fluid nodes, {len(pl.R)} cells), after set-up")
    else:
        what = f"{steps} coupled step(s) of the workload itself ({n_fluid} fluid nodes, {len(pl.R)} cells)"
    nthr = orc.num_threads()
    rates = {}
    for threads in (nthr, 1):
        orc.set_num_threads(threads)
        o = orc.Oracle(ocfg, solid, R=pl.R, Q=pl.Q)
        t0 = time.perf_counter()
        st = o.step(steps)
        dt = time.perf_counter() - t0
        del o
        if st != 0:
            return None
        rates[threads] = (n_fluid * steps / dt / 1e6, dt)
        print(f"[bench] oracle on {threads} thread(s): {rates[threads][0]:.4f} MLUPS ({dt:.1f} s)",
              file=sys.stderr, flush=True)
    orc.set_num_threads(nthr)
    return {"value": round(rates[nthr][0], 4), "unit": "MLUPS", "cores": nthr, "kind": "oracle",
            "sample": f"{what}; {rates[nthr][1]:.1f} s on {nthr} threads, {rates[1][1]:.1f} s on one",
            "value_one_thread": round(rates[1][0], 4)}


def run_serving(args):
    """Continuous batching of a seeded request stream (Poisson arrivals in wall-clock time):
    p50/p99 request latency beside the aggregate MLUPS over the makespan. Returns
    (aggregate MLUPS, serving record, workload description, total steps)."""
    import numpy as np
    import torch

    from paper_1107_4889_amd import synth
    from paper_1107_4889_amd.serving import Request, Server, summary

    t0 = time.perf_counter()
    tr = synth.serving_trace(args.requests, args.rate, seed=2011, bent_fraction=0.5,
                             workers=args.workers)
    print(f"[serve] {len(tr)} requests generated in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)

    def req(d, arrival=None):
        cfg = dict(nx=d["nx"], ny=d["ny"], nz=d["nz"], periodic=(0, 0, 1), tau0=0.8,
                   g_ext=(0.0, 0.0, 1e-6), storage=args.storage, f16_scale=2.0 ** 21,
                   layout=LAYOUTS[getattr(args, "layout", "auto")])
        return Request(rid=d["rid"], arrival=d["arrival"] if arrival is None else arrival,
                       cfg=cfg, solid=d["solid"], R=d["R"], Q=d["Q"], steps=d["steps"])

    # untimed warm-up: one small request through the same server path (module load, graphs)
    small = min(tr, key=lambda d: d["nx"] * d["ny"] * d["nz"])
    w = dict(small, steps=2 * args.chunk)
    Server(1 << 40, chunk_steps=args.chunk, use_graphs=args.graphs, fused=args.fused).run([req(w, 0.0)])
    torch.cuda.synchronize()

    n_done = [0]

    def progress(r):
        n_done[0] += 1
        if n_done[0] % 16 == 0 or n_done[0] == len(tr):
            print(f"[serve] {n_done[0]}/{len(tr)} done, last latency {r.latency:.2f} s",
                  file=sys.stderr, flush=True)

    srv = Server(int(args.budget_gib * (1 << 30)), chunk_steps=args.chunk,
                 use_graphs=args.graphs, max_active=args.max_active, progress=progress,
                 fused=args.fused)
    results, makespan = srv.run([req(d) for d in tr])
    sm = summary(results, makespan)
    lu = sum(r.n_fluid * r.steps for r in results)
    desc = (f"serving: {len(tr)} requests, Poisson arrivals at {args.rate:g}/s, "
            "straight tubes and 20-degree chevrons (1:1), R ~ U(8, 32), length "
            "~ U(4, 16) R, target hematocrit ~ U(0.2, 0.5) (placement by inflation: "
            "achieved values reported), steps ~ U{500..5000}, "
            f"{args.storage} storage")
    record = {
        "aggregate_mlups": round(sm["aggregate_mlups"], 2),
        "p50_latency_s": round(sm["p50_latency_s"], 4),
        "p99_latency_s": round(sm["p99_latency_s"], 4),
        "makespan_s": round(makespan, 3),
        "requests": sm["requests"],
        "failed": sm["failed"],
        "lattice_updates": int(lu),
        "mean_hematocrit": round(float(np.mean([d["hematocrit"] for d in tr])), 4),
        "chunk_steps": args.chunk,
        "hip_graphs": bool(args.graphs),
        "fused_launches": bool(args.fused),
        # fused: one launch per stage over every resident request (cell binning, scan, scatter,
        # sort, map pass, overflow map pass, Gay-Berne, kick, stream-collide); otherwise the
        # same stages per request
        "kernel_launches_per_step": 9 if args.fused else "9-11 per request",
        "budget_gib": args.budget_gib,
        "max_active": args.max_active,
        "mean_queue_wait_s": round(float(np.mean([r.admitted - r.arrival for r in results])), 4),
        "workload": desc,
    }
    return sm["aggregate_mlups"], record, desc, int(sum(r.steps for r in results))


def serve(args):
    """Serving mode: the JSON line's value is the aggregate MLUPS of the request stream."""
    agg, record, desc, steps = run_serving(args)
    line = {
        "metric": "MLUPS & achieved HBM GB/s (LBM+RBC step); p50/p99 request latency",
        "value": round(agg, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": steps,
        "warmup": 1,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.storage,
        "compute_dtype": "f64" if args.storage == "f64" else "f32",
        "data": "synthetic",
        "config": {
            "workload": desc,
            "storage": args.storage,
            "parallelism": ("single GPU, one launch per stage over all resident requests" if args.fused
                            else "single GPU, one HIP stream per resident request"),
        },
        "serving": record,
    }
    print(json.dumps(line), flush=True)


def precision(args):
    """Reduced-precision storage against FP64 on the same GPU: a 64x64x256 tube of radius
    30 lu at target hematocrit 0.40 (the subsample of the 256x256x1024 study), run for
    --steps steps in each storage; velocity and wall-shear-stress errors against the FP64
    run, with and without cells (the FP64 path itself is held to the oracle by the parity
    tests, also at this size)."""
    import numpy as np
    import torch

    from paper_1107_4889_amd import lbrbc, synth

    nx, ny, nz, R, H = 64, 64, 256, 30.0, 0.40
    solid, pl = synth.tube_workload(nx, ny, nz, R, hematocrit=H, seed=1107)
    fluid = (solid.reshape(-1) == 0)
    n_fluid = int(fluid.sum())
    print(f"[precision] tube {nx}x{ny}x{nz} R={R:g}, {len(pl.R)} cells (H={pl.hematocrit:.3f})",
          file=sys.stderr, flush=True)

    def cfg(st):
        # "bf16": stochastic rounding (the default); "bf16rne": round to nearest even
        return dict(nx=nx, ny=ny, nz=nz, periodic=(0, 0, 1), tau0=0.8, g_ext=(0.0, 0.0, 1e-6),
                    storage="bf16" if st.startswith("bf16") else st, f16_scale=2.0 ** 21,
                    bf16_nearest=1 if st == "bf16rne" else 0)

    def run(st, cells):
        sim = lbrbc.Simulation(cfg(st), solid, R=pl.R if cells else None,
                               Q=pl.Q if cells else None)
        half = args.steps // 2
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.lb_step(half)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        sim.lb_wss_accumulate(True)
        t0 = time.perf_counter()
        sim.lb_step(args.steps - half)
        torch.cuda.synchronize()
        dt += time.perf_counter() - t0
        obs = sim.lb_observe()
        u = sim.lb_get_fields(f=False, u=True, sigma=False)["u"][fluid]
        _, wss = sim.lb_wall_shear_stress(False)
        _, wss_t = sim.lb_wall_shear_stress(True)
        Rc = sim.rbc_get_state()[0] if cells else None
        print(f"[precision] {st} {'cells' if cells else 'plasma'}: {args.steps} steps in {dt:.2f} s, "
              f"flags {obs.flags}", file=sys.stderr, flush=True)
        return dict(u=u, wss=wss, wss_t=wss_t, eta=obs.eta_app, Q=obs.flow_rate, R=Rc,
                    mlups=n_fluid * args.steps / dt / 1e6, flags=int(obs.flags))

    def rel(a, b):
        return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))

    out = {}
    for cells in (False, True):
        key = "cells" if cells else "plasma_only"
        ref = run("f64", cells)
        rows = {"f64": {"mlups": round(ref["mlups"], 1), "flags": ref["flags"]}}
        for st in ("f32", "bf16", "bf16rne", "f16"):
            r = run(st, cells)
            row = {
                "mlups": round(r["mlups"], 1),
                "speedup_vs_f64": round(r["mlups"] / ref["mlups"], 3),
                "u_rel_l2": rel(r["u"], ref["u"]),
                "u_max_abs_over_umax": float(np.abs(r["u"] - ref["u"]).max() / np.abs(ref["u"]).max()),
                "wss_rel_l2": rel(r["wss"], ref["wss"]),
                "wss_time_avg_rel_l2": rel(r["wss_t"], ref["wss_t"]),
                "eta_app_rel": abs(r["eta"] - ref["eta"]) / abs(ref["eta"]),
                "flags": r["flags"],
            }
            if cells:
                d = r["R"] - ref["R"]
                d[:, 2] -= nz * np.round(d[:, 2] / nz)
                row["cell_pos_rms_lu"] = float(np.sqrt((d ** 2).sum(1).mean()))
            rows[st] = row
        out[key] = rows

    line = {
        "metric": "velocity / wall-shear-stress error of reduced-precision storage vs FP64, and MLUPS",
        "config": {"workload": (f"tube {nx}x{ny}x{nz} R={R:g} periodic z, {len(pl.R)} cells "
                                f"(H={pl.hematocrit:.3f}, target {H}), T0=0.8, g=1e-6, "
                                f"{args.steps} steps; WSS time average over the second half"),
                   "n_fluid": n_fluid},
        "results": out,
    }
    print(json.dumps(line), flush=True)


def observables(args):
    """The tube's observables near steady state (Sec. III): the cell-laden 128x128x512 tube and
    its H = 0 twin run for --obs-steps steps; flow rate, apparent and relative viscosity
    (eta_rel = Q_0 / Q_H), the radial profile of u_z (1-lu bins, averaged over z and angle), the
    time-averaged wall shear stress (mean and spread) over the last quarter, the radial density of
    the cell centres, the cell-free layer and the rouleaux cluster-size histogram, the last two
    averaged over four snapshots of the last quarter."""
    import numpy as np
    import torch

    from paper_1107_4889_amd import lbrbc
    from paper_1107_4889_amd import observables as ob
    from paper_1107_4889_amd.synth import AXES

    out = {}
    prof = {}
    for name in ("tube128_h0", "tube128"):
        cfg, solid, pl, desc = workload(name, "f32")
        sim = lbrbc.Simulation(cfg, solid, R=pl.R if len(pl.R) else None, Q=pl.Q if len(pl.R) else None)
        n = args.obs_steps
        nx, ny, nz = cfg["nx"], cfg["ny"], cfg["nz"]
        t0 = time.perf_counter()
        sim.lb_step(n - n // 4)
        sim.lb_wss_accumulate(True)
        cfl, hist = [], []
        for k in range(4):
            sim.lb_step(n // 16)
            torch.cuda.synchronize()
            if len(pl.R):
                Rc, Qc = sim.rbc_get_state()[:2]
                cfl.append(ob.cell_free_layer(Rc, Qc, AXES, nx, ny, R_vessel=60.0))
                hist.append(ob.rouleaux_histogram(Rc, Qc, AXES, box=(nx, ny, nz), periodic=(0, 0, 1)))
            print(f"[observables] {name}: {n - n // 4 + (k + 1) * (n // 16)}/{n} steps", file=sys.stderr,
                  flush=True)
        dt = time.perf_counter() - t0
        o = sim.lb_observe()
        u = sim.lb_get_fields(f=False, u=True, sigma=False)["u"]
        prof[name] = ob.radial_velocity_profile(u, solid, nx, ny, nz).tolist()
        _, wss_t = sim.lb_wall_shear_stress(True)
        rec = {"steps": n, "seconds": round(dt, 2), "flow_rate": o.flow_rate, "eta_app": o.eta_app,
               "wss_time_avg_mean": float(wss_t.mean()), "wss_time_avg_std": float(wss_t.std()),
               "flags": int(o.flags)}
        if len(pl.R):
            Rc = sim.rbc_get_state()[0]
            dens, edges = ob.cell_radial_density(Rc, nx, ny, nz, r_max=60.0)
            rec["cell_centre_radial_density"] = [round(float(x), 7) for x in dens]
            rec["cell_centre_r_max"] = float(np.hypot(Rc[:, 0] - (nx - 1) / 2, Rc[:, 1] - (ny - 1) / 2).max())
            rec["cell_free_layer"] = {k: float(np.mean([c[k] for c in cfl])) for k in cfl[0]}
            L = max(len(h) for h in hist)
            rec["rouleaux_histogram_mean"] = (np.mean([np.pad(h, (0, L - len(h))) for h in hist], axis=0)
                                              .round(2).tolist())
        out[name] = rec
        del sim
    line = {
        "metric": "tube observables near steady state (FP32)",
        "config": {"workload": "tube 128x128x512 R=60, 20,150 cells (H=0.35) and its H=0 twin, "
                               "T0=0.8, g=1e-6"},
        "results": out,
        "eta_rel": out["tube128_h0"]["flow_rate"] / out["tube128"]["flow_rate"],
        "u_z_radial_profile": prof,
    }
    print(json.dumps(line), flush=True)


def mobility(args):
    """Single-cell mobilities (Sec. III): a lone cell in a periodic 60^3 box of quiescent plasma
    (no viscosity contrast, M = 10, I = 1000, shape-function radii 2, 2, 1 with the short one
    on the symmetry axis), driven by a constant external force along the symmetry axis
    (frontal) or along a long axis (side-wise), or spun by a constant torque about the same
    two axes. A uniform body force of the opposite total acts on the plasma, so the total
    momentum stays zero. The steady mobilities, relative to the mean plasma velocity, are
    fitted as linear in 1/(M gT) (1/(I gR)): the intercepts are the mobilities the coupling
    keeps at infinite friction, mu_T = 1/(M gT^mesh) and 1/(I gR^mesh)."""
    import numpy as np
    import torch

    from paper_1107_4889_amd import lbrbc

    n = 60
    solid = np.zeros((n, n, n), dtype=np.uint8)
    R0 = np.array([[n / 2.0, n / 2.0, n / 2.0]])
    Q0 = np.eye(3).reshape(1, 9)
    xs = args.mob_xi_scale
    base = dict(nx=n, ny=n, nz=n, periodic=(1, 1, 1), tau0=1.0, wall_particles=0, delta_visc=0.0,
                xi=(2.0 * xs, 2.0 * xs, 1.0 * xs), mass=10.0, inertia=(1000.0, 1000.0, 1000.0),
                storage="f64")
    # translation: gT swept at gR = 0.01; rotation: gR swept at gT = 0.01 (the explicit
    # rotational exchange, I gR against the plasma inside a support one node thick across the
    # disc, is the first to lose stability)
    sweeps = {"frontal": [0.01, 0.02, 0.05, 0.1], "side-wise": [0.01, 0.02, 0.05, 0.1],
              "spin_short_axis": [0.005, 0.01, 0.02, 0.05], "spin_long_axis": [0.005, 0.01, 0.02, 0.05]}
    F, T = 1e-4, 1e-2
    steps = args.mob_steps
    out = {}
    kinds = [k for k in (("frontal", 2), ("side-wise", 0), ("spin_short_axis", 2), ("spin_long_axis", 0))
             if k[0] in args.mob_kinds.split(",")]
    for kind, axis in kinds:
        rows = []
        spin = kind.startswith("spin")
        for g in sweeps[kind]:
            cfg = dict(base, gammaT=0.01 if spin else g, gammaR=g if spin else 0.01)
            e = np.zeros(3)
            e[axis] = 1.0
            if spin:
                cfg["ext_torque"] = tuple(T * e)
            else:
                cfg["ext_force"] = tuple(F * e)
                cfg["g_ext"] = tuple(-F * e / n ** 3)
            sim = lbrbc.Simulation(cfg, solid, R=R0, Q=Q0)
            t0 = time.perf_counter()
            vals = []
            try:
                for part in (steps // 2, steps - steps // 2):
                    sim.lb_step(part)
                    o = sim.lb_observe()
                    Rg, Qg, Vg, Og = sim.rbc_get_state()
                    if spin:
                        vals.append(float(Og[0][axis]) / T)
                    else:
                        ubar = np.array(o.momentum) / o.mass
                        vals.append(float(Vg[0][axis] - ubar[axis]) / F)
            except lbrbc.LbError as err:
                print(f"[mobility] {kind} gamma={g}: {err}", file=sys.stderr, flush=True)
                rows.append({"gamma": g, "unstable": True})
                del sim
                continue
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            x = 1.0 / (1000.0 * g) if spin else 1.0 / (10.0 * g)
            rows.append({"gamma": g, "x": x, "mobility": vals[-1], "mobility_half_steps": vals[0],
                         "seconds": round(dt, 2)})
            print(f"[mobility] {kind} gamma={g}: {vals[0]:.5g} -> {vals[-1]:.5g} ({dt:.1f} s)",
                  file=sys.stderr, flush=True)
            del sim
        rows_ok = [r for r in rows if not r.get("unstable")]
        rec = {"runs": rows}
        if len(rows_ok) >= 2:
            xs = np.array([r["x"] for r in rows_ok])
            ys = np.array([r["mobility"] for r in rows_ok])
            slope, icpt = np.polyfit(xs, ys, 1)
            rec.update(fit_slope=float(slope), intercept=float(icpt))
            if spin:
                rec["gammaR_mesh"] = float(1.0 / (1000.0 * icpt)) if icpt > 0 else None
        out[kind] = rec
    line = {
        "metric": "single-cell mobilities at infinite coupling (Sec. III)",
        "config": {"workload": f"lone cell, periodic {n}^3 plasma at rest, T0=1.0 (nu=1/6), Delta=0, "
                               f"xi={tuple(base['xi'])}, M=10, I=1000; force {F} (gR=0.01), torque {T} (gT=0.01); "
                               f"{steps} steps per run; FP64 storage"},
        "paper_printed": {"frontal": 6.6, "side-wise": 10.3, "gammaR_mesh_short_axis": 1 / 44.0,
                          "gammaR_mesh_long_axis": 1 / 38.0},
        "results": out,
    }
    print(json.dumps(line), flush=True)


def shear_cell_config(alpha: float, storage: str = "f64", U: float = 0.02, n=(64, 42, 32)):
    """Wall-bounded shear cell: solid rows y = 0 and y = ny - 1 moving along x with -U and +U
    (shear rate 2U/(ny - 2)), periodic in x and z, T0 = 1 (nu = 1/6), gammaT = gammaR = 0.1, one
    cell of semi-axes (4, 4, 1.5) at the centre with its symmetry axis along the gradient y."""
    import numpy as np

    nx, ny, nz = n
    cfg = dict(nx=nx, ny=ny, nz=nz, periodic=(1, 0, 1), tau0=1.0, gammaT=0.1, gammaR=0.1,
               alpha=alpha, wall_u_lo=(-U, 0.0, 0.0), wall_u_hi=(U, 0.0, 0.0), storage=storage)
    from paper_1107_4889_amd import synth

    solid = synth.slab(nx, ny, nz)
    R = np.array([[nx / 2.0, (ny - 1) / 2.0, nz / 2.0]])
    # body axes as columns: n = x, t = -z, g = y (right-handed)
    Q = np.array([[1.0, 0.0, 0.0, 0.0, 0.0, 1.0, 0.0, -1.0, 0.0]])
    return cfg, solid, R, Q


def tank_treading(args):
    """Single cell in shear against the elongational torque factor alpha (Sec. II C; Sec. III,
    the tank-treading torque figure). The paper uses a Lees-Edwards shear field and reports the
    transition to a fixed orientation (tank treading) at alpha = 0.063 with an angle of about 40
    degrees, and 20-35 degrees in a bounded slab; this run uses the bounded slab of
    shear_cell_config. Per alpha: the orientation psi of the cell's long axis in the shear plane
    (angle to the flow direction x, from the symmetry axis g as atan2(-g_x, g_y)), unwrapped, and the
    z component of the elongational torque T^S, sampled every 250 steps after a warm-up that
    establishes the shear flow; tumbling if psi turns through more than 180 degrees, else the
    fixed angle (mean over the last quarter)."""
    import numpy as np
    import torch

    from paper_1107_4889_amd import lbrbc

    alphas = [a * args.tt_alpha_scale for a in (0.0, 0.02, 0.04, 0.063, 0.08, 0.1, 0.15)]
    warm, steps, every = args.tt_warmup, args.tt_steps, 250
    out = {}
    for alpha in alphas:
        cfg, solid, R, Q = shear_cell_config(alpha)
        cfg["inertia"] = (args.tt_inertia,) * 3
        sim = lbrbc.Simulation(cfg, solid, R=R, Q=Q)
        t0 = time.perf_counter()
        psi, ts, th, om = [], [], [], []
        try:
            sim.lb_step(warm)
            for k in range(steps // every):
                sim.lb_step(every)
                Qc = sim.rbc_get_state()[1][0].reshape(3, 3)
                g = Qc[:, 2]
                psi.append(float(np.arctan2(-g[0], g[1])))
                cp = sim.rbc_get_coupling()[0]
                ts.append(float(cp[9]))
                th.append(float(cp[15]))
                om.append(float(cp[6]))
        except lbrbc.LbError as e:
            # the flow itself went unstable (the torques' back-reaction on the plasma)
            out[str(alpha)] = {"regime": "unstable", "error": str(e), "samples_before": len(psi)}
            print(f"[tank-treading] alpha={alpha}: unstable after {len(psi)} samples", file=sys.stderr,
                  flush=True)
            del sim
            continue
        torch.cuda.synchronize()
        ps = np.degrees(np.unwrap(np.array(psi)))
        turned = float(ps.max() - ps.min())
        q = len(ps) // 4
        rec = {"psi_deg_samples": [round(x, 2) for x in ps[::4]],
               "TS_z_samples": [float(f"{x:.4g}") for x in ts[::4]],
               "T_hyd_z_samples": [float(f"{x:.4g}") for x in th[::4]],
               "vorticity_z_samples": [float(f"{x:.4g}") for x in om[::4]],
               "turned_deg": round(turned, 1), "seconds": round(time.perf_counter() - t0, 2),
               "flags": int(sim.lb_observe().flags)}
        if turned > 180.0:
            crossings = np.nonzero(np.diff(np.floor(ps / 180.0)) != 0)[0]
            period = (2 * every * float(np.mean(np.diff(crossings)))) if len(crossings) > 1 else None
            rec.update(regime="tumbling", period_steps=period)
        else:
            rec.update(regime="fixed orientation", psi_deg=round(float(np.mean(ps[-q:]) % 180.0), 2),
                       psi_spread_deg=round(float(np.ptp(ps[-q:])), 3))
        out[str(alpha)] = rec
        print(f"[tank-treading] alpha={alpha}: {rec['regime']}, turned {turned:.0f} deg "
              f"({rec['seconds']} s)", file=sys.stderr, flush=True)
        del sim
    cfg, _, _, _ = shear_cell_config(0.0)
    line = {
        "metric": "single-cell orientation in shear against the elongational torque factor alpha",
        "config": {"workload": (f"wall-bounded shear cell {cfg['nx']}x{cfg['ny']}x{cfg['nz']}, walls moving "
                                f"+/-{cfg['wall_u_hi'][0]} along x (shear rate "
                                f"{2 * cfg['wall_u_hi'][0] / (cfg['ny'] - 2):.2e}), T0=1, gammaT=gammaR=0.1, "
                                f"one cell (4, 4, 1.5) at the centre, FP64; {warm} warm-up + {steps} steps"),
                   "alpha_scale": args.tt_alpha_scale, "inertia": args.tt_inertia},
        "paper_printed": {"transition_alpha": 0.063, "fixed_angle_deg_lees_edwards": 40,
                          "fixed_angle_deg_bounded_slab": "20-35"},
        "results": out,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--storage", default="f32", choices=list(STORAGE_BYTES))
    ap.add_argument("--workload", default="tube256")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain device copy of 1 GiB (HBM counter calibration)")
    ap.add_argument("--serve", action="store_true",
                    help="serving mode: continuous batching of a seeded request stream")
    ap.add_argument("--requests", type=int, default=256)
    ap.add_argument("--rate", type=float, default=20.0)
    ap.add_argument("--chunk", type=int, default=50)
    ap.add_argument("--graphs", action="store_true", help="replay captured HIP graphs per chunk")
    ap.add_argument("--fused", action="store_true",
                    help="serving mode: one stream, each stage one launch over all resident requests")
    ap.add_argument("--observables", action="store_true",
                    help="flow rate, eta_app, eta_rel, u_z profile, WSS near steady state")
    ap.add_argument("--obs-steps", type=int, default=40000)
    ap.add_argument("--mobility", action="store_true",
                    help="single-cell translational and rotational mobilities vs the coupling rates")
    ap.add_argument("--mob-steps", type=int, default=20000)
    ap.add_argument("--mob-xi-scale", type=float, default=1.0,
                    help="mobility runs: shape-function radii (2, 2, 1) times this factor")
    ap.add_argument("--mob-kinds", default="frontal,side-wise,spin_short_axis,spin_long_axis")
    ap.add_argument("--no-serving", action="store_true",
                    help="default run: skip the request-stream leg (p50/p99 latency)")
    ap.add_argument("--budget-gib", type=float, default=64.0)
    ap.add_argument("--max-active", type=int, default=64)
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--tank-treading", action="store_true",
                    help="single cell in a shear cell: orientation against alpha")
    ap.add_argument("--tt-warmup", type=int, default=20000)
    ap.add_argument("--tt-steps", type=int, default=40000)
    ap.add_argument("--tt-inertia", type=float, default=1000.0,
                    help="principal moments of inertia of the cell (the paper's 1000 by default)")
    ap.add_argument("--tt-alpha-scale", type=float, default=1.0,
                    help="multiply the paper's alpha values (the balance of the elongational torque "
                         "against the rotational friction)")
    ap.add_argument("--cpu-baseline-only", action="store_true",
                    help="time only the oracle on the host, on the workload itself (--cpu-steps steps)")
    ap.add_argument("--cpu-steps", type=int, default=1)
    ap.add_argument("--layout", default="auto", choices=["auto", "dense", "compact"],
                    help="storage layout of the per-node planes (auto: compact for sparse geometries)")
    ap.add_argument("--precision", action="store_true",
                    help="reduced-precision storage study against FP64 on the same GPU")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported (the hot path runs "
              "on a single MI355X; a multi-GPU run would shard the lattice in z-slabs)",
              file=sys.stderr, flush=True)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        n = 1 << 30
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "launches": 5}), flush=True)
        return

    if args.serve:
        serve(args)
        return
    if args.precision:
        precision(args)
        return
    if args.observables:
        observables(args)
        return
    if args.mobility:
        mobility(args)
        return
    if args.tank_treading:
        tank_treading(args)
        return

    from paper_1107_4889_amd import lbrbc

    cfg, solid, pl, desc = workload(args.workload, args.storage)
    if args.cpu_baseline_only:
        n_fluid = int((solid == 0).sum())
        rec = cpu_baseline(cfg, solid, pl, n_fluid, hematocrit=None, steps=args.cpu_steps)
        print(json.dumps({"workload": desc, "cpu_baseline": rec}), flush=True)
        return
    cfg["layout"] = LAYOUTS[args.layout]
    print(f"[bench] {desc}", file=sys.stderr, flush=True)
    sim = lbrbc.Simulation(cfg, solid, R=pl.R, Q=pl.Q)
    arena = sim.bytes
    n_fluid = int((solid == 0).sum())
    layout = "compact" if sim.lb_observe().compact else "dense"

    sim.lb_step(args.warmup)
    torch.cuda.synchronize()
    sim.lb_sync()
    sim.lb_set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.lb_step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sc_ms, step_ev_ms = sim.lb_kernel_time()
    map_ms = sim.lb_map_time()
    sim.lb_set_timing(False)
    sim.lb_sync()
    obs = sim.lb_observe()
    print(f"[bench] timed {args.steps} steps in {t1 - t0:.3f} s; stream-collide {sc_ms:.4f} ms/launch",
          file=sys.stderr, flush=True)

    ms_per_step = (t1 - t0) * 1e3 / args.steps
    mlups = n_fluid * args.steps / (t1 - t0) / 1e6
    alg_bytes = n_fluid * 2 * 19 * STORAGE_BYTES[args.storage]
    achieved = alg_bytes / (sc_ms * 1e-3) / 1e9 if sc_ms > 0 else 0.0
    line = {
        "metric": "MLUPS & achieved HBM GB/s (LBM+RBC step); p50/p99 request latency",
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.storage,
        "compute_dtype": "f64" if args.storage == "f64" else "f32",
        "data": "synthetic",
        "config": {
            "workload": desc,
            "lattice": [cfg["nx"], cfg["ny"], cfg["nz"]],
            "n_fluid": n_fluid,
            "n_cells": int(len(pl.R)),
            "hematocrit": round(pl.hematocrit, 4),
            "storage": args.storage,
            "layout": layout,
            "stored_slots": int(obs.n_stored),
            "arena_gib": round(arena / 2 ** 30, 3),
            "parallelism": "single GPU",
        },
        "stream_collide": {
            "mlups": round(n_fluid / (sc_ms * 1e-3) / 1e6, 2) if sc_ms > 0 else None,
            "ms_per_launch": round(sc_ms, 5),
            "algorithmic_bytes_per_lu": 2 * 19 * STORAGE_BYTES[args.storage],
            "hbm_gbs_algorithmic": round(achieved, 1),
        },
        "map_pass": map_pass_record(args.storage, len(pl.R), map_ms),
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4),
            "traffic": measured_traffic(args.workload, args.storage, layout),
        },
        "observables": {"flow_rate": obs.flow_rate, "eta_app": obs.eta_app,
                        "wss_mean": obs.wss_mean, "mass": obs.mass},
    }
    del sim
    if not args.no_serving and args.workload in ("tube256", "tube128"):
        # the metric's request-latency part: the seeded request stream, fused launches
        print("[bench] serving the seeded request stream (fused launches)", file=sys.stderr,
              flush=True)
        sargs = argparse.Namespace(**{**vars(args), "fused": True, "graphs": False,
                                      "storage": "f32"})
        _, record, _, _ = run_serving(sargs)
        line["serving"] = record
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a sample of the same workload", file=sys.stderr,
              flush=True)
        H = {"tube256": 0.40, "tube128": 0.35}.get(args.workload)
        line["cpu_baseline"] = cpu_baseline(cfg, solid, pl, n_fluid, hematocrit=H)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
