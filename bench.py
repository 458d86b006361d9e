#!/usr/bin/env python
"""Throughput of the coupled phase-field / lattice-Boltzmann step on one MI355X.

Default workload: four spheres (R = 24) at the vertices of a regular tetrahedron around a central
liquid drop of 5 % liquid fraction, seeded 1e-3 perturbations of the phase fields, 30 degree
wetting, 256^3 D3Q19, tau = 1.1, FP32 populations, rigid-body motion and phase-field kinetics on;
beside it the same workload with FP16 population storage.  A step is the whole coupled step
(every kernel).  Inputs are resident in HBM before the timed region.  The fluid pass runs its
default tile of the precision (DEFAULT_TILES; --tile or --autotune choose another).

Prints one JSON line: MLUPS (all nodes x steps / s), the step's algorithmic fraction of HBM peak,
the dominant kernel's roofline (algorithmic bytes per launch over its mean launch time measured
with HIP events on the library's stream), and the FP64 CPU oracle timed on the host on a bounded
sample of the same workload.  --oracle-timing instead times the oracle alone on the three
single-grid workloads, on all host cores and on one thread.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PF+LBM step MLUPS & % HBM peak; fp16-store/batched vs fp32 at force err≤1e-3"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
KERNEL = "k_collide_stream"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_sha() -> str:
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1902_10432_amd", "csrc")
    for name in sorted(os.listdir(d)):
        with open(os.path.join(d, name), "rb") as f:
            h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


MASK_BYTES = 4  # one 32-bit cell word per node


# bytes per stored population and per pseudopotential value of each precision form
FORMS = {"fp64": (8, 8), "fp32": (4, 4), "fp16": (2, 4)}


def _bit_bytes(q: int) -> int:
    """D3Q27 keeps the solid-neighbour bits in a word of their own (D3Q19: in the cell word)."""
    return 4 if q == 27 else 0


def step_bytes_per_cell(pop: int, arith: int, q: int = 19) -> float:
    """Algorithmic bytes of one coupled step per node: q populations read and written, the cell
    word (and on D3Q27 the neighbour-bit word) read, the pseudopotential written (the force scan
    and the next step read it back at interface nodes only), and in the FP16-storage form the
    previous step's pseudopotential read (the reference density of the stored deviations).  The
    phase-field work on the tiles around the bodies is not counted."""
    return 2 * q * pop + arith + MASK_BYTES + _bit_bytes(q) + (arith if pop == 2 else 0)


def kernel_bytes(n_fluid: int, n_solid: int, pop: int, arith: int, q: int = 19) -> float:
    """Algorithmic bytes of one launch of the fluid pass: a fluid node reads and writes its q
    populations, reads its cell word (and on D3Q27 its neighbour-bit word; in the FP16-storage
    form its previous pseudopotential) and writes its pseudopotential; a solid node reads its cell
    word and writes its pseudopotential (the wetting value).  Neighbour values are re-reads of the
    same arrays and are not counted."""
    fluid = 2 * q * pop + arith + MASK_BYTES + _bit_bytes(q) + (arith if pop == 2 else 0)
    return n_fluid * fluid + n_solid * float(MASK_BYTES + arith)


def copy_calibration(mib: int, reps: int) -> int:
    """Plain device-to-device copies of a known size, for scaling the HBM byte counters of a
    profiler run (FETCH_SIZE / WRITE_SIZE per dispatch against the bytes actually moved)."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "dispatches": reps}), flush=True)
    return 0


def traffic_from_profile(workload: str, precision: str, sha: str, tile: dict):
    """HBM bytes per launch of the fluid pass from the stored counter summary, when it was taken
    on the same sources and tile shape (else None)."""
    path = os.path.join(ROOT, "profiles", f"{KERNEL}_{workload}_{precision}_hbm.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        prof = json.load(f)
    if prof.get("source_sha") != sha:
        return None  # the kernel changed since the counters were taken
    if prof.get("tile") != [tile.get("rows"), tile.get("planes")]:
        return None  # counted on another launch shape
    return prof.get("hbm_bytes_per_launch")


def cpu_baseline(w, seconds: float) -> dict:
    import oracle
    oracle.build(force=False)
    threads = oracle.Oracle.max_threads()
    o = oracle.Oracle(w.params, w.bodies, w.rho0, w.phi0)
    t0 = time.perf_counter()
    o.step(1)
    t1 = time.perf_counter() - t0
    n = max(1, int(seconds / max(t1, 1e-6)))
    t0 = time.perf_counter()
    o.step(n)
    dt = time.perf_counter() - t0
    return {"value": round(w.cells * n / dt / 1e6, 3), "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"{n} steps of the same {w.shape[2]}x{w.shape[1]}x{w.shape[0]} workload in FP64 "
                      f"after 1 warm-up step ({dt:.1f} s)"}


def oracle_timing() -> int:
    """The FP64 oracle on the host: MLUPS on all cores (OpenMP threads) and on one thread, for the
    32^3 plates bridge (200 steps), the 128^3 two-sphere bridge and the 256^3 four-sphere workload
    (short slices after one untimed warm-up step, which also touches the oracle's memory).  One
    JSON line per run."""
    import platform

    import oracle
    from pflbm_inputs import plates_bridge, tetrahedron_drop, two_spheres_bridge
    oracle.build(force=False)
    cores = oracle.Oracle.max_threads()
    cpu = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as f:
            cpu = next(l.split(":", 1)[1].strip() for l in f if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    plan = [("plates_bridge", plates_bridge, {cores: 200, 1: 200}),
            ("two_spheres_bridge", two_spheres_bridge, {cores: 10, 1: 2}),
            ("tetrahedron_drop", tetrahedron_drop, {cores: 4, 1: 1})]
    for name, make, runs in plan:
        w = make()
        for threads, steps in runs.items():
            oracle.Oracle.set_threads(threads)
            o = oracle.Oracle(w.params, w.bodies, w.rho0, w.phi0)
            o.step(1)
            t0 = time.perf_counter()
            o.step(steps)
            dt = time.perf_counter() - t0
            del o
            rec = {"oracle_timing": name, "shape": list(w.shape), "threads": threads, "steps": steps,
                   "seconds": round(dt, 3), "MLUPS": round(w.cells * steps / dt / 1e6, 4), "host_cpu": cpu,
                   "host_threads_available": cores}
            print(json.dumps(rec), flush=True)
        oracle.Oracle.set_threads(cores)
    return 0


def force_errors(ws, hist, hist64, steps: int) -> dict:
    """Per-instance force error of one sweep against its FP64 twin: |F - F_fp64| over
    max(|F_fp64|, pi sigma R_min), on the mean of the last 500 steps and per step over the first
    200; max, median, the count above 1e-3 and the worst instances."""
    sigma, window, early = 3.3e-2, min(500, steps), min(200, steps)
    late, first = [], []
    for w, h, h64 in zip(ws, hist, hist64):
        scale_r = math.pi * sigma * min(w.meta["radii"])
        f, f64 = h[-window:, :, :3].mean(axis=0), h64[-window:, :, :3].mean(axis=0)
        late.append(float(np.abs(f - f64).max() / max(np.abs(f64).max(), scale_r)))
        d = np.abs(h[:early, :, :3] - h64[:early, :, :3]).max(axis=(1, 2))
        sc = np.maximum(np.abs(h64[:early, :, :3]).max(axis=(1, 2)), scale_r)
        first.append(float((d / sc).max()))

    def stats(e):
        worst = np.argsort(e)[::-1][:3]
        return {"max": float(f"{max(e):.3g}"), "median": float(f"{np.median(e):.3g}"),
                "over_1e-3": int(sum(x > 1e-3 for x in e)),
                "worst": [[int(k), float(f"{e[k]:.3g}")] for k in worst]}

    return {f"mean_of_last_{window}_steps": stats(late), f"per_step_first_{early}_steps": stats(first)}


def batched_sweep(args) -> int:
    """The sweep of uneven two-sphere bridges (grids 48^3..128^3, seeded; config 4), stepped three
    ways over the same number of steps: every instance alone, one after the other; all instances
    by pf_lbm_step_batch (launches interleaved over the instances' streams); all instances as one
    captured HIP graph (pf_lbm_batch_*).  Each instance's fluid-pass tile is autotuned first
    (unless --no-autotune).  The same sweep in FP64 gives each instance's force error, as
    |F - F_fp64| over max(|F_fp64|, pi sigma R_min), averaged over the last 500 steps (the
    instantaneous force carries the period-2 staggered mode) and per step over the first 200.
    The error is taken twice: with the spheres held at their gap (the field solve of the force
    table: precision alone separates the two runs) and with the spheres moving (node conversions
    a step apart in the two precisions let the trajectories part, so the late window measures
    that divergence, not the precision of one solve).  Prints one JSON line (MLUPS over all
    instances' nodes)."""
    import torch

    from paper_1902_10432_amd.simulation import Batch, Simulation, step_batch
    from pflbm_inputs import bridge_sweep

    steps = args.batched_steps
    t0 = time.perf_counter()
    ws = bridge_sweep(args.batched, seed=0)
    cells = sum(w.cells for w in ws)
    log(f"{len(ws)} instances, {cells / 1e6:.1f} M nodes, generated in {time.perf_counter() - t0:.1f} s")

    def make(prec):
        return [Simulation(w.params, w.bodies, w.rho0, w.phi0, precision=prec) for w in ws]

    sims = make(args.precision)
    tiles = None
    if not args.no_autotune:
        tiles = [s.autotune(4) for s in sims]
        log("autotuned tiles: " + json.dumps(sorted({(t["tile_rows"], t["chunk_planes"]) for t in tiles})))
    graph = Batch(sims, graph_steps=args.graph_steps)
    # warm-up of every path (each captures its graphs)
    step_batch(sims, 2)
    graph.step(args.graph_steps)
    for s in sims:
        s.step(32)
    torch.cuda.synchronize()
    # sequential: one instance at a time
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    seq_ms = 0.0
    for s in sims:
        ev[0].record(s.stream)
        s.step(steps)
        ev[1].record(s.stream)
        torch.cuda.synchronize()
        seq_ms += ev[0].elapsed_time(ev[1])

    def timed(fn):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t1) * 1e3

    rr_ms = timed(lambda: step_batch(sims, steps))
    gr_ms = timed(lambda: graph.step(steps))
    rate = lambda ms: cells * steps / (ms / 1e3) / 1e6
    seq, rr, gr = rate(seq_ms), rate(rr_ms), rate(gr_ms)
    ok = all(np.isfinite(s.force_history(steps)).all() for s in sims)
    pop, arith = FORMS[args.precision]
    achieved = gr * 1e6 * step_bytes_per_cell(pop, arith) / 1e9
    out = {"metric": "batched uneven bridge sweep MLUPS (one captured graph)", "value": round(gr, 2),
           "unit": "MLUPS", "n_gpus": 1, "steps": steps, "higher_is_better": True,
           "sequential": round(seq, 2), "round_robin_streams": round(rr, 2),
           "vs_sequential": round(gr / seq, 3), "round_robin_vs_sequential": round(rr / seq, 3),
           "instances": len(ws), "cells": cells, "graph_steps": args.graph_steps, "precision": args.precision,
           "tiles": None if tiles is None else sorted({f"{t['tile_rows']}x{t['chunk_planes']}" for t in tiles}),
           "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                        "kernel": "whole step, all instances (kernels of different instances overlap)",
                        "bytes_per_cell_step": step_bytes_per_cell(pop, arith)},
           "finite_force_histories": bool(ok), "data": "synthetic",
           "config": {"workload": f"bridge_sweep seed 0: {len(ws)} two-sphere instances, grids 48..128 per axis",
                      "cells": cells}}
    if not args.no_fp64_check and args.precision != "fp64":
        # fresh sweeps of `steps` steps each through the batch graph, in the bench's precision and
        # in FP64 (default tiles: the arithmetic does not depend on them)
        graph.close()
        for s in sims:
            s.close()
        del graph, sims
        torch.cuda.empty_cache()
        out["force_error_vs_fp64"] = {}
        for label, fixed in (("spheres_fixed", True), ("spheres_moving", False)):
            wk = bridge_sweep(args.batched, seed=0, fixed=fixed)
            hists = {}
            for prec in (args.precision, "fp64"):
                run = [Simulation(w.params, w.bodies, w.rho0, w.phi0, precision=prec) for w in wk]
                bg = Batch(run, graph_steps=args.graph_steps)
                bg.step(steps)
                hists[prec] = [r.force_history(steps) for r in run]
                bg.close()
                for r in run:
                    r.close()
                del bg, run
                torch.cuda.empty_cache()
            out["force_error_vs_fp64"][label] = force_errors(wk, hists[args.precision], hists["fp64"], steps)
            log(f"force error vs fp64, {label}: {json.dumps(out['force_error_vs_fp64'][label])}")
        out["force_error_vs_fp64"]["definition"] = (
            f"|F - F_fp64| / max(|F_fp64|, pi sigma R_min) per instance over {steps} steps")
    print(json.dumps(out), flush=True)
    return 0


def mlp_forward_rate(batch: int = 65536, reps: int = 50) -> dict:
    """Forward throughput of the 4 -> 128 x 4 -> 1 network on one batch, timed with HIP events on
    the network's stream."""
    import ctypes as C

    import torch

    from paper_1902_10432_amd import surrogate as S

    net = S.Surrogate(4, 128, 4, max_batch=batch, seed=0)
    x = torch.randn(batch, 4, device="cuda")
    y = torch.empty(batch, device="cuda")
    lib = S._load()
    torch.cuda.synchronize()
    for _ in range(5):
        lib.pf_mlp_forward(net._h, C.c_void_p(x.data_ptr()), batch, C.c_void_p(y.data_ptr()))
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(net.stream)
    for _ in range(reps):
        lib.pf_mlp_forward(net._h, C.c_void_p(x.data_ptr()), batch, C.c_void_p(y.data_ptr()))
    ev[1].record(net.stream)
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / reps
    flops = 2.0 * batch * (4 * 128 + 3 * 128 * 128 + 128)
    tf = flops / ms / 1e9
    # one fused launch: only the inputs and outputs cross HBM, so the products bound it
    return {"batch": batch, "ms": round(ms, 4), "tflops": round(tf, 2), "rows_per_s": round(batch / ms * 1e3, 1),
            "roofline": {"bound": "mfma", "achieved": round(tf, 2), "peak": 2500.0, "unit": "TFLOP/s",
                         "frac": round(tf / 2500.0, 4), "traffic": None}}


def surrogate_run(args) -> int:
    """The learned bridge-force surrogate end to end: training data from the two-sphere bridge
    sweep (64 bridges per seed, fixed spheres, 2000 steps), training on the GPU, and the
    1000-sphere rigid-body run at 3 % liquid in which 32 bridges are re-solved at 96^3 every 100
    steps as error judge and fallback.  Prints one JSON line: the cost ratio per bridge force
    (field solve / network), the network's error on the judged bridges, and the network's forward
    throughput."""
    from paper_1902_10432_amd import deploy as Dp

    t0 = time.perf_counter()
    X, y, st = Dp.training_set(64, seeds=tuple(range(args.surrogate_seeds)), log=log)
    t_data = time.perf_counter() - t0
    norm = Dp.normalisation(X, y)
    net, rep = Dp.train(X, y, norm, log=log)
    s = Dp.deploy(net, norm, steps=args.surrogate_steps, train_data=(X, y), refine_steps=args.surrogate_refine,
                  log=log)
    fwd = mlp_forward_rate()
    rounds = s.pop("rounds")
    out = {"metric": "surrogate bridge force: GPU time per bridge, PF-LBM re-solve / network",
           "value": round(s["speedup_per_bridge"], 1), "unit": "x", "higher_is_better": True,
           "judged_rmse": round(s["rmse"], 5), "judged_field_rms": round(s["rms_field"], 5),
           "judged_rel_rmse": round(s["rmse"] / s["rms_field"], 4), "judged": s["judged"], "fallbacks": s["fallbacks"],
           "judged_rel_rmse_first_half": round(s["rel_rmse_first_half"], 4),
           "judged_rel_rmse_second_half": round(s["rel_rmse_second_half"], 4), "refine_steps": s["refine_steps"],
           "seconds_per_bridge_network": s["seconds_per_bridge_network"],
           "seconds_per_bridge_field": s["seconds_per_bridge_field"],
           "training": {k: (round(v, 6) if isinstance(v, float) else v) for k, v in rep.items()},
           "training_data_seconds": round(t_data, 1), "training_bridges": int(len(y)),
           "run": {k: v for k, v in s.items() if k not in ("seconds_per_bridge_network", "seconds_per_bridge_field")},
           "bridges_per_round": [r.get("bridges") for r in rounds], "network_forward": fwd,
           "dtype": "bf16-mfma/f32", "data": "synthetic",
           "config": {"workload": "1000 spheres, radii 12..18, 3% liquid, theta 30, 96^3 re-solves",
                      "network": "4 -> 128 x 4 -> 1 SiLU"}}
    print(json.dumps(out), flush=True)
    return 0


# Tile of the fluid pass timed by default on the 256^3 workload, per population storage: the
# shapes the autotuner picked most often there (its candidates differ by a few per cent, within
# run-to-run noise), fixed so that runs and the profiler's counters describe the same launch.
# Other workloads run the library's default shape.
DEFAULT_TILES = {"fp32": (8, 8), "fp16": (4, 8), "fp64": (4, 8)}


def tune_tile(sim, args, precision: str, workload: str) -> dict:
    """Tile shape of the fluid pass: given (--tile), the autotuner's choice (--autotune; candidates
    timed on the live run before the warm-up, the state advancing like warm-up steps), the default
    of the precision on the 256^3 workload, else the library's default."""
    if args.autotune:
        t = sim.autotune(5)
        log(f"autotuned tile: {t}")
        return {"rows": t["tile_rows"], "planes": t["chunk_planes"], "chosen_by": "autotune"}
    if not args.tile and workload != "tetrahedron_drop":
        return {"chosen_by": "library default"}
    rows, planes = (int(v) for v in args.tile.split(",")) if args.tile else DEFAULT_TILES[precision]
    sim.set_tile(rows, planes)
    return {"rows": rows, "planes": planes, "chosen_by": "given" if args.tile else "default"}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="tetrahedron_drop")
    ap.add_argument("--n", type=int, default=None, help="grid size override (cubic)")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64", "fp16"])
    ap.add_argument("--lattice", type=int, default=19, choices=[19, 27], help="velocity set (27: Sec. 3.2.1)")
    ap.add_argument("--tau", type=float, default=None,
                    help="BGK relaxation time (workload default: 1.1 for tetrahedron_drop, else 1.0)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the FP16-storage comparison")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run plain copies of MIB MiB (profiler counter calibration)")
    ap.add_argument("--batched", type=int, default=0, metavar="N",
                    help="only the batched sweep of N uneven two-sphere instances against sequential runs")
    ap.add_argument("--batched-steps", type=int, default=2000, help="steps of each path of the batched sweep")
    ap.add_argument("--graph-steps", type=int, default=4, help="steps per replay of the batch graph (even)")
    ap.add_argument("--no-fp64-check", action="store_true", help="skip the FP64 twin of the batched sweep")
    ap.add_argument("--surrogate", action="store_true",
                    help="only the bridge-force surrogate: sweep, GPU training, 1000-sphere run with re-solves")
    ap.add_argument("--surrogate-seeds", type=int, default=4, help="64-bridge sweeps of training data")
    ap.add_argument("--surrogate-steps", type=int, default=1000, help="rigid-body steps (judged every 100)")
    ap.add_argument("--surrogate-refine", type=int, default=100,
                    help="Adam steps on sweep + judged bridges after each judgement (0: none)")
    ap.add_argument("--tile", default=None, metavar="ROWS,PLANES",
                    help="tile shape of the fluid pass (default: the autotuner's choice)")
    ap.add_argument("--autotune", action="store_true",
                    help="single-grid runs: time the tile candidates and keep the fastest instead of the default tile")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batched sweep: keep the library's default tile shape of every instance instead of autotuning it")
    ap.add_argument("--oracle-timing", action="store_true",
                    help="only the FP64 CPU oracle: all host cores and one thread on each single-grid workload")
    args = ap.parse_args()
    if args.oracle_timing:
        return oracle_timing()
    if args.copy_calibration:
        return copy_calibration(args.copy_calibration, 5)
    if args.batched:
        return batched_sweep(args)
    if args.surrogate:
        return surrogate_run(args)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: there is no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1902_10432_amd.simulation import Simulation
    from pflbm_inputs import make_workload

    kw = {"n": args.n} if args.n else {}
    if args.lattice != 19:
        kw["lattice"] = args.lattice
    if args.tau is not None:
        kw["tau"] = args.tau
    w = make_workload(args.workload, **kw)
    q = args.lattice
    pop, arith = FORMS[args.precision]
    log(f"workload {w.name} {w.shape} bodies={len(w.bodies)} {args.precision}")
    sim = Simulation(w.params, w.bodies, w.rho0, w.phi0, precision=args.precision)
    stream = sim.stream
    tile = tune_tile(sim, args, args.precision, w.name)

    sim.step(args.warmup)
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(stream)
    sim.step(args.steps)
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(end)
    ms_per_step = ms / args.steps
    mlups = w.cells * args.steps / (ms / 1e3) / 1e6
    pct_step = mlups * 1e6 * step_bytes_per_cell(pop, arith, q) / (HBM_PEAK_GBS * 1e9)
    log(f"timed {args.steps} steps: {ms:.2f} ms (wall {wall * 1e3:.2f} ms), {mlups:.1f} MLUPS")

    # dominant kernel: mean launch time from events recorded around it on the library's stream
    sim.timing(True)
    sim.step(args.steps)
    tm = sim.timing(False)
    solid = sim.field("solid").sum().item()
    n_solid = int(solid)
    n_fluid = w.cells - n_solid
    kb = kernel_bytes(n_fluid, n_solid, pop, arith, q)
    achieved = kb / (tm["kernel_ms"] / 1e3) / 1e9
    sha = source_sha()
    traffic = traffic_from_profile(w.name, args.precision, sha, tile) if q == 19 else None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": KERNEL,
                "kernel_ms": round(tm["kernel_ms"], 5), "bytes_per_launch": kb}
    b = sim.bodies()
    ok = all(math.isfinite(v) for v in np.asarray(b["F"]).ravel())
    d = sim.diag()

    # the FP16-storage form on the same workload, timed the same way (its force error against
    # the FP64 oracle is checked by the GPU tests: <= 1e-3 relative)
    forms = None
    if args.precision == "fp32" and not args.no_forms:
        del sim
        torch.cuda.empty_cache()
        h = Simulation(w.params, w.bodies, w.rho0, w.phi0, precision="fp16")
        htile = tune_tile(h, args, "fp16", w.name)
        h.step(args.warmup)
        torch.cuda.synchronize()
        s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s0.record(h.stream)
        h.step(args.steps)
        s1.record(h.stream)
        torch.cuda.synchronize()
        hms = s0.elapsed_time(s1)
        hm = w.cells * args.steps / (hms / 1e3) / 1e6
        forms = {"fp16_store": {"value": round(hm, 2), "unit": "MLUPS", "ms_per_step": round(hms / args.steps, 5),
                                "vs_fp32": round(hm / mlups, 3), "tile": htile,
                                "pct_hbm_step_algorithmic": round(hm * 1e6 * step_bytes_per_cell(*FORMS["fp16"], q)
                                                                  / (HBM_PEAK_GBS * 1e9), 4)}}
        log(f"fp16 storage: {hm:.1f} MLUPS ({hm / mlups:.2f}x fp32)")
        del h

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, args.cpu_seconds)

    out = {
        "metric": METRIC, "value": round(mlups, 2), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": {"fp64": "f64", "fp32": "f32", "fp16": "f16-store/f32"}[args.precision], "data": "synthetic",
        "config": {"workload": f"{w.name} {w.shape[2]}x{w.shape[1]}x{w.shape[0]} D3Q{q}, {len(w.bodies)} bodies, "
                               f"motion+kinetics on", "cells": w.cells, "precision": args.precision},
        "pct_hbm_step_algorithmic": round(pct_step, 4),
        "tile": tile,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "forms": forms,
        "finite_forces": ok,
        "node_conversions": {"steps": d["step"], "fluid_to_solid": d["n_f2s"], "solid_to_fluid": d["n_s2f"]},
        "source_sha": sha,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
