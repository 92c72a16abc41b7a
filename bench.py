"""Benchmark of the per-step particle update (gather + push + deposit).

Workload: 128^3 periodic box, turbulent E and B (|k|^-5/3, dB/B0 = 0.5,
E = -v x B), 2^24 charged particles (q/m = 1, weight 1) placed uniformly with
Maxwellian velocities (sigma = 0.05 c), TSC weights, dt = 0.05; every step
gathers E and B, pushes (relativistic Boris) and deposits rho, J and F at the
new positions.  The headline path is the float32 + cell-offset form with the
run-based LDS kernel; its sort (particles in run order: tile, run inside the
cell, cell) runs inside the timed loop at the tuned cadence.  The plain float64 path runs on the same inputs for the
speedup, and the run-based float64 path and the tiled float32 path beside it.

Each timed step: zero the moment grids, then one fused gather/push/deposit
launch (a replayed hipGraph) bracketed by HIP events on the library's stream;
sorts are bracketed separately.  Prints ONE JSON line.  Inputs are generated
on the host and are resident in HBM before the timed region starts.
"""

from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def kernel_name(cfg, B):
    """Name of the dominant kernel of a float32 configuration: the fused
    gather -> push -> deposit kernel for TSC, 3D, charged particles, channels
    rho + J + F (compile-time tile shape 8^3 or 8x8x4 when the tile is one)."""
    tile = tuple(cfg["tile"])
    if cfg["algo"] == B.PL_ALGO_RUNS:
        # compile-time field halo: two cells where the LDS allows (float32, rho+J+F)
        ts = {(8, 8, 8): 1, (8, 8, 4): 2}.get(tile, 0)
        return f"pl::k_runs<1, 2, 3, 0, {2 if ts else 0}, {ts}, {1 if ts else 0}>"
    ts = {(8, 8, 8): 1, (8, 8, 4): 2}.get(tile, 0)
    return f"pl::k_step<1, 2, 3, true, 0, {ts}, {1 if ts else 0}>"

TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_runs_f32_turbulent128_traffic.json")
INSTR_FILE = os.path.join(ROOT, "profiles", "k_runs_f32_turbulent128_instructions.json")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def algorithmic_bytes(prec, npart, cells, weights=True, fields=6, channels=7):
    """Bytes the method must move per step: each particle read and written
    once, each touched field cell read once, each touched moment cell
    read-modify-written once (every cell is touched at 8 particles/cell)."""
    if prec == "f32":
        pread = 4 + 12 + 12 + (4 if weights else 0)      # cell, offsets, u, w
        pwrite = 4 + 12 + 12
    else:
        pread = 24 + 24 + (8 if weights else 0)           # x, u, w
        pwrite = 24 + 24
    return npart * (pread + pwrite) + cells * (8 * fields + 2 * 8 * channels)


def src_digest():
    from paper_2602_23434_amd import profiling
    return profiling.src_digest()


def timed_loop(run, steps, every, graph, torch, B):
    """`steps` steps with a sort every `every` steps (0: never); returns
    (loop ms, per-launch kernel ms list, per-sort ms list)."""
    ev = lambda: torch.cuda.Event(enable_timing=True)
    flags = B.PL_FUSE_DEPOSIT | (B.PL_GRAPH if graph else 0)
    kpairs, spairs = [], []
    t0, t1 = ev(), ev()
    t0.record(run.stream)
    for s in range(steps):
        if every and s % every == 0:
            a, b = ev(), ev()
            a.record(run.stream)
            run.sort()
            b.record(run.stream)
            spairs.append((a, b))
        run.zero_moments()
        a, b = ev(), ev()
        a.record(run.stream)
        run.step(flags=flags)
        b.record(run.stream)
        kpairs.append((a, b))
    t1.record(run.stream)
    t1.synchronize()
    st = run.sync()
    if st != B.PL_OK:
        raise RuntimeError(f"device reported status {st}")
    return (t0.elapsed_time(t1), [a.elapsed_time(b) for a, b in kpairs], [a.elapsed_time(b) for a, b in spairs])


def time_path(run, steps, warmup, reps, every, graph, torch, B):
    if warmup:
        timed_loop(run, warmup, every, graph, torch, B)
    loops, kern, sorts = [], [], []
    for _ in range(reps):
        ms, k, s = timed_loop(run, steps, every, graph, torch, B)
        loops.append(ms / steps)
        kern.extend(k)
        sorts.extend(s)
    return {"ms_per_step": statistics.median(loops), "ms_min": min(loops), "ms_max": max(loops),
            "kernel_ms": sum(kern) / len(kern), "sort_ms": (sum(sorts) / len(sorts)) if sorts else 0.0}


def time_workload(wl, cfg, steps, every, torch, B, driver):
    """Whole-step time of a multi-item workload (all items in one call per
    step: one persistent launch per species kind), sort every `every` steps."""
    run = driver.Run(wl, **cfg)
    try:
        run.sort()
        run.sync()
        total = sum(it.particles.n for it in wl.items)
        timed_loop(run, 2, every, True, torch, B)
        ms, kern, sorts = timed_loop(run, steps, every, True, torch, B)
        stats = B.pl_part_stats(run.ctx)
        return {"value": total * steps / (ms * 1e-3), "unit": "particle-updates/s", "particles": total,
                "ms_per_step": ms / steps, "kernel_ms": sum(kern) / len(kern),
                "sort_ms": (sum(sorts) / len(sorts)) if sorts else 0.0, "sort_every": every, "steps": steps,
                "run_kernel_launches": stats[4], "tiled_fallback_groups": stats[5]}
    finally:
        run.close()


def extra_workloads(head_cfg, torch, B, driver, inputs):
    """The clumped 256^3 box (2^26 particles, half in 32 Gaussian clumps, sort
    every 4 steps) and the batched workload (192^3 box with charged, dust and
    tracer species plus 16 independent 64^3 boxes), both in the float32 form
    with the headline's kernel configuration, 20 steps each."""
    out = {}
    cfg = {k: v for k, v in head_cfg.items() if k != "sort_every"}
    t0 = time.perf_counter()
    wl = inputs.clumped_box()
    log(f"[bench] clumped 256^3 inputs in {time.perf_counter() - t0:.1f} s")
    out["clumped_256"] = time_workload(wl, cfg, 20, 4, torch, B, driver)
    log(f"[bench] clumped 256^3: {out['clumped_256']}")
    del wl
    torch.cuda.empty_cache()
    t0 = time.perf_counter()
    wl = inputs.batched()
    log(f"[bench] batched inputs in {time.perf_counter() - t0:.1f} s")
    bcfg = dict(cfg)
    bcfg["channels"] = None
    out["batched_192"] = time_workload(wl, bcfg, 20, head_cfg["sort_every"], torch, B, driver)
    log(f"[bench] batched: {out['batched_192']}")
    del wl
    torch.cuda.empty_cache()
    return out


def cpu_baseline(wl, target_s=15.0):
    """The float64 oracle on the host cores, on a bounded sample of the same
    workload: the first `ns` particles (same fields, grid, dt), whole steps of
    gather + push + deposit."""
    import numpy as np

    import oracle
    it = wl.items[0].particles
    box = wl.boxes[0]
    ns = 1 << 20
    x = np.ascontiguousarray(it.x[:, :ns])
    u = np.ascontiguousarray(it.u[:, :ns])
    w = np.ascontiguousarray(it.w[:ns])
    steps = 0
    t_total = 0.0
    while t_total < target_s and steps < 50:
        mom = oracle.new_moments(box.n, oracle.LORENTZ)
        mom["eng"] = None
        t0 = time.perf_counter()
        oracle.step(3, box.n, oracle.TSC, (oracle.LORENTZ, 1.0, 1.0, 0.0), x, u, w, box.fields, wl.dt,
                    moments=mom)
        t_total += time.perf_counter() - t0
        steps += 1
    return {"value": ns * steps / t_total, "unit": "particle-updates/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"first {ns} of the 2^24 particles, {steps} full steps (gather+push+deposit of rho,J,F) "
                      f"on the 128^3 turbulent fields, {t_total:.1f} s of CPU time"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=32)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--sort-every", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-tiled", action="store_true")
    ap.add_argument("--extra", action="store_true", help="also time the clumped and batched workloads")
    ap.add_argument("--eager", action="store_true", help="launch steps without hipGraph replay")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library runs on one GPU per process and has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2602_23434_amd import benchcfg as BC
    from paper_2602_23434_amd import binding as B
    from paper_2602_23434_amd import driver, inputs

    B.lib()
    head_cfg, f64_cfg = BC.headline(), BC.f64_sorted()
    every = head_cfg["sort_every"] if args.sort_every is None else args.sort_every
    every64 = f64_cfg["sort_every"] if args.sort_every is None else args.sort_every
    t0 = time.perf_counter()
    wl = inputs.turbulent_box(n=BC.TURB_N, npart=BC.TURB_NP, steps=args.steps)
    log(f"[bench] inputs generated in {time.perf_counter() - t0:.1f} s")
    npart = BC.TURB_NP
    cells = BC.TURB_N ** 3

    results = {}
    paths = [("f32_runs", BC.run_kwargs(head_cfg), every, args.reps)]
    if not args.no_tiled:
        paths.append(("f32_tiled", BC.F32_TILED, every, args.reps))
    if not args.no_fp64:
        paths.append(("f64_plain", BC.F64_PLAIN, 0, 1))
        paths.append(("f64_runs", BC.run_kwargs(f64_cfg), every64, args.reps))
    for name, cfg, ev_every, reps in paths:
        log(f"[bench] path {name}: setup")
        run = driver.Run(wl, **cfg)
        if cfg["algo"] != B.PL_ALGO_PLAIN:
            run.sort()
        run.sync()
        log(f"[bench] path {name}: {args.warmup} warmup + {reps} x {args.steps} timed steps, sort every {ev_every}")
        r = time_path(run, args.steps, args.warmup, reps, ev_every, not args.eager, torch, B)
        prec = "f32" if cfg["prec"] == B.PL_F32_OFFSET else "f64"
        r["alg_bytes"] = algorithmic_bytes(prec, npart, cells)
        r["updates_per_s"] = npart / (r["ms_per_step"] * 1e-3)
        r["stats"] = B.pl_part_stats(run.ctx)
        results[name] = r
        log(f"[bench] path {name}: {r['ms_per_step']:.3f} ms/step (min {r['ms_min']:.3f} max {r['ms_max']:.3f}), "
            f"kernel {r['kernel_ms']:.3f} ms, sort {r['sort_ms']:.3f} ms, {r['updates_per_s']:.3e} updates/s, "
            f"{r['alg_bytes'] / (r['kernel_ms'] * 1e-3) / 1e9:.0f} GB/s algorithmic, stats {r['stats']}")
        run.close()
        del run
        torch.cuda.empty_cache()

    head = results["f32_runs"]
    if head_cfg["algo"] == B.PL_ALGO_RUNS and (head["stats"][4] == 0 or head["stats"][5] != 0):
        raise RuntimeError(f"the run-based kernel did not take the timed steps: stats {head['stats']}")
    achieved = head["alg_bytes"] / (head["kernel_ms"] * 1e-3) / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as fh:
            tr = json.load(fh)
        from paper_2602_23434_amd import profiling
        if tr.get("src_digest") == src_digest() and tr.get("config") == profiling.workload_config():
            traffic = tr.get("bytes_per_launch")
    # secondary ceilings (VALU issue, LDS) from the committed instruction counts
    # of the same kernel source, measured live against this run's kernel time
    secondary = None
    if os.path.exists(INSTR_FILE):
        with open(INSTR_FILE) as fh:
            ins = json.load(fh)
        from paper_2602_23434_amd import profiling
        if ins.get("src_digest") == src_digest() and ins.get("config") == profiling.workload_config():
            secondary = {
                "valu": {"floor_ms": ins["valu_floor_ms"], "frac": ins["valu_floor_ms"] / head["kernel_ms"],
                         "lane_insts_per_update": ins["valu_wave_insts"] * 64 / npart},
                "lds": {"wave_insts_per_64_updates": ins["lds_wave_insts"] * 64 / npart,
                        "bank_conflict_ms_per_cu": ins["lds_conflict_ms_per_cu"],
                        "bank_conflict_frac": ins["lds_conflict_ms_per_cu"] / head["kernel_ms"]},
            }
    sort_name = {B.PL_KEY_TILE: "tile", B.PL_KEY_TILE_CELL: "tile+cell", B.PL_KEY_TILE_RANK: "tile+rank",
                 B.PL_KEY_TILE_RUN: "run-order"}.get(head_cfg["key_mode"], str(head_cfg["key_mode"]))
    out = {
        "metric": "particle updates/sec (gather+push+deposit) and % HBM roofline, FP32 vs FP64 path",
        "value": head["updates_per_s"],
        "unit": "particle-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "turbulent 128^3 periodic box, 2^24 charged particles (8/cell), TSC, "
                               f"float32 + cell-offset form, run-based LDS kernel, {sort_name} sort every "
                               f"{every} steps inside the timed loop, deposit rho+J+F (inputs of the float64 "
                               "128^3 configuration)",
                   "grid": [BC.TURB_N] * 3, "particles": npart, "dt": 0.05, "shape": "tsc",
                   "tile": list(head_cfg["tile"]), "block": head_cfg["block"], "sort_key": sort_name,
                   "sort_every": every, "graph": not args.eager, "reps": args.reps,
                   "ms_per_step_min": head["ms_min"], "ms_per_step_max": head["ms_max"],
                   "sort_ms": head["sort_ms"], "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": kernel_name(head_cfg, B),
                     "kernel_ms": head["kernel_ms"], "alg_bytes_per_launch": head["alg_bytes"]},
        "secondary_ceilings": secondary,
    }
    for name, key in (("f32_tiled", "fp32_tiled"), ("f64_plain", "fp64_plain"), ("f64_runs", "fp64_runs")):
        if name in results:
            r = results[name]
            out[key] = {"value": r["updates_per_s"], "ms_per_step": r["ms_per_step"], "kernel_ms": r["kernel_ms"],
                        "sort_ms": r["sort_ms"],
                        "achieved_GBs": r["alg_bytes"] / (r["kernel_ms"] * 1e-3) / 1e9}
    if "f64_plain" in results:
        out["speedup_f32_over_f64_plain"] = head["updates_per_s"] / results["f64_plain"]["updates_per_s"]
    if "f64_runs" in results:
        out["speedup_f32_over_f64_runs"] = head["updates_per_s"] / results["f64_runs"]["updates_per_s"]
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle on host cores)")
        out["cpu_baseline"] = cpu_baseline(wl)
    if args.extra:
        del wl
        out["extra_workloads"] = extra_workloads(head_cfg, torch, B, driver, inputs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
