"""Benchmark of the per-step particle update (gather + push + deposit).

Workload: 128^3 periodic box, turbulent E and B (|k|^-5/3, dB/B0 = 0.5,
E = -v x B), 2^24 charged particles (q/m = 1, weight 1) placed uniformly with
Maxwellian velocities (sigma = 0.05 c), TSC weights, dt = 0.05; every step
gathers E and B, pushes (relativistic Boris) and deposits rho, J and F at the
new positions.  The headline path is the float32 + cell-offset form with
LDS-tiled kernels (one initial cell-tile sort as setup, outside the timed
region); the plain float64 path runs on the same inputs for the speedup.

Prints ONE JSON line.  Inputs are generated on the host, moved to HBM, and
are resident before the timed region starts.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# the dominant kernel: fused gather -> push -> deposit, float32 form, TSC, 3D,
# tiled, charged particles
KERNEL = "pl::k_step<1, 2, 3, true, 0, 1, 1>"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_step_f32_tiled_turbulent128_traffic.json")


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
    h = hashlib.sha256()
    for f in ("k_step_impl.h", "k_step_f32.hip", "pl_device.h", "pl_internal.h"):
        with open(os.path.join(ROOT, "paper_2602_23434_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def time_path(run, steps, warmup, flags, torch):
    """Whole-step timing (zeroing + fused kernel) and per-launch timing of the
    fused kernel alone, both with HIP events on the context's stream."""
    from paper_2602_23434_amd import binding as B
    for _ in range(warmup):
        run.step(flags=flags)
    run.stream.synchronize()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(run.stream)
    for _ in range(steps):
        run.step(flags=flags)
    e1.record(run.stream)
    e1.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = e0.elapsed_time(e1) / steps
    st = run.sync()
    if st != B.PL_OK:
        raise RuntimeError(f"device reported status {st}")
    # the fused kernel alone: one launch per call (no zeroing; deposits add up)
    kflags = B.PL_FUSE_DEPOSIT
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * steps)]
    for k in range(steps):
        ev[2 * k].record(run.stream)
        run.step(flags=kflags)
        ev[2 * k + 1].record(run.stream)
    ev[-1].synchronize()
    kern_ms = sum(ev[2 * k].elapsed_time(ev[2 * k + 1]) for k in range(steps)) / steps
    st = run.sync()
    if st != B.PL_OK:
        raise RuntimeError(f"device reported status {st}")
    return step_ms, kern_ms, wall


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
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--eager", action="store_true", help="launch steps without hipGraph replay")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (see DESIGN.md, sharding)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2602_23434_amd import benchcfg as BC
    from paper_2602_23434_amd import binding as B
    from paper_2602_23434_amd import driver, inputs

    B.lib()
    flags = BC.STEP_FLAGS & ~(B.PL_GRAPH if args.eager else 0)
    t0 = time.perf_counter()
    wl = inputs.turbulent_box(n=BC.TURB_N, npart=BC.TURB_NP, steps=args.steps)
    log(f"[bench] inputs generated in {time.perf_counter() - t0:.1f} s")
    npart = BC.TURB_NP
    cells = BC.TURB_N ** 3

    results = {}
    paths = [("f32_tiled", BC.F32_TILED)]
    if not args.no_fp64:
        paths.append(("f64_plain", BC.F64_PLAIN))
        paths.append(("f64_tiled", BC.F64_TILED))
    for name, cfg in paths:
        log(f"[bench] path {name}: setup")
        run = driver.Run(wl, **cfg)
        if cfg["algo"] == B.PL_ALGO_TILED:
            run.sort()
        run.sync()
        log(f"[bench] path {name}: {args.warmup} warmup + {args.steps} timed steps")
        step_ms, kern_ms, wall = time_path(run, args.steps, args.warmup, flags, torch)
        prec = "f32" if cfg["prec"] == B.PL_F32_OFFSET else "f64"
        abytes = algorithmic_bytes(prec, npart, cells)
        results[name] = {"ms_per_step": step_ms, "kernel_ms": kern_ms, "updates_per_s": npart / (step_ms * 1e-3),
                         "alg_bytes": abytes, "wall_s": wall}
        log(f"[bench] path {name}: {step_ms:.3f} ms/step, kernel {kern_ms:.3f} ms, "
            f"{npart / (step_ms * 1e-3):.3e} updates/s, {abytes / (kern_ms * 1e-3) / 1e9:.0f} GB/s algorithmic")
        run.close()
        del run
        torch.cuda.empty_cache()

    head = results["f32_tiled"]
    achieved = head["alg_bytes"] / (head["kernel_ms"] * 1e-3) / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as fh:
            tr = json.load(fh)
        if tr.get("src_digest") == src_digest():
            traffic = tr.get("bytes_per_launch")
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
                               "float32 + cell-offset form, LDS-tiled, rank-interleaved cell-tile sort at "
                               "setup, deposit rho+J+F (inputs of the float64 128^3 configuration)",
                   "grid": [BC.TURB_N] * 3, "particles": npart, "dt": 0.05, "shape": "tsc",
                   "tile": list(BC.F32_TILED["tile"]), "block": BC.F32_TILED["block"],
                   "sort_key": "tile+rank+cell",
                   "graph": not args.eager, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": KERNEL,
                     "kernel_ms": head["kernel_ms"], "alg_bytes_per_launch": head["alg_bytes"]},
    }
    if "f64_plain" in results:
        f64 = results["f64_plain"]
        out["fp64_plain"] = {"value": f64["updates_per_s"], "ms_per_step": f64["ms_per_step"],
                             "kernel_ms": f64["kernel_ms"],
                             "achieved_GBs": f64["alg_bytes"] / (f64["kernel_ms"] * 1e-3) / 1e9}
        out["speedup_f32_over_f64_plain"] = head["updates_per_s"] / f64["updates_per_s"]
    if "f64_tiled" in results:
        f64t = results["f64_tiled"]
        out["fp64_tiled"] = {"value": f64t["updates_per_s"], "ms_per_step": f64t["ms_per_step"],
                             "kernel_ms": f64t["kernel_ms"],
                             "achieved_GBs": f64t["alg_bytes"] / (f64t["kernel_ms"] * 1e-3) / 1e9}
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle on host cores)")
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
