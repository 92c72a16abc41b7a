"""Benchmark of the per-step particle update (gather + push + deposit).

Workload: 128^3 periodic box, turbulent E and B (|k|^-5/3, dB/B0 = 0.5,
E = -v x B), 2^24 charged particles (q/m = 1, weight 1) placed uniformly with
Maxwellian velocities (sigma = 0.05 c), TSC weights, dt = 0.05; every step
gathers E and B, pushes (relativistic Boris) and deposits rho, J and F at the
new positions.  The headline path is the float32 + cell-offset form with the
run-based LDS kernel; its sort (particles in run order: tile, run inside the
cell, cell) runs inside the timed loop at the tuned cadence.  The plain float64
path runs on the same inputs for the speedup, and the run-based float64 path
and the tiled float32 path beside it.

Each timed step is bracketed by HIP events on the library's stream: a step
without a sort zeroes the moment grids (one fill) and replays the fused
gather/push/deposit graph; a step at the sort cadence replays one graph that
sorts, zeroes and steps (PL_SORT_FIRST).  Prints ONE JSON line.  Inputs are
generated on the host and are resident in HBM before the timed region starts.

Beside the headline, in the same line: the clumped 256^3 box and the batched
workload (each with its own roofline), the Lagrangian spectral update on the
paper's particle workload (160^3 cells x 4 particles, 128 spectral points
each), the open-boundary deletion and compaction pass, the float32 error
table measured by the parity tests on the same kernel sources, and the
float64 oracle timed on the host cores (all threads and one).
"""

from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

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
LDS_FILE = os.path.join(ROOT, "profiles", "k_runs_f32_turbulent128_lds.json")
# LDS peak: 256 CUs x 128 bytes per clock at 2.4 GHz
LDS_PEAK_TBS = 256 * 128 * 2.4e9 / 1e12
ERR_FILE = os.path.join(ROOT, "profiles", "f32_error_table_turbulent32.json")


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
    (loop ms, per-launch kernel ms of the steps without a sort, per-step ms
    of the steps with one).  With graphs, a sorting step is one recorded
    sequence (PL_SORT_FIRST: sort, zeroing, step); the other steps zero the
    moments with one fill and replay the step alone."""
    ev = lambda: torch.cuda.Event(enable_timing=True)
    flags = B.PL_FUSE_DEPOSIT | (B.PL_GRAPH if graph else 0)
    kpairs, spairs = [], []
    t0, t1 = ev(), ev()
    t0.record(run.stream)
    for s in range(steps):
        a, b = ev(), ev()
        if every and s % every == 0:
            a.record(run.stream)
            if graph:
                run.step(flags=flags | B.PL_SORT_FIRST | B.PL_ZERO_FIRST)
            else:
                run.sort()
                run.step(flags=flags | B.PL_ZERO_FIRST)
            b.record(run.stream)
            spairs.append((a, b))
        else:
            run.zero_moments()
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
    kms = sum(kern) / len(kern)
    # a sorting step's time beyond a plain step's: the sort (and the zeroing fill)
    return {"ms_per_step": statistics.median(loops), "ms_min": min(loops), "ms_max": max(loops),
            "kernel_ms": kms, "sort_ms": (sum(sorts) / len(sorts) - kms) if sorts else 0.0}


def touched_cells(x, n):
    """Distinct cells in the union of the particles' TSC stencils (3^3 around
    each particle's cell, periodic), from float64 grid positions (3, np)."""
    import numpy as np
    nx, ny, nz = n
    c = [np.floor(np.mod(x[d], n[d])).astype(np.int64) % n[d] for d in range(3)]
    occ = np.zeros(nx * ny * nz, dtype=bool)
    occ[c[0] + nx * (c[1] + ny * c[2])] = True
    g = occ.reshape(nz, ny, nx)
    for ax in (2, 1, 0):
        g = g | np.roll(g, 1, axis=ax) | np.roll(g, -1, axis=ax)
    return int(g.sum())


# float32 form, bytes per particle read and written (cell 4, offsets 12, u 12, w 4 read; no w written)
F32_PART = 32 + 28
KIND_FIELDS = {"lorentz": 48, "dust": 24, "tracer": 24}     # E,B / gas velocity, float64
KIND_MOMENTS = {"lorentz": 7, "dust": 4, "tracer": 0}       # channels deposited, float64


def workload_bytes(wl, per_box_cells):
    """Algorithmic bytes of one step of every item of a float32 workload and
    of its charged items alone: each particle read and written once, each
    touched cell's fields read once per box and kind of field, each touched
    moment cell read-modify-written once per channel."""
    total = charged = 0
    fields_seen = set()
    for it in wl.items:
        kind = wl.species[it.species].kind
        cells = per_box_cells[it.box]
        fkey = (it.box, "EB" if kind == "lorentz" else "vg")
        fbytes = 0 if fkey in fields_seen else KIND_FIELDS[kind] * cells
        fields_seen.add(fkey)
        b = F32_PART * it.particles.n + fbytes + 2 * 8 * KIND_MOMENTS[kind] * cells
        total += b
        if kind == "lorentz":
            charged += F32_PART * it.particles.n + KIND_FIELDS[kind] * cells + 2 * 8 * 7 * cells
    return total, charged


def time_workload(wl, cfg, steps, every, torch, B, driver):
    """Whole-step time of a multi-item workload (all items in one call per
    step: one persistent launch per species kind), sort every `every` steps,
    and the charged-particle run kernel's time per launch (HIP events on the
    library's stream, one call per kind)."""
    run = driver.Run(wl, **cfg)
    try:
        run.sync()
        total = sum(it.particles.n for it in wl.items)
        timed_loop(run, 2, every, True, torch, B)
        ms, kern, sorts = timed_loop(run, steps, every, True, torch, B)
        stats = B.pl_part_stats(run.ctx)
        # the charged items alone, one call per step (their own launch), at the
        # same sort cadence; the steps without a sort are timed
        ci = [i for i, it in enumerate(wl.items) if wl.species[it.species].kind == "lorentz"]
        sub = (B.pl_item * len(ci))(*[run.items[i] for i in ci])
        ev = lambda: torch.cuda.Event(enable_timing=True)
        pairs = []
        for s in range(steps):
            if s % every == 0:
                run.step(flags=B.PL_FUSE_DEPOSIT | B.PL_ZERO_FIRST | B.PL_GRAPH | B.PL_SORT_FIRST, items=sub)
                continue
            run.zero_moments()
            a, b = ev(), ev()
            a.record(run.stream)
            run.step(flags=B.PL_FUSE_DEPOSIT | B.PL_GRAPH, items=sub)
            b.record(run.stream)
            pairs.append((a, b))
        torch.cuda.synchronize()
        if run.sync() != B.PL_OK:
            raise RuntimeError("device reported an error")
        charged_ms = sum(a.elapsed_time(b) for a, b in pairs) / len(pairs)
        kms = sum(kern) / len(kern)
        return {"value": total * steps / (ms * 1e-3), "unit": "particle-updates/s", "particles": total,
                "ms_per_step": ms / steps, "kernel_ms": kms,
                "sort_ms": (sum(sorts) / len(sorts) - kms) if sorts else 0.0, "sort_every": every, "steps": steps,
                "charged_kernel_ms": charged_ms, "run_kernel_launches": stats[4], "tiled_fallback_groups": stats[5]}
    finally:
        run.close()


def extra_workloads(head_cfg, torch, B, driver, inputs):
    """The clumped 256^3 box (2^26 particles, half in 32 Gaussian clumps, sort
    every 4 steps) and the batched workload (192^3 box with charged, dust and
    tracer species plus 16 independent 64^3 boxes), both in the float32 form
    (the clumped box in the headline's configuration, the batched workload in
    its own tuned one), timed over a whole number of sort periods of at least
    20 steps, each with its roofline: algorithmic bytes of the charged run
    kernel's launch over its time, and of the whole step (sort amortised) over
    the step time."""
    from paper_2602_23434_amd import benchcfg as BC
    out = {}
    bcfg = BC.batched_cfg()
    for name, make, every, wcfg in (("clumped_256", inputs.clumped_box, 4, BC.run_kwargs(head_cfg)),
                                    ("batched_192", inputs.batched, bcfg["sort_every"], BC.run_kwargs(bcfg))):
        t0 = time.perf_counter()
        wl = make()
        cells = [touched_cells(it.particles.x, wl.boxes[it.box].n) for it in wl.items]
        per_box = {}
        for it, c in zip(wl.items, cells):
            per_box[it.box] = max(per_box.get(it.box, 0), c)
        # every item of a box shares the box's cells: the union over its items
        for bidx in per_box:
            xs = [it.particles.x for it in wl.items if it.box == bidx]
            per_box[bidx] = touched_cells(np.concatenate(xs, axis=1), wl.boxes[bidx].n) if len(xs) > 1 \
                else per_box[bidx]
        log(f"[bench] {name}: inputs in {time.perf_counter() - t0:.1f} s")
        # a whole number of sort periods, at least 20 steps
        nsteps = every * max(2, -(-20 // every))
        r = time_workload(wl, wcfg, nsteps, every, torch, B, driver)
        r["config"] = {"tile": list(wcfg["tile"]), "sort_key": wcfg["key_mode"]}
        step_bytes, charged_bytes = workload_bytes(wl, per_box)
        npart = sum(it.particles.n for it in wl.items)
        sort_bytes = 132 * npart / every
        k_ach = charged_bytes / (r["charged_kernel_ms"] * 1e-3) / 1e9
        s_ach = (step_bytes + sort_bytes) / (r["ms_per_step"] * 1e-3) / 1e9
        r["roofline"] = {"bound": "hbm", "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "kernel": "charged-particle run kernel launch", "achieved": k_ach,
                         "frac": k_ach / HBM_PEAK_GBS, "alg_bytes_per_launch": charged_bytes,
                         "step_achieved": s_ach, "step_frac": s_ach / HBM_PEAK_GBS,
                         "alg_bytes_per_step": step_bytes + sort_bytes,
                         "alg_bytes_per_update": (step_bytes + sort_bytes) / npart}
        out[name] = r
        log(f"[bench] {name}: {r['ms_per_step']:.3f} ms/step, {r['value']:.3e} updates/s, charged kernel "
            f"{r['charged_kernel_ms']:.3f} ms ({k_ach:.0f} GB/s), step {s_ach:.0f} GB/s")
        del wl
        torch.cuda.empty_cache()
    return out


def spectra_leg(torch, B, driver, inputs, steps=10):
    """The Lagrangian spectral update on the paper's particle workload shape
    (Sec. 4.2 and Table 1: 160^3 cells x 4 particles = 16 384 000 particles,
    128 spectral points each, float64): one call per step for every particle.
    Algorithmic bytes per step: every spectral value read and written once
    (2 arrays x 128 x 8 B x 2), each particle's position read once (float32
    form: 16 B), and each touched cell's B, gas velocity and divergence read
    once (7 x 8 B)."""
    t0 = time.perf_counter()
    wl = inputs.spectra_box(n=160, ppc=4, nb=128, steps=steps)
    cells = touched_cells(wl.items[0].particles.x, wl.boxes[0].n)
    log(f"[bench] spectra: inputs in {time.perf_counter() - t0:.1f} s")
    run = driver.Run(wl, prec=B.PL_F32_OFFSET, algo=B.PL_ALGO_PLAIN, spectra=True, spectra_sets=1,
                     sort_buffers=False, channels=[])
    try:
        npart = wl.items[0].particles.n
        nb = len(wl.notes["eng0"])
        ev = lambda: torch.cuda.Event(enable_timing=True)
        for _ in range(2):
            run.spectra(cr=1e-4, u_rad=0.0, ub=0.5)
        pairs = []
        for _ in range(steps):
            a, b = ev(), ev()
            a.record(run.stream)
            run.spectra(cr=1e-4, u_rad=0.0, ub=0.5)
            b.record(run.stream)
            pairs.append((a, b))
        torch.cuda.synchronize()
        if run.sync() != B.PL_OK:
            raise RuntimeError("device reported an error in the spectral update")
        ms = sorted(a.elapsed_time(b) for a, b in pairs)[len(pairs) // 2]
        alg = npart * (2 * nb * 8 * 2 + 16) + cells * 7 * 8
        ach = alg / (ms * 1e-3) / 1e9
        r = {"workload": "160^3 box, 4 particles per cell (16 384 000), 128 spectral points each, float64 spectra, "
                         "turbulent B and gas velocity, random four-divergence (rms 0.1)",
             "particles": npart, "bins": nb, "ms_per_step": ms, "value": npart / (ms * 1e-3),
             "unit": "particle-spectra/s",
             "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": ach / HBM_PEAK_GBS, "alg_bytes_per_launch": alg,
                          "kernel": "pl::k_spectra<1, 2, 3>"},
             "paper_context": "Particles_Spectra: 190 ms per step for 16.4 M particles on one A100 (Table 1)"}
        log(f"[bench] spectra: {ms:.3f} ms/step, {ach:.0f} GB/s algorithmic")
        return r
    finally:
        run.close()
        del run
        torch.cuda.empty_cache()


def boundary_leg(wl, run_kw, torch, B, driver):
    """Deletion at open boundaries and the holes-and-fillers compaction on the
    headline's 2^24 particles (float32 form), all three dimensions open with
    two ghost layers: one synchronous call, timed on the host clock.
    Algorithmic bytes: each particle's cell read once, and every moved
    particle's arrays read and written once (cell, offsets, u, w, id: 40 B)."""
    run = driver.Run(wl, **run_kw)
    try:
        run.sort()
        run.sync()
        n0 = run.items[0].p.n
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        removed = run.boundary((1, 1, 1), 2)[0]
        ms = (time.perf_counter() - t0) * 1e3
        moved = min(removed, run.items[0].p.n)
        alg = 4 * n0 + 2 * 40 * moved
        return {"particles": n0, "removed": removed, "ms": ms, "value": n0 / (ms * 1e-3),
                "unit": "particles/s", "alg_bytes": alg, "achieved_GBs": alg / (ms * 1e-3) / 1e9,
                "note": "one call, host clock (kernels, the count read-back and the stream synchronisation)"}
    finally:
        run.close()


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, target_s=12.0):
    """The float64 oracle on the host cores, on a bounded sample of the same
    workload: the first `ns` particles (same fields, grid, dt), whole steps of
    gather + push + deposit, with every thread and with one.  The oracle's
    push runs on all threads (OpenMP over particles); its deposit is a serial
    loop in particle order, so the all-thread rate is not a per-core rate
    times the core count."""
    import oracle
    it = wl.items[0].particles
    box = wl.boxes[0]
    ns = 1 << 20

    def rate(threads, budget):
        oracle.set_threads(threads)
        x = np.ascontiguousarray(it.x[:, :ns])
        u = np.ascontiguousarray(it.u[:, :ns])
        w = np.ascontiguousarray(it.w[:ns])
        steps, t_total = 0, 0.0
        while t_total < budget and steps < 50:
            mom = oracle.new_moments(box.n, oracle.LORENTZ)
            mom["eng"] = None
            t0 = time.perf_counter()
            oracle.step(3, box.n, oracle.TSC, (oracle.LORENTZ, 1.0, 1.0, 0.0), x, u, w, box.fields, wl.dt,
                        moments=mom)
            t_total += time.perf_counter() - t0
            steps += 1
        return ns * steps / t_total, steps, t_total

    cores = os.cpu_count() or 1
    allv, asteps, at = rate(cores, target_s)
    used = oracle.num_threads()
    onev, osteps, ot = rate(1, target_s / 2)
    oracle.set_threads(cores)
    return {"value": allv, "unit": "particle-updates/s", "cores": used, "kind": "oracle",
            "sample": f"first {ns} of the 2^24 particles, {asteps} full steps (gather+push+deposit of rho,J,F) "
                      f"on the 128^3 turbulent fields, {at:.1f} s; the push runs on {used} threads, the "
                      f"deposit serially",
            "one_thread": {"value": onev, "steps": osteps, "seconds": ot},
            "cpu_model": cpu_model()}


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
    ap.add_argument("--no-extra", action="store_true", help="skip the clumped and batched workloads")
    ap.add_argument("--no-spectra", action="store_true", help="skip the spectral update leg")
    ap.add_argument("--no-boundary", action="store_true", help="skip the open-boundary leg")
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
        if not args.no_tiled:
            paths.append(("f64_tiled", BC.F64_TILED, every64, args.reps))
        paths.append(("f64_runs", BC.run_kwargs(f64_cfg), every64, args.reps))
    for name, cfg, ev_every, reps in paths:
        log(f"[bench] path {name}: setup")
        run = driver.Run(wl, **cfg)
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
    step_gbs = (head["alg_bytes"] + 132 * npart / every) / (head["ms_per_step"] * 1e-3) / 1e9
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
    # LDS occupancy and bytes per launch from the committed counters of the
    # same kernel source; the bandwidth against this run's kernel time
    if os.path.exists(LDS_FILE):
        with open(LDS_FILE) as fh:
            ld = json.load(fh)
        from paper_2602_23434_amd import profiling
        if ld.get("src_digest") == src_digest() and ld.get("config") == profiling.workload_config():
            lds_tbs = ld["lds_bytes"] / (head["kernel_ms"] * 1e-3) / 1e12
            secondary = dict(secondary or {})
            secondary["lds"] = dict(secondary.get("lds", {}))
            secondary["lds"].update({"busy_frac": ld["lds_util"],
                                     "bank_conflict_share_of_busy": ld["bank_conflict_share_of_active"],
                                     "bytes_per_launch": ld["lds_bytes"], "achieved_TBs": lds_tbs,
                                     "peak_TBs": LDS_PEAK_TBS, "bw_frac": lds_tbs / LDS_PEAK_TBS})
    # float32 error table of the same kernel sources (written by the whole-grid
    # parity test of the benchmarked variant)
    error_table = None
    if os.path.exists(ERR_FILE):
        with open(ERR_FILE) as fh:
            et = json.load(fh)
        if et.get("src_digest") == src_digest():
            error_table = et
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
                     "kernel_ms": head["kernel_ms"], "alg_bytes_per_launch": head["alg_bytes"],
                     # the whole step (moment zeroing and the sort, amortised, included)
                     "step_achieved": step_gbs, "step_frac": step_gbs / HBM_PEAK_GBS},
        "secondary_ceilings": secondary,
        "error_table": error_table,
    }
    for name, key in (("f32_tiled", "fp32_tiled"), ("f64_plain", "fp64_plain"), ("f64_tiled", "fp64_tiled"),
                      ("f64_runs", "fp64_runs")):
        if name in results:
            r = results[name]
            out[key] = {"value": r["updates_per_s"], "ms_per_step": r["ms_per_step"], "kernel_ms": r["kernel_ms"],
                        "sort_ms": r["sort_ms"],
                        "achieved_GBs": r["alg_bytes"] / (r["kernel_ms"] * 1e-3) / 1e9}
    if "f64_plain" in results:
        out["speedup_f32_over_f64_plain"] = head["updates_per_s"] / results["f64_plain"]["updates_per_s"]
    if "f64_tiled" in results:
        out["speedup_f32_over_f64_tiled"] = head["updates_per_s"] / results["f64_tiled"]["updates_per_s"]
    if "f64_runs" in results:
        out["speedup_f32_over_f64_runs"] = head["updates_per_s"] / results["f64_runs"]["updates_per_s"]
    if not args.no_boundary:
        log("[bench] open-boundary deletion and compaction")
        out["boundary"] = boundary_leg(wl, BC.run_kwargs(head_cfg), torch, B, driver)
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle on host cores)")
        out["cpu_baseline"] = cpu_baseline(wl)
    del wl
    if not args.no_extra:
        out["workloads"] = extra_workloads(head_cfg, torch, B, driver, inputs)
    if not args.no_spectra:
        out["spectra"] = spectra_leg(torch, B, driver, inputs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
