"""Autotuner for the tiled step: tile shape, threads per block, sort key and
sort cadence.

    python -m paper_2602_23434_amd.tune --out tune_cache.txt [--n 128 --ppc 8 --steps 8]

For every candidate it builds a context on a synthetic turbulent box of the
requested size, sorts, and times `steps` fused steps with the sort repeated at
the candidate cadence (the sort's cost is amortised into the per-step time).
The winner is written as "key value" lines that pl_part_init reads (block,
tile) and the Python driver reads (key, sort_every).
"""

from __future__ import annotations

import argparse
import itertools
import json
import sys
import time

from . import binding as B
from . import driver, inputs

TILES = [(8, 8, 8), (8, 8, 4), (16, 8, 8), (8, 4, 4), (16, 8, 4)]
BLOCKS = [256, 512]
KEYS = [B.PL_KEY_TILE, B.PL_KEY_TILE_RANK]
CADENCES = [1, 4, 0]          # 0 = sort once at setup only
CHANNELS = ["rho", "J0", "J1", "J2", "F0", "F1", "F2"]


def time_candidate(wl, prec, tile, block, key, every, steps, torch):
    run = driver.Run(wl, prec=prec, algo=B.PL_ALGO_TILED, tile=tile, block=block, key_mode=key,
                     channels=CHANNELS, eng=False)
    try:
        run.sort()
        flags = B.PL_FUSE_DEPOSIT | B.PL_ZERO_FIRST
        run.step(flags=flags)
        run.sync()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(run.stream)
        for s in range(steps):
            if every and s % every == every - 1:
                run.sort()
            run.step(flags=flags)
        e1.record(run.stream)
        e1.synchronize()
        st = run.sync()
        if st != B.PL_OK:
            return None
        return e0.elapsed_time(e1) / steps
    except B.PLError:
        return None
    finally:
        run.close()


def tune(n=128, ppc=8, steps=8, prec=B.PL_F32_OFFSET, log=print):
    import torch
    wl = inputs.turbulent_box(n=n, npart=ppc * n ** 3, steps=steps)
    best = None
    results = []
    for tile, block, key, every in itertools.product(TILES, BLOCKS, KEYS, CADENCES):
        if any(n % t for t in tile):
            continue
        ms = time_candidate(wl, prec, tile, block, key, every, steps, torch)
        results.append({"tile": tile, "block": block, "key": key, "sort_every": every, "ms": ms})
        log(f"[tune] tile {tile} block {block} key {key} sort_every {every}: "
            f"{'unsupported' if ms is None else f'{ms:.3f} ms/step'}")
        if ms is not None and (best is None or ms < best["ms"]):
            best = results[-1]
    return best, results


def write_cache(path, best):
    with open(path, "w") as fh:
        fh.write(f"block {best['block']}\n")
        fh.write("tile {} {} {}\n".format(*best["tile"]))
        fh.write(f"key {best['key']}\n")
        fh.write(f"sort_every {best['sort_every']}\n")
        fh.write(f"ms_per_step {best['ms']:.4f}\n")


def read_cache(path):
    out = {}
    with open(path) as fh:
        for line in fh:
            parts = line.split()
            if not parts:
                continue
            vals = [float(v) if "." in v else int(v) for v in parts[1:]]
            out[parts[0]] = vals[0] if len(vals) == 1 else tuple(vals)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default="tune_cache.txt")
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--ppc", type=int, default=8)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--f64", action="store_true")
    a = ap.parse_args()
    t0 = time.perf_counter()
    best, results = tune(a.n, a.ppc, a.steps, B.PL_F64 if a.f64 else B.PL_F32_OFFSET,
                         log=lambda m: print(m, file=sys.stderr, flush=True))
    write_cache(a.out, best)
    print(json.dumps({"best": best, "seconds": time.perf_counter() - t0}))


if __name__ == "__main__":
    main()
