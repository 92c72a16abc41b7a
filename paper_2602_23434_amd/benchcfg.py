"""Launch configurations the benchmark times (shared with the full-size
parity tests, so both exercise exactly the same path)."""

from . import binding as B

# 128^3 turbulent box, 2^24 charged particles; deposits rho, J, F (7 channels)
TURB_N = 128
TURB_NP = 1 << 24
CHANNELS = ["rho", "J0", "J1", "J2", "F0", "F1", "F2"]
STEP_FLAGS = B.PL_FUSE_DEPOSIT | B.PL_ZERO_FIRST | B.PL_GRAPH

F32_TILED = dict(prec=B.PL_F32_OFFSET, algo=B.PL_ALGO_TILED, key_mode=B.PL_KEY_TILE_RANK, tile=(8, 8, 8), block=512,
                 channels=CHANNELS, eng=False)
F64_PLAIN = dict(prec=B.PL_F64, algo=B.PL_ALGO_PLAIN, key_mode=B.PL_KEY_TILE, tile=None, block=256,
                 channels=CHANNELS, eng=False)
F64_TILED = dict(prec=B.PL_F64, algo=B.PL_ALGO_TILED, key_mode=B.PL_KEY_TILE_RANK, tile=(8, 8, 4), block=512,
                 channels=CHANNELS, eng=False)
# run-based kernels (particles sorted into run order, runs of up to four particles per thread)
F32_RUNS = dict(prec=B.PL_F32_OFFSET, algo=B.PL_ALGO_RUNS, key_mode=B.PL_KEY_TILE_RUN, tile=(8, 8, 8), block=512,
                channels=CHANNELS, eng=False)
F64_RUNS = dict(prec=B.PL_F64, algo=B.PL_ALGO_RUNS, key_mode=B.PL_KEY_TILE_RUN, tile=(8, 8, 4), block=512,
                channels=CHANNELS, eng=False)
# steps between sorts inside the timed loop when no tune file is present
SORT_EVERY = 8


def _tuned(cfg, prec, batched=False):
    """cfg with the autotuner's choice (tune_mi355x_*.txt next to this
    module, written by `python -m paper_2602_23434_amd.tune`) applied:
    algorithm, sort key, tile, block and sort cadence."""
    import os

    from . import tune
    path = tune.tune_file(prec, batched)
    out = dict(cfg)
    out["sort_every"] = SORT_EVERY
    if not os.path.exists(path):
        return out
    t = tune.read_cache(path)
    out["algo"] = int(t.get("algo", out["algo"]))
    out["key_mode"] = int(t.get("key", out["key_mode"]))
    out["tile"] = tuple(int(v) for v in t.get("tile", out["tile"]))
    out["block"] = int(t.get("runs_block", t.get("block", out["block"])))
    out["sort_every"] = int(t.get("sort_every", SORT_EVERY))
    return out


def headline():
    """The float32 configuration the benchmark times (tuned when a tune file exists)."""
    return _tuned(F32_RUNS, B.PL_F32_OFFSET)


def batched_cfg():
    """The float32 configuration of the batched workload: the autotuner's
    choice on that workload when its tune file exists, else the headline's;
    every channel each species kind deposits."""
    import os

    from . import tune
    path = tune.tune_file(B.PL_F32_OFFSET, batched=True)
    if os.path.exists(path):
        cfg = dict(_tuned(F32_RUNS, B.PL_F32_OFFSET, batched=True))
        cfg["tune_cache"] = path            # the library reads its launch choice there
    else:
        cfg = dict(headline())
    cfg["channels"] = None
    return cfg


def f64_sorted():
    """The sorted float64 configuration beside it (tuned when a tune file exists)."""
    return _tuned(F64_RUNS, B.PL_F64)


def run_kwargs(cfg):
    """driver.Run keyword arguments of a configuration."""
    return {k: v for k, v in cfg.items() if k != "sort_every"}
