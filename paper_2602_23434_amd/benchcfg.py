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
# run-based kernels (tile+cell sort, runs of up to four particles per thread)
F32_RUNS = dict(prec=B.PL_F32_OFFSET, algo=B.PL_ALGO_RUNS, key_mode=B.PL_KEY_TILE_CELL, tile=(8, 8, 8), block=512,
                channels=CHANNELS, eng=False)
F64_RUNS = dict(prec=B.PL_F64, algo=B.PL_ALGO_RUNS, key_mode=B.PL_KEY_TILE_CELL, tile=(8, 8, 4), block=512,
                channels=CHANNELS, eng=False)
# steps between sorts inside the timed loop (the autotuner's cadence choice
# for this workload)
SORT_EVERY = 8
