"""Parity of the run-based kernels (PL_ALGO_RUNS) through the C ABI.

* the run table written by the sort equals the one built here from the
  oracle's stable tile+cell permutation, entry for entry;
* particle states are bit-identical to the tiled kernel's (same terms in the
  same order), for every drift regime: particles that left their run's cell
  or tile since the sort go through the LDS queues, and past the queue
  capacity through the immediate path;
* states and deposits match the float64 oracle within the tolerances of
  test_parity_gpu (float64: 1e-11 cells, 1e-12 relative; float32 form: the
  error-table bounds).
"""

import sys

import numpy as np
import pytest

from tests import _cmp
from tests.test_parity_gpu import M_TOL, U_TOL, X_TOL, _check_item, _run_gpu, _small_batch, _turb

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mods():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    from paper_2602_23434_amd import binding, driver, inputs
    binding.lib()
    return oracle, driver, inputs, binding


RUN_LEN = 4


def _assert_runs_kernel(run, B):
    """The run-based kernel took every fused step (no tiled fallback)."""
    st = B.pl_part_stats(run.ctx)
    assert st[4] > 0 and st[5] == 0, st


def expected_runs(sorted_keys, per_tile, ntiles):
    """Run table from sorted tile * per_tile + cell keys: per tile, the runs of
    every cell (up to RUN_LEN consecutive positions), listed by (index of the
    run inside its cell, cell); entry (first << 2) | (length - 1)."""
    np_ = len(sorted_keys)
    out = np.zeros(np_ + ntiles, dtype=np.int64)
    tiles = sorted_keys // per_tile
    tstart = np.searchsorted(tiles, np.arange(ntiles + 1), side="left")
    for t in range(ntiles):
        beg, end = tstart[t], tstart[t + 1]
        loc = sorted_keys[beg:end] - t * per_tile
        cnt = np.bincount(loc, minlength=per_tile)
        first = beg + np.concatenate(([0], np.cumsum(cnt)[:-1]))
        pos = beg
        b = 0
        while True:
            cells = np.nonzero(cnt > b * RUN_LEN)[0]
            if len(cells) == 0:
                break
            for c in cells:
                ln = min(RUN_LEN, cnt[c] - b * RUN_LEN)
                out[pos] = ((first[c] + b * RUN_LEN) << 2) | (ln - 1)
                pos += 1
            b += 1
        out[np_ + t] = pos - beg
    return out, tstart


def expected_units(counts, split=1024, min_piece=1024, rank_max=1024):
    """Work units of the run kernel as (tile, piece | npieces << 16) pairs.
    With P = max(ceil(total / split), min_piece) a tile of c runs gives
    ceil(c / P) pieces, an empty tile none; tiles cut in several pieces or
    holding more than twice the mean run count come first (the first
    rank_max in index order), by decreasing runs per piece then tile index,
    then the other non-empty tiles in index order."""
    from fractions import Fraction
    ntiles = len(counts)
    total = int(counts.sum())
    pz = max(-(-total // split), min_piece)
    thr = 2 * (total // max(ntiles, 1)) + 1
    k = [-(-int(c) // pz) for c in counts]
    cand = [t for t in range(ntiles) if k[t] >= 2 or counts[t] > thr][:rank_max]
    cs = set(cand)
    ranked = sorted(cand, key=lambda t: (-Fraction(int(counts[t]), k[t]), t))
    units = []
    for t in ranked + [t for t in range(ntiles) if t not in cs and k[t] > 0]:
        units += [(t, p | (k[t] << 16)) for p in range(k[t])]
    return np.array(units, dtype=np.int64).reshape(-1, 2)


def swizzled_keys(keys, tile):
    """Tile+cell keys with the cell numbering of PL_KEY_TILE_RUN: the rows y
    of every group of eight listed as 0, 2, 4, 6, 1, 3, 5, 7 (tile y size a
    multiple of eight), else those of every group of four as 0, 2, 1, 3 (a
    multiple of four); the key holds each row's place in that list."""
    tx, ty, tz = tile
    per_tile = tx * ty * tz
    t, loc = keys // per_tile, keys % per_tile
    x, y, z = loc % tx, (loc // tx) % ty, loc // (tx * ty)
    if ty % 8 == 0:
        listed = [0, 2, 4, 6, 1, 3, 5, 7]
        y = (y // 8) * 8 + np.argsort(listed)[y % 8]
    elif ty % 4 == 0:
        listed = [0, 2, 1, 3]
        y = (y // 4) * 4 + np.argsort(listed)[y % 4]
    return t * per_tile + x + tx * (y + ty * z)


def run_order(sorted_keys, per_tile):
    """Positions of the tile+cell order in run order, from the definition of
    PL_KEY_TILE_RUN: stable sort by (tile, rank in cell // 4, cell, rank % 4)."""
    n = len(sorted_keys)
    first = np.searchsorted(sorted_keys, sorted_keys, side="left")
    rank = np.arange(n) - first
    tile, cell = sorted_keys // per_tile, sorted_keys % per_tile
    return np.lexsort((rank % RUN_LEN, cell, rank // RUN_LEN, tile))


def relaid_runs(exp, tstart, npart, ntiles):
    """The run table with every tile's runs laid out one after another in table
    order from its first position; returns the entries and, per new position,
    the tile+cell position it came from."""
    out = exp.copy()
    src = np.zeros(npart, dtype=np.int64)
    for t in range(ntiles):
        q = tstart[t]
        for k in range(tstart[t], tstart[t] + exp[npart + t]):
            first, ln = exp[k] >> 2, (exp[k] & 3) + 1
            out[k] = (q << 2) | (ln - 1)
            src[q:q + ln] = np.arange(first, first + ln)
            q += ln
    return out, src


@pytest.mark.parametrize("key", ["cell", "run"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_runs_table_exact(mods, prec, key):
    oracle, driver, inputs, B = mods
    kmode = B.PL_KEY_TILE_CELL if key == "cell" else B.PL_KEY_TILE_RUN
    # 40 per cell: most cells of every tile hold more than eight runs (the
    # run-table build shares the rounds beyond eight among its waves); the
    # 16x8x8 tile has the largest cell count a tile may have (1024)
    for n, npart, tile in ((32, 8 * 32 ** 3 - 37, (8, 8, 8)), (16, 1, (4, 4, 4)), (16, 3001, (16, 8, 2)),
                           (16, 20000, (4, 4, 4)), (16, 40 * 16 ** 3 + 5, (8, 8, 8)),
                           (16, 40 * 16 ** 3 + 5, (16, 8, 8)), (32, -1, (4, 4, 4)), (32, -2, (4, 4, 4)),
                           (32, -2, (8, 8, 8)), (24, 5 * 24 ** 3 + 3, (6, 4, 3))):
        say(f"[runs] run table {prec} key {key} n={n} np={npart} tile={tile}")
        split = npart < 0 and tile == (4, 4, 4)
        if npart < 0:
            # clumped: crowded tiles cut into pieces that go first in the order
            ck = dict(npart=60000, nclumps=3, sigma=1.5) if npart == -1 else dict(npart=200000, nclumps=2, sigma=1.0)
            wl = inputs.clumped_box(n=n, steps=0, **ck)
            npart = wl.items[0].particles.n
        else:
            wl = inputs.turbulent_box(n=n, npart=npart, steps=0)
        p = B.PL_F64 if prec == "f64" else B.PL_F32_OFFSET
        run = driver.Run(wl, prec=p, algo=B.PL_ALGO_RUNS, tile=tile, key_mode=kmode)
        run.sort()
        assert run.sync() == B.PL_OK
        raw = run.raw(0)
        x = wl.items[0].particles.x
        bx = wl.boxes[0].n
        if p == B.PL_F64:
            cells = oracle.cells_of_positions(3, bx, x)
        else:
            cells, _ = oracle.split_positions(3, bx, x)
        keys = np.array([oracle.tile_key(3, bx, tile, 1, *cells[:, q]) for q in range(npart)], dtype=np.int64)
        if key == "run":
            keys = swizzled_keys(keys, tile)
        perm = oracle.stable_sort_perm(keys.astype(np.uint32))
        ntiles = (n // tile[0]) * (n // tile[1]) * (n // tile[2])
        per_tile = tile[0] * tile[1] * tile[2]
        exp, tstart = expected_runs(keys[perm], per_tile, ntiles)
        if key == "run":
            exp, src = relaid_runs(exp, tstart, npart, ntiles)
            assert np.array_equal(src, run_order(keys[perm], per_tile))
            perm = perm[src]
        assert np.array_equal(raw["id"].astype(np.int64), perm)
        assert np.array_equal(raw["tile_start"][: ntiles + 1], tstart)
        got = raw["runs"].astype(np.int64)
        for t in range(ntiles):
            beg = tstart[t]
            nr = exp[npart + t]
            assert got[npart + t] == nr, (t, got[npart + t], nr)
            assert np.array_equal(got[beg:beg + nr], exp[beg:beg + nr]), t
        units = expected_units(exp[npart:npart + ntiles])
        nunits = got[npart + 3 * ntiles + 2 * B.PL_RUNS_SPLIT_UNITS]
        say(f"  {ntiles} tiles -> {nunits} units, largest piece {np.max(exp[npart:npart + ntiles])} runs")
        assert nunits == len(units)
        assert np.array_equal(got[npart + ntiles:npart + ntiles + 2 * nunits].reshape(-1, 2), units)
        if split:
            assert (units[:, 1] >> 16).max() >= 2, "no tile was split"
        run.close()


def test_runs_turbulent_fp64(mods):
    oracle, driver, inputs, B = mods
    say("[runs] turbulent 32^3, 262107 particles, 5 steps, f64 runs vs oracle")
    wl = _turb(inputs)
    ores = oracle.run_workload(wl)
    run, st = _run_gpu(driver, wl, wl.steps, True, prec=B.PL_F64, algo=B.PL_ALGO_RUNS)
    assert st == B.PL_OK
    _assert_runs_kernel(run, B)
    _check_item(run, 0, ores[0], wl, X_TOL, U_TOL, M_TOL)
    run.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_runs_tile_not_power_of_two(mods, prec):
    """A 6x4x3 tile (72 cells: tile and cell indices by division, rows
    swizzled in groups of four) on a 24^3 box, sorted every 2 of 6 steps:
    float64 against the oracle within the parity tolerances; float32 per-id
    states bit-identical to the tiled kernel on the same tile and deposits
    within 2e-6 of its largest value."""
    oracle, driver, inputs, B = mods
    say(f"[runs] {prec} tile (6, 4, 3) on 24^3, 6 steps, sort every 2")
    wl = inputs.turbulent_box(n=24, npart=8 * 24 ** 3 - 13, steps=6)
    tile = (6, 4, 3)
    if prec == "f64":
        ores = oracle.run_workload(wl)
        run, st = _run_gpu(driver, wl, wl.steps, True, sort_every=2, prec=B.PL_F64, algo=B.PL_ALGO_RUNS,
                           tile=tile)
        assert st == B.PL_OK
        _assert_runs_kernel(run, B)
        ex, eu, _ = _check_item(run, 0, ores[0], wl, X_TOL, U_TOL, M_TOL)
        say(f"  max |dx| {ex:.3e} cells, max |du|/max(|u|, sigma) {eu:.3e}")
        run.close()
        return
    res = {}
    for algo in (B.PL_ALGO_TILED, B.PL_ALGO_RUNS):
        kmode = B.PL_KEY_TILE_CELL if algo == B.PL_ALGO_TILED else B.PL_KEY_TILE_RUN
        run, st = _run_gpu(driver, wl, wl.steps, True, sort_every=2, prec=B.PL_F32_OFFSET, algo=algo, tile=tile,
                           key_mode=kmode)
        assert st == B.PL_OK
        if algo == B.PL_ALGO_RUNS:
            _assert_runs_kernel(run, B)
        raw = run.raw(0)
        ids = raw["id"].astype(np.int64)
        res[algo] = ({k: _cmp.by_id(np.stack(v) if isinstance(v, list) else v, ids) for k, v in raw.items()
                      if k in ("x", "u", "cell")}, run.moments(0))
        run.close()
    (sa, ma), (sb, mb) = res[B.PL_ALGO_TILED], res[B.PL_ALGO_RUNS]
    for k in sa:
        assert np.array_equal(sa[k], sb[k]), k
    for k in ma:
        va, vb = np.asarray(ma[k]), np.asarray(mb[k])
        assert np.abs(va - vb).max() <= 2e-6 * np.abs(va).max(), k


def test_runs_f32_error_table(mods):
    oracle, driver, inputs, B = mods
    say("[runs] turbulent 32^3, 20 steps, f32+offset runs vs f64 oracle")
    wl = _turb(inputs, steps=20)
    ores = oracle.run_workload(wl)
    run, st = _run_gpu(driver, wl, wl.steps, True, sort_every=4, prec=B.PL_F32_OFFSET, algo=B.PL_ALGO_RUNS)
    assert st == B.PL_OK
    _assert_runs_kernel(run, B)
    gx, gu, gid, _ = run.state(0)
    table = _cmp.state_error_stats(gx, gu, gid, ores[0]["x"], ores[0]["u"], wl.boxes[0].n, 3)
    merr = _cmp.moment_errors(run.moments(0), ores[0]["moments"], ores[0]["abs"])
    for k, (mx, rms) in table.items():
        say(f"  {k:4s} max {mx:.3e} rms {rms:.3e}")
    for k, (mx, rms, rel) in merr.items():
        say(f"  {k:4s} max/A_c {mx:.3e} rms/A_c {rms:.3e} max/max|M| {rel:.3e}")
    bad = _cmp.check_fp32_table(table, merr)
    assert not bad, bad
    run.close()


def _hot_box(inputs, n=16, steps=10, dt=1.0, speed=0.6, ragged=11):
    """Fast particles (|v| = 0.6 c, dt = 1: up to 0.6 cells per step and
    dimension): after a few steps most particles have left the cell and often
    the tile they were sorted into."""
    wl = inputs.turbulent_box(n=n, npart=8 * n ** 3 - ragged, steps=steps)
    p = wl.items[0].particles
    p.u = inputs.isotropic_u(np.random.default_rng(4242), p.n, speed)
    wl.dt = dt
    return wl


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("tile,key", [((4, 4, 4), "run"), ((8, 8, 4), "run"), ((4, 4, 4), "cell")])
def test_runs_states_match_tiled_under_drift(mods, prec, tile, key):
    """No re-sort for 10 fast steps: queues fill and overflow on the 4^3
    tiles.  Per-id states bit-identical to the tiled kernel; deposits within
    the precision's tolerance of it (run kernel on run-ordered or tile+cell
    ordered particles)."""
    oracle, driver, inputs, B = mods
    say(f"[runs] drift {prec} tile {tile} key {key}: runs vs tiled, 10 steps without re-sort")
    wl = _hot_box(inputs)
    p = B.PL_F64 if prec == "f64" else B.PL_F32_OFFSET
    res = {}
    for algo in (B.PL_ALGO_TILED, B.PL_ALGO_RUNS):
        kmode = B.PL_KEY_TILE_CELL if (algo == B.PL_ALGO_TILED or key == "cell") else B.PL_KEY_TILE_RUN
        run, st = _run_gpu(driver, wl, wl.steps, True, prec=p, algo=algo, tile=tile, key_mode=kmode)
        assert st == B.PL_OK
        if algo == B.PL_ALGO_RUNS:
            _assert_runs_kernel(run, B)
        raw = run.raw(0)
        ids = raw["id"].astype(np.int64)
        res[algo] = ({k: _cmp.by_id(np.stack(v) if isinstance(v, list) else v, ids) for k, v in raw.items()
                      if k in ("x", "u", "cell")}, run.moments(0))
        run.close()
    (sa, ma), (sb, mb) = res[B.PL_ALGO_TILED], res[B.PL_ALGO_RUNS]
    for k in sa:
        assert np.array_equal(sa[k], sb[k]), k
    rtol = 1e-12 if p == B.PL_F64 else 2e-6
    for k in ma:
        va, vb = np.asarray(ma[k]), np.asarray(mb[k])
        scale = np.abs(va).max()
        assert np.abs(va - vb).max() <= rtol * scale, (k, float(np.abs(va - vb).max() / scale))


def test_runs_drift_fp64_vs_oracle(mods):
    oracle, driver, inputs, B = mods
    say("[runs] drift f64 tile 4^3 vs oracle, 10 fast steps without re-sort")
    wl = _hot_box(inputs)
    ores = oracle.run_workload(wl)
    run, st = _run_gpu(driver, wl, wl.steps, True, prec=B.PL_F64, algo=B.PL_ALGO_RUNS, tile=(4, 4, 4))
    assert st == B.PL_OK
    _assert_runs_kernel(run, B)
    ex, eu, _ = _check_item(run, 0, ores[0], wl, X_TOL, U_TOL, M_TOL)
    say(f"  max |dx| {ex:.3e} cells, max |du|/max(|u|, sigma) {eu:.3e}")
    run.close()


def _split_box(inputs, steps=4):
    """Two tight clumps in a 32^3 box: with 4^3 tiles the crowded tiles hold up
    to ~8400 runs, cut into as many as 9 pieces processed by different CUs."""
    return inputs.clumped_box(n=32, npart=200000, nclumps=2, sigma=1.0, steps=steps)


def test_runs_split_tiles_fp64_vs_oracle(mods):
    oracle, driver, inputs, B = mods
    say("[runs] clumped 32^3 f64, 200000 particles, split tiles, 4 steps (sorted every 2) vs oracle")
    wl = _split_box(inputs)
    ores = oracle.run_workload(wl)
    run, st = _run_gpu(driver, wl, wl.steps, True, sort_every=2, prec=B.PL_F64, algo=B.PL_ALGO_RUNS,
                       tile=(4, 4, 4))
    assert st == B.PL_OK
    _assert_runs_kernel(run, B)
    raw = run.raw(0)
    ntiles = 8 ** 3
    units = raw["runs"][wl.items[0].particles.n + ntiles:].astype(np.int64)
    nunits = units[2 * (ntiles + B.PL_RUNS_SPLIT_UNITS)]
    assert nunits > np.count_nonzero(raw["runs"][wl.items[0].particles.n:][:ntiles]), "no tile was split"
    _check_item(run, 0, ores[0], wl, X_TOL, U_TOL, M_TOL)
    run.close()


def test_runs_split_tiles_f32_match_tiled(mods):
    """Split tiles, float32 form: per-id states bit-identical to the tiled
    kernel's, deposits within float32 rounding of it."""
    oracle, driver, inputs, B = mods
    say("[runs] clumped 32^3 f32, split tiles, 4 steps: runs vs tiled")
    wl = _split_box(inputs)
    res = {}
    for algo in (B.PL_ALGO_TILED, B.PL_ALGO_RUNS):
        kmode = B.PL_KEY_TILE_CELL if algo == B.PL_ALGO_TILED else B.PL_KEY_TILE_RUN
        run, st = _run_gpu(driver, wl, wl.steps, True, sort_every=2, prec=B.PL_F32_OFFSET, algo=algo,
                           tile=(4, 4, 4), key_mode=kmode)
        assert st == B.PL_OK
        if algo == B.PL_ALGO_RUNS:
            _assert_runs_kernel(run, B)
        raw = run.raw(0)
        ids = raw["id"].astype(np.int64)
        res[algo] = ({k: _cmp.by_id(np.stack(v) if isinstance(v, list) else v, ids) for k, v in raw.items()
                      if k in ("x", "u", "cell")}, run.moments(0))
        run.close()
    (sa, ma), (sb, mb) = res[B.PL_ALGO_TILED], res[B.PL_ALGO_RUNS]
    for k in sa:
        assert np.array_equal(sa[k], sb[k]), k
    for k in ma:
        va, vb = np.asarray(ma[k]), np.asarray(mb[k])
        scale = np.abs(va).max()
        assert np.abs(va - vb).max() <= 2e-6 * scale, (k, float(np.abs(va - vb).max() / scale))


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_runs_gyration_2d(mods, prec):
    oracle, driver, inputs, B = mods
    say(f"[runs] gyration 2D {prec}")
    wl = inputs.gyration_2d()
    ores = oracle.run_workload(wl)
    p = B.PL_F64 if prec == "f64" else B.PL_F32_OFFSET
    run, st = _run_gpu(driver, wl, wl.steps, True, prec=p, algo=B.PL_ALGO_RUNS)
    assert st == B.PL_OK
    _assert_runs_kernel(run, B)
    if p == B.PL_F64:
        _check_item(run, 0, ores[0], wl, X_TOL, U_TOL, M_TOL)
    else:
        _check_item(run, 0, ores[0], wl, 1e-5, 2e-6, 1e-5, eng=False)
    s = run.sums()[0]
    assert abs(s[0] - 4096.0) < (1e-12 if p == B.PL_F64 else 1e-6) * 4096
    run.close()


def test_runs_cic_fp64(mods):
    oracle, driver, inputs, B = mods
    say("[runs] turbulent 16^3 CIC f64 runs vs oracle")
    wl = _turb(inputs, n=16, steps=3, ragged=5)
    wl.shape = "cic"
    ores = oracle.run_workload(wl)
    run, st = _run_gpu(driver, wl, wl.steps, True, prec=B.PL_F64, algo=B.PL_ALGO_RUNS)
    assert st == B.PL_OK
    _assert_runs_kernel(run, B)
    _check_item(run, 0, ores[0], wl, X_TOL, U_TOL, M_TOL)
    run.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_runs_batched_species(mods, prec):
    """Charged, dust and tracer items plus small boxes: every step is one
    launch of the run kernel that takes each unit with its item's kind
    (pl_part_stats: one run-kernel launch per step, the mixed variant)."""
    oracle, driver, inputs, B = mods
    say(f"[runs] batched species {prec}, one launch per step for every kind")
    wl = _small_batch(inputs)
    ores = oracle.run_workload(wl)
    p = B.PL_F64 if prec == "f64" else B.PL_F32_OFFSET
    run, st = _run_gpu(driver, wl, wl.steps, True, prec=p, algo=B.PL_ALGO_RUNS)
    assert st == B.PL_OK
    _assert_runs_kernel(run, B)
    stats = B.pl_part_stats(run.ctx)
    assert stats[4] == wl.steps and stats[7] >> 12 == 1, stats
    f64 = p == B.PL_F64
    for i in range(len(wl.items)):
        _check_item(run, i, ores[i], wl, X_TOL if f64 else 1e-5, U_TOL if f64 else 2e-5,
                    M_TOL if f64 else 2e-5, eng=f64)
    run.close()


def test_runs_sums_and_graph(mods):
    oracle, driver, inputs, B = mods
    say("[runs] conservation sums and graph replay, f32 runs")
    wl = _small_batch(inputs)
    kw = dict(prec=B.PL_F32_OFFSET, algo=B.PL_ALGO_RUNS)
    eager = driver.Run(wl, **kw)
    graph = driver.Run(wl, **kw)
    eager.sort()
    graph.sort()
    flags = B.PL_FUSE_DEPOSIT | B.PL_ZERO_FIRST | B.PL_SUMS
    for s in range(4):
        eager.step(flags=flags)
        graph.step(flags=flags | B.PL_GRAPH)
        assert graph.sync() == B.PL_OK and eager.sync() == B.PL_OK
        for i in range(len(wl.items)):
            a, b = eager.raw(i), graph.raw(i)
            for k in ("cell", "x", "u"):
                assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), (s, i, k)
            ma, mb = eager.moments(i), graph.moments(i)
            for k in ma:
                va, vb = np.asarray(ma[k]), np.asarray(mb[k])
                assert np.allclose(va, vb, rtol=1e-6, atol=1e-6 * np.abs(va).max()), (s, i, k)
    sums = graph.sums()
    for i, it in enumerate(wl.items):
        sp = wl.species[it.species]
        if sp.kind == "tracer":
            continue
        g, p = sums[i][:8], sums[i][8:]
        expect = (sp.q if sp.kind == "lorentz" else sp.m) * it.particles.n
        assert abs(g[0] - expect) <= 1e-6 * expect and abs(p[0] - expect) <= 1e-6 * expect
    stats = B.pl_part_stats(graph.ctx)
    assert stats[2] == 1 and stats[1] == 4
    _assert_runs_kernel(eager, B)
    eager.close()
    graph.close()


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_sort_first_graph_matches_eager(mods, prec):
    """PL_SORT_FIRST | PL_GRAPH records sort + zeroing + step as one graph
    per buffer set and replays them: over 12 steps with a sort every 3 (the
    two graphs replayed alternately, eager work and synchronisation between
    replays) every step's particle state equals the eager sort-then-step
    sequence bit for bit and its deposits agree to round-off."""
    oracle, driver, inputs, B = mods
    say(f"[runs] sort + zero + step in one graph vs eager, {prec}")
    wl = _small_batch(inputs)
    p = B.PL_F64 if prec == "f64" else B.PL_F32_OFFSET
    kw = dict(prec=p, algo=B.PL_ALGO_RUNS)
    eager = driver.Run(wl, **kw)
    graph = driver.Run(wl, **kw)
    base = B.PL_FUSE_DEPOSIT | B.PL_ZERO_FIRST
    for s in range(12):
        if s % 3 == 0:
            eager.sort()
            eager.step(flags=base)
            graph.step(flags=base | B.PL_GRAPH | B.PL_SORT_FIRST)
        else:
            eager.step(flags=base)
            graph.step(flags=base | B.PL_GRAPH)
        assert eager.sync() == B.PL_OK and graph.sync() == B.PL_OK
        for i in range(len(wl.items)):
            assert eager.items[i].p.cur == graph.items[i].p.cur
            a, b = eager.raw(i), graph.raw(i)
            for k in ("cell", "x", "u", "id"):
                if k in a:
                    assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), (s, i, k)
            ma, mb = eager.moments(i), graph.moments(i)
            for k in ma:
                va, vb = np.asarray(ma[k]), np.asarray(mb[k])
                assert np.allclose(va, vb, rtol=1e-6 if prec == "f32" else 1e-12,
                                   atol=(1e-6 if prec == "f32" else 1e-12) * np.abs(va).max()), (s, i, k)
    st = B.pl_part_stats(graph.ctx)
    # two sort graphs (one per buffer set) and two plain ones; every item sorted 4 times
    assert st[2] == 4 and st[1] == 12 and st[3] == 4 * len(wl.items), st
    eager.close()
    graph.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("rk", [2, 3])
def test_runs_tracers_match_tiled(mods, prec, rk):
    """Tracers in the run kernel (gathers from its LDS field records, the
    grid for stages whose stencil leaves the field tile): per-id states
    bit-identical to the tiled kernel's for both Runge-Kutta options, fast
    enough that stages leave their cell and tile (10 steps, one sort)."""
    oracle, driver, inputs, B = mods
    say(f"[runs] tracers {prec} rk{rk}: run kernel vs tiled kernel")
    n = 16
    nn = (n, n, n)
    flds = inputs.turbulent_fields(nn, 1000 + 9, 2000 + 9, v_rms=3.0)
    rng = np.random.default_rng(3000 + 9)
    npart = 8 * n ** 3 - 7
    x = rng.random((3, npart)) * n
    wl = inputs.Workload(name="tracers", boxes=[inputs.Box(3, nn, {"vg": flds["vg"]})],
                         species=[inputs.Species("tracer", rk_stages=rk)],
                         items=[inputs.Item(0, 0, inputs.make_particles(x, np.zeros((3, npart))))], dt=0.1,
                         steps=10)
    p = B.PL_F64 if prec == "f64" else B.PL_F32_OFFSET
    res = {}
    for algo in (B.PL_ALGO_TILED, B.PL_ALGO_RUNS):
        kmode = B.PL_KEY_TILE_CELL if algo == B.PL_ALGO_TILED else B.PL_KEY_TILE_RUN
        run, st = _run_gpu(driver, wl, wl.steps, True, prec=p, algo=algo, tile=(4, 4, 4), key_mode=kmode)
        assert st in (B.PL_OK, B.PL_ECFL)
        if algo == B.PL_ALGO_RUNS:
            stats = B.pl_part_stats(run.ctx)
            assert stats[4] == wl.steps and stats[5] == 0, stats
        raw = run.raw(0)
        ids = raw["id"].astype(np.int64)
        res[algo] = {k: _cmp.by_id(np.stack(v) if isinstance(v, list) else v, ids) for k, v in raw.items()
                     if k in ("x", "u", "cell")}
        run.close()
    a, b = res[B.PL_ALGO_TILED], res[B.PL_ALGO_RUNS]
    moved = np.abs(a["u"]).max()
    say(f"  largest tracer speed {moved:.2f} cells per unit time")
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_one_launch_matches_per_kind(mods, tmp_path):
    """The batched species workload with every kind in one launch and, from a
    tune cache with one_launch 0, with one launch per kind: per-id particle
    states bit-identical, deposits equal to round-off."""
    oracle, driver, inputs, B = mods
    say("[runs] one launch for every kind vs one launch per kind")
    wl = _small_batch(inputs)
    cache = tmp_path / "per_kind.txt"
    cache.write_text("one_launch 0\n")
    res = []
    for tc in (None, str(cache)):
        run, st = _run_gpu(driver, wl, wl.steps, True, prec=B.PL_F32_OFFSET, algo=B.PL_ALGO_RUNS, tune_cache=tc)
        assert st == B.PL_OK
        stats = B.pl_part_stats(run.ctx)
        # per kind: charged and dust in run kernels, tracers in the tiled kernel
        assert stats[4] == (wl.steps if tc is None else 2 * wl.steps), stats
        out = []
        for i in range(len(wl.items)):
            raw = run.raw(i)
            ids = raw["id"].astype(np.int64)
            out.append(({k: _cmp.by_id(np.stack(v) if isinstance(v, list) else v, ids) for k, v in raw.items()
                         if k in ("x", "u", "cell")}, run.moments(i)))
        res.append(out)
        run.close()
    for i in range(len(wl.items)):
        (sa, ma), (sb, mb) = res[0][i], res[1][i]
        for k in sa:
            assert np.array_equal(sa[k], sb[k]), (i, k)
        for k in ma:
            va, vb = np.asarray(ma[k]), np.asarray(mb[k])
            assert np.abs(va - vb).max() <= 2e-6 * max(np.abs(va).max(), 1e-300), (i, k)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_sparse_tracers(mods, prec):
    """Sparse passive tracers (about 31 per 4^3 tile, most tiles holding a
    few) under the tiled algorithm: per-id states bit-identical to the plain
    algorithm's, and (float64) equal to the oracle's."""
    oracle, driver, inputs, B = mods
    say(f"[runs] sparse tracers {prec}: tiled algorithm vs plain algorithm")
    n = 16
    nn = (n, n, n)
    flds = inputs.turbulent_fields(nn, 1000 + 11, 2000 + 11, v_rms=1.0)
    rng = np.random.default_rng(3000 + 11)
    npart = 2003
    x = rng.random((3, npart)) * n
    wl = inputs.Workload(name="sparse tracers", boxes=[inputs.Box(3, nn, {"vg": flds["vg"]})],
                         species=[inputs.Species("tracer", rk_stages=2)],
                         items=[inputs.Item(0, 0, inputs.make_particles(x, np.zeros((3, npart))))], dt=0.1,
                         steps=5)
    p = B.PL_F64 if prec == "f64" else B.PL_F32_OFFSET
    res = {}
    for algo in (B.PL_ALGO_TILED, B.PL_ALGO_PLAIN):
        kmode = B.PL_KEY_TILE_CELL if algo == B.PL_ALGO_TILED else B.PL_KEY_TILE
        run, st = _run_gpu(driver, wl, wl.steps, algo != B.PL_ALGO_PLAIN, prec=p, algo=algo, tile=(4, 4, 4),
                           key_mode=kmode)
        assert st in (B.PL_OK, B.PL_ECFL)
        raw = run.raw(0)
        ids = raw["id"].astype(np.int64)
        res[algo] = {k: _cmp.by_id(np.stack(v) if isinstance(v, list) else v, ids) for k, v in raw.items()
                     if k in ("x", "u", "cell")}
        if algo == B.PL_ALGO_TILED and prec == "f64":
            ores = oracle.run_workload(wl)
            _check_item(run, 0, ores[0], wl, X_TOL, U_TOL, M_TOL, eng=False)
        run.close()
    a, b = res[B.PL_ALGO_TILED], res[B.PL_ALGO_PLAIN]
    for k in a:
        assert np.array_equal(a[k], b[k]), k
