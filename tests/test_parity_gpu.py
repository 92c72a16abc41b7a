"""Parity of the HIP path (through the C ABI) with the float64 CPU oracle.

Element by element per particle id and per cell, on seeded inputs that span
several tiles and end in a ragged tail.  Tolerances (float64 path):
positions 1e-11 cells (minimum image), velocities 1e-12 * max(|u|, sigma),
deposits 1e-12 * A_c per cell and channel (A_c = sum over particles of
|mu| W, the scale of the round-off of the sum), except the energy channel,
whose per-particle value m w c^2 (gamma_new - gamma_old)/dt carries the
cancellation of two gammas: there the bound adds 8 ulp(gamma)/dt times the
mass deposited in the cell.
"""

import math
import sys

import numpy as np
import pytest

from tests import _cmp

pytestmark = pytest.mark.gpu

U_TOL = 1e-12
X_TOL = 1e-11
M_TOL = 1e-12


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


def _run_gpu(driver, wl, steps, sort_first, sort_every=0, **kw):
    run = driver.Run(wl, **kw)
    if sort_first:
        run.sort()
    for s in range(steps):
        if sort_every and s > 0 and s % sort_every == 0:
            run.sort()
        run.step()
    st = run.sync()
    return run, st


def _check_item(run, i, ores, wl, x_tol, u_tol, m_tol, eng=True):
    box = wl.boxes[wl.items[i].box]
    gx, gu, gid, st = run.state(i)
    ex, eu = _cmp.state_errors(gx, gu, gid, ores["x"], ores["u"], box.n, box.ndim)
    assert ex <= x_tol, f"item {i}: position error {ex}"
    assert eu <= u_tol, f"item {i}: velocity error {eu}"
    if ores["moments"] is None:
        return ex, eu, {}
    gm = run.moments(i)
    errs = _cmp.moment_errors(gm, ores["moments"], ores["abs"])
    for name, (mx, rms, rel) in errs.items():
        if name == "eng":
            continue
        assert mx <= m_tol, f"item {i} channel {name}: {mx} > {m_tol} of A_c"
    if eng and "eng" in gm:
        sp = wl.species[wl.items[i].species]
        d = np.abs(gm["eng"] - ores["moments"]["eng"])
        bound = m_tol * ores["abs"]["eng"] + 8 * 2.0 ** -53 * 1.2 / wl.dt * (sp.m / abs(sp.q)) * ores["abs"]["rho"]
        assert (d <= bound + 1e-300).all(), f"item {i}: energy channel off by {float((d / (bound + 1e-300)).max())} of bound"
    return ex, eu, errs


# ---------------------------------------------------------------- gyration (2D)

@pytest.mark.parametrize("algo", ["plain", "tiled"])
def test_gyration_2d_fp64(mods, algo):
    oracle, driver, inputs, B = mods
    say(f"[parity] gyration 2D 32^2, 4096 particles, 10 steps, f64 {algo}")
    wl = inputs.gyration_2d()
    ores = oracle.run_workload(wl)
    a = B.PL_ALGO_TILED if algo == "tiled" else B.PL_ALGO_PLAIN
    run, st = _run_gpu(driver, wl, wl.steps, sort_first=(a == B.PL_ALGO_TILED), prec=B.PL_F64, algo=a)
    assert st == B.PL_OK
    _check_item(run, 0, ores[0], wl, X_TOL, U_TOL, M_TOL)
    # charge conservation: sum_cells rho dV = sum_p q w = 4096
    s = run.sums()[0]
    assert abs(s[0] - 4096.0) < 1e-12 * 4096
    run.close()


def test_gyration_2d_f32_offset(mods):
    oracle, driver, inputs, B = mods
    say("[parity] gyration 2D, f32+offset tiled vs f64 oracle")
    wl = inputs.gyration_2d()
    ores = oracle.run_workload(wl)
    run, st = _run_gpu(driver, wl, wl.steps, True, prec=B.PL_F32_OFFSET, algo=B.PL_ALGO_TILED)
    assert st == B.PL_OK
    ex, eu, errs = _check_item(run, 0, ores[0], wl, 1e-5, 2e-6, 1e-5, eng=False)
    say(f"  f32 gyration: x {ex:.2e} u {eu:.2e} " + " ".join(f"{k}:{v[0]:.1e}" for k, v in errs.items()))
    run.close()


# ---------------------------------------------------------------- turbulent (3D)

def _turb(inputs, n=32, steps=5, ragged=37):
    return inputs.turbulent_box(n=n, npart=8 * n ** 3 - ragged, steps=steps)


@pytest.mark.parametrize("algo", ["plain", "tiled"])
def test_turbulent_fp64(mods, algo):
    oracle, driver, inputs, B = mods
    say(f"[parity] turbulent 32^3, 262107 particles, 5 steps, f64 {algo}")
    wl = _turb(inputs)
    ores = oracle.run_workload(wl)
    a = B.PL_ALGO_TILED if algo == "tiled" else B.PL_ALGO_PLAIN
    run, st = _run_gpu(driver, wl, wl.steps, sort_first=(a == B.PL_ALGO_TILED), prec=B.PL_F64, algo=a)
    assert st == B.PL_OK
    _check_item(run, 0, ores[0], wl, X_TOL, U_TOL, M_TOL)
    run.close()


def test_turbulent_fp64_cic(mods):
    oracle, driver, inputs, B = mods
    say("[parity] turbulent 16^3 CIC, f64 plain and tiled")
    wl = _turb(inputs, n=16, steps=3, ragged=5)
    wl.shape = "cic"
    ores = oracle.run_workload(wl)
    for a in (B.PL_ALGO_PLAIN, B.PL_ALGO_TILED):
        run, st = _run_gpu(driver, wl, wl.steps, sort_first=(a == B.PL_ALGO_TILED), prec=B.PL_F64, algo=a)
        assert st == B.PL_OK
        _check_item(run, 0, ores[0], wl, X_TOL, U_TOL, M_TOL)
        run.close()


def test_turbulent_f32_error_table(mods):
    """The precision form against the float64 oracle after 20 steps: max and
    RMS error of every particle quantity and deposited channel."""
    oracle, driver, inputs, B = mods
    say("[parity] turbulent 32^3, 20 steps, f32+offset tiled vs f64 oracle (error table)")
    wl = _turb(inputs, steps=20)
    ores = oracle.run_workload(wl)
    run, st = _run_gpu(driver, wl, wl.steps, True, prec=B.PL_F32_OFFSET, algo=B.PL_ALGO_TILED)
    assert st == B.PL_OK
    gx, gu, gid, _ = run.state(0)
    box = wl.boxes[0]
    table = _cmp.state_error_stats(gx, gu, gid, ores[0]["x"], ores[0]["u"], box.n, 3)
    merr = _cmp.moment_errors(run.moments(0), ores[0]["moments"], ores[0]["abs"])
    for k, (mx, rms) in table.items():
        say(f"  {k:4s} max {mx:.3e} rms {rms:.3e}")
    for k, (mx, rms, rel) in merr.items():
        say(f"  {k:4s} max/A_c {mx:.3e} rms/A_c {rms:.3e} max/max|M| {rel:.3e}")
    bad = _cmp.check_fp32_table(table, merr)
    assert not bad, bad
    run.close()


# ---------------------------------------------------------------- sort

@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("key_mode", [0, 1, 2])
def test_sort_bitexact(mods, prec, key_mode):
    oracle, driver, inputs, B = mods
    say(f"[parity] sort {prec} key_mode {key_mode}")
    for n, npart, tile in ((32, 8 * 32 ** 3 - 37, (8, 8, 8)), (16, 1, (4, 4, 4)), (16, 3001, (16, 8, 2))):
        wl = inputs.turbulent_box(n=n, npart=npart, steps=0)
        p = B.PL_F64 if prec == "f64" else B.PL_F32_OFFSET
        run = driver.Run(wl, prec=p, algo=B.PL_ALGO_TILED, key_mode=key_mode, tile=tile)
        run.sort()
        assert run.sync() == B.PL_OK
        raw = run.raw(0)
        x = wl.items[0].particles.x
        bx = wl.boxes[0].n
        if p == B.PL_F64:
            cells = oracle.cells_of_positions(3, bx, x)
        else:
            cells, _ = oracle.split_positions(3, bx, x)
        if key_mode == 2:
            keys, rb = oracle.rank_keys(3, bx, tile, cells)
        else:
            keys = np.array([oracle.tile_key(3, bx, tile, key_mode, *cells[:, q]) for q in range(npart)],
                            dtype=np.uint32)
        perm = oracle.stable_sort_perm(keys)
        assert np.array_equal(raw["id"].astype(np.int64), perm)
        ntiles = (n // tile[0]) * (n // tile[1]) * (n // tile[2])
        per_tile = tile[0] * tile[1] * tile[2]
        if key_mode == 2:
            tkeys = keys[perm] >> (rb + int(per_tile - 1).bit_length())
        else:
            tkeys = keys[perm] // (per_tile if key_mode == 1 else 1)
        expect = np.searchsorted(tkeys, np.arange(ntiles + 1), side="left")
        assert np.array_equal(raw["tile_start"][: ntiles + 1], expect)
        # every array moved with the permutation
        gx, gu, gid, _ = run.state(0)
        ex, eu = _cmp.state_errors(gx, gu, gid, x, wl.items[0].particles.u, wl.boxes[0].n, 3)
        assert ex <= (0 if p == B.PL_F64 else 1e-6) and eu <= (0 if p == B.PL_F64 else 1e-7)
        run.close()


@pytest.mark.parametrize("key_mode", [1, 2])
def test_sort_bitexact_wide_keys(mods, key_mode):
    """Keys of 21 and 31 bits (128^3 box, 8^3 tiles: three and four radix
    passes, the last one narrower) and a tile whose sides are not powers of
    two (the rank-interleaved key splits tile and cell by division): the
    permutation and the tile offsets are the oracle's, bit for bit."""
    oracle, driver, inputs, B = mods
    say(f"[parity] sort with wide keys, key_mode {key_mode}")
    for n, npart, tile in ((128, (1 << 18) + 3, (8, 8, 8)), (48, 48 ** 3 + 7, (6, 4, 3))):
        wl = inputs.turbulent_box(n=n, npart=npart, steps=0)
        run = driver.Run(wl, prec=B.PL_F64, algo=B.PL_ALGO_TILED, key_mode=key_mode, tile=tile)
        run.sort()
        assert run.sync() == B.PL_OK
        raw = run.raw(0)
        bx = wl.boxes[0].n
        cells = oracle.cells_of_positions(3, bx, wl.items[0].particles.x)
        if key_mode == 2:
            keys, rb = oracle.rank_keys(3, bx, tile, cells)
        else:
            keys = np.array([oracle.tile_key(3, bx, tile, key_mode, *cells[:, q]) for q in range(npart)],
                            dtype=np.uint32)
        say(f"  n {n} tile {tile}: keys up to {int(keys.max()).bit_length()} bits")
        perm = oracle.stable_sort_perm(keys)
        assert np.array_equal(raw["id"].astype(np.int64), perm)
        ntiles = (n // tile[0]) * (n // tile[1]) * (n // tile[2])
        per_tile = tile[0] * tile[1] * tile[2]
        if key_mode == 2:
            tkeys = keys[perm] >> (rb + int(per_tile - 1).bit_length())
        else:
            tkeys = keys[perm] // per_tile
        expect = np.searchsorted(tkeys, np.arange(ntiles + 1), side="left")
        assert np.array_equal(raw["tile_start"][: ntiles + 1], expect)
        run.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_rank_key_tile_not_power_of_two(mods, prec):
    """The tiled kernel on particles in rank-interleaved order with a 6x4x3
    tile (72 cells per tile), 24^3 box, sorted every 2 of 6 steps: per-id
    states bit-identical to the plain kernel's, deposits within the
    precision's tolerance of them."""
    oracle, driver, inputs, B = mods
    say(f"[parity] {prec} tiled kernel, rank key, tile (6, 4, 3) vs plain kernel")
    wl = inputs.turbulent_box(n=24, npart=8 * 24 ** 3 - 29, steps=6)
    p = B.PL_F64 if prec == "f64" else B.PL_F32_OFFSET
    res = []
    for algo, tile, km in ((B.PL_ALGO_PLAIN, None, 0), (B.PL_ALGO_TILED, (6, 4, 3), B.PL_KEY_TILE_RANK)):
        run, st = _run_gpu(driver, wl, wl.steps, algo == B.PL_ALGO_TILED, sort_every=2 if tile else 0, prec=p,
                           algo=algo, tile=tile, key_mode=km)
        assert st == B.PL_OK
        raw = run.raw(0)
        ids = raw["id"].astype(np.int64)
        res.append(({k: _cmp.by_id(np.stack(v) if isinstance(v, list) else v, ids) for k, v in raw.items()
                     if k in ("x", "u", "cell")}, run.moments(0)))
        run.close()
    (sa, ma), (sb, mb) = res
    for k in sa:
        assert np.array_equal(sa[k], sb[k]), k
    rtol = 1e-12 if p == B.PL_F64 else 2e-6
    for k in ma:
        va, vb = np.asarray(ma[k]), np.asarray(mb[k])
        assert np.abs(va - vb).max() <= rtol * np.abs(va).max(), k


@pytest.mark.parametrize("nn,ppc", [((40, 24, 16), 8), ((1024, 8, 8), 2)])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_non_cubic_box(mods, prec, nn, ppc):
    """A 40x24x16 box (every extent different, so a swapped dimension
    anywhere shows) and a 1024x8x8 box (the largest extent the float32
    form's packed cell holds, particles wrapping from cell 1023 to 0),
    sorted every 2 of 4 steps: float64 plain, tiled and run-based kernels
    against the oracle; float32 tiled and run-based kernels with per-id
    states bit-identical to the float32 plain kernel and deposits within
    2e-6 of its largest value."""
    oracle, driver, inputs, B = mods
    wl = inputs.turbulent_box(n=nn, npart=ppc * nn[0] * nn[1] * nn[2] - 7, steps=4)
    if nn[0] == 1024:
        wl.dt = 1.0          # about 0.05 cells per step: a few dozen particles cross x = 1024
    p = B.PL_F64 if prec == "f64" else B.PL_F32_OFFSET
    # the run kernel's float64 LDS tiles fit 8x8x4 tiles, its float32 ones 8^3
    configs = ((B.PL_ALGO_PLAIN, None, B.PL_KEY_TILE), (B.PL_ALGO_TILED, (8, 8, 4), B.PL_KEY_TILE_CELL),
               (B.PL_ALGO_RUNS, (8, 8, 4) if prec == "f64" else (8, 8, 8), B.PL_KEY_TILE_RUN))
    ores = oracle.run_workload(wl) if prec == "f64" else None
    ref = None
    for algo, tile, km in configs:
        say(f"[parity] {prec} box {nn} algo {algo} tile {tile}")
        run, st = _run_gpu(driver, wl, wl.steps, tile is not None, sort_every=2 if tile else 0, prec=p, algo=algo,
                           tile=tile, key_mode=km)
        assert st == B.PL_OK
        if algo == B.PL_ALGO_RUNS:
            stats = B.pl_part_stats(run.ctx)
            assert stats[4] > 0 and stats[5] == 0, stats
        if prec == "f64":
            _check_item(run, 0, ores[0], wl, X_TOL, U_TOL, M_TOL)
            if nn[0] == 1024 and algo == B.PL_ALGO_PLAIN:
                x0 = wl.items[0].particles.x[0]
                crossed = int(np.count_nonzero(np.abs(ores[0]["x"][0] - x0) > nn[0] / 2))
                say(f"  {crossed} particles crossed x = {nn[0]}")
                assert crossed > 0
        else:
            raw = run.raw(0)
            ids = raw["id"].astype(np.int64)
            cur = ({k: _cmp.by_id(np.stack(v) if isinstance(v, list) else v, ids) for k, v in raw.items()
                    if k in ("x", "u", "cell")}, run.moments(0))
            if ref is None:
                ref = cur
            else:
                for k in cur[0]:
                    assert np.array_equal(cur[0][k], ref[0][k]), (algo, k)
                for k in cur[1]:
                    va, vb = np.asarray(ref[1][k]), np.asarray(cur[1][k])
                    assert np.abs(va - vb).max() <= 2e-6 * np.abs(va).max(), (algo, k)
        run.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_non_square_2d(mods, prec):
    """A 48x16 2D box with turbulent in-plane fields, sorted every 2 of 6
    steps: float64 plain, tiled and run-based kernels (8x8 tiles) against the
    oracle; float32 tiled and run-based kernels with per-id states
    bit-identical to the float32 plain kernel and deposits within 2e-6 of
    its largest value."""
    oracle, driver, inputs, B = mods
    wl = inputs.turbulent_2d(n=(48, 16), npart=6000 - 5, steps=6)
    p = B.PL_F64 if prec == "f64" else B.PL_F32_OFFSET
    configs = ((B.PL_ALGO_PLAIN, None, B.PL_KEY_TILE), (B.PL_ALGO_TILED, (8, 8, 1), B.PL_KEY_TILE_CELL),
               (B.PL_ALGO_RUNS, (8, 8, 1), B.PL_KEY_TILE_RUN))
    ores = oracle.run_workload(wl) if prec == "f64" else None
    ref = None
    for algo, tile, km in configs:
        say(f"[parity] {prec} 2D 48x16 algo {algo} tile {tile}")
        run, st = _run_gpu(driver, wl, wl.steps, tile is not None, sort_every=2 if tile else 0, prec=p, algo=algo,
                           tile=tile, key_mode=km)
        assert st == B.PL_OK
        if algo == B.PL_ALGO_RUNS:
            stats = B.pl_part_stats(run.ctx)
            assert stats[4] > 0 and stats[5] == 0, stats
        if prec == "f64":
            _check_item(run, 0, ores[0], wl, X_TOL, U_TOL, M_TOL)
        else:
            raw = run.raw(0)
            ids = raw["id"].astype(np.int64)
            cur = ({k: _cmp.by_id(np.stack(v) if isinstance(v, list) else v, ids) for k, v in raw.items()
                    if k in ("x", "u", "cell")}, run.moments(0))
            if ref is None:
                ref = cur
            else:
                for k in cur[0]:
                    assert np.array_equal(cur[0][k], ref[0][k]), (algo, k)
                for k in cur[1]:
                    va, vb = np.asarray(ref[1][k]), np.asarray(cur[1][k])
                    assert np.abs(va - vb).max() <= 2e-6 * np.abs(va).max(), (algo, k)
        run.close()


def test_sort_invariance(mods):
    """The per-particle state does not depend on tile size, key mode or sort
    cadence, bit for bit (the push of a particle reads only fields)."""
    oracle, driver, inputs, B = mods
    say("[parity] sort invariance of per-id state (f64 and f32)")
    wl = _turb(inputs, n=32, steps=6)
    for prec in (B.PL_F64, B.PL_F32_OFFSET):
        ref = None
        if prec == B.PL_F64:
            configs = [(B.PL_ALGO_PLAIN, None, 0, 0), (B.PL_ALGO_TILED, (8, 4, 4), 0, 0),
                       (B.PL_ALGO_TILED, (4, 4, 8), 1, 2), (B.PL_ALGO_TILED, (8, 8, 2), 0, 1),
                       (B.PL_ALGO_TILED, (8, 8, 4), 2, 3)]
        else:
            configs = [(B.PL_ALGO_PLAIN, None, 0, 0), (B.PL_ALGO_TILED, (8, 8, 8), 0, 0),
                       (B.PL_ALGO_TILED, (4, 8, 16), 1, 2), (B.PL_ALGO_TILED, (16, 8, 2), 0, 1),
                       (B.PL_ALGO_TILED, (8, 8, 8), 2, 3)]
        for algo, tile, km, every in configs:
            run, st = _run_gpu(driver, wl, wl.steps, algo == B.PL_ALGO_TILED, sort_every=every, prec=prec,
                               algo=algo, tile=tile, key_mode=km)
            assert st == B.PL_OK
            raw = run.raw(0)
            ids = raw["id"].astype(np.int64)
            cur = {k: _cmp.by_id(np.stack(v) if isinstance(v, list) else v, ids) for k, v in raw.items()
                   if k in ("x", "u", "cell")}
            if ref is None:
                ref = cur
            else:
                for k in cur:
                    assert np.array_equal(cur[k], ref[k]), (prec, tile, km, every, k)
            run.close()


# ---------------------------------------------------------------- species kinds, batching

def _small_batch(inputs):
    return inputs.batched(n_main=16, n_cr=20000, n_dust=9000, n_tracer=3001, n_small=8, n_boxes=3,
                          small_lo=50, small_hi=3000, steps=4)


@pytest.mark.parametrize("form", ["f64-plain", "f64-tiled", "f32-tiled"])
def test_batched_species(mods, form):
    oracle, driver, inputs, B = mods
    say(f"[parity] batched species (charged, dust, tracer + small boxes), {form}")
    wl = _small_batch(inputs)
    ores = oracle.run_workload(wl)
    prec = B.PL_F64 if form.startswith("f64") else B.PL_F32_OFFSET
    algo = B.PL_ALGO_PLAIN if form.endswith("plain") else B.PL_ALGO_TILED
    run, st = _run_gpu(driver, wl, wl.steps, algo == B.PL_ALGO_TILED, prec=prec, algo=algo)
    assert st == B.PL_OK
    f64 = prec == B.PL_F64
    for i in range(len(wl.items)):
        _check_item(run, i, ores[i], wl, X_TOL if f64 else 1e-5, U_TOL if f64 else 2e-5,
                    M_TOL if f64 else 2e-5, eng=f64)
    run.close()


def test_graph_replay_matches_eager(mods):
    oracle, driver, inputs, B = mods
    say("[parity] hipGraph replay vs eager, batched f32 tiled")
    wl = _small_batch(inputs)
    kw = dict(prec=B.PL_F32_OFFSET, algo=B.PL_ALGO_TILED)
    eager = driver.Run(wl, **kw)
    graph = driver.Run(wl, **kw)
    eager.sort()
    graph.sort()
    for s in range(5):
        eager.step()
        graph.step(flags=B.PL_FUSE_DEPOSIT | B.PL_ZERO_FIRST | B.PL_GRAPH)
        # eager work and a synchronisation between replays
        graph.sync()
        for i in range(len(wl.items)):
            a, b = eager.raw(i), graph.raw(i)
            for k in ("cell", "x", "u"):
                assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), (s, i, k)
            ma, mb = eager.moments(i), graph.moments(i)
            for k in ma:
                va = np.asarray(ma[k])
                vb = np.asarray(mb[k])
                # float32 LDS sums: the order of the atomic adds may differ
                assert np.allclose(va, vb, rtol=1e-6, atol=1e-6 * np.abs(va).max()), (s, i, k)
    stats = B.pl_part_stats(graph.ctx)
    assert stats[2] == 1 and stats[1] == 5      # one recording, five replays
    eager.close()
    graph.close()


def test_conservation_sums(mods):
    oracle, driver, inputs, B = mods
    say("[parity] conservation sums (grid vs particle side)")
    wl = _small_batch(inputs)
    # scale of each sum: sum over particles of |mu| (the oracle's one-step A_c summed over cells)
    ref = oracle.run_workload(wl, steps=1)
    for prec, tol in ((B.PL_F64, 1e-12), (B.PL_F32_OFFSET, 1e-6)):
        run = driver.Run(wl, prec=prec, algo=B.PL_ALGO_TILED)
        run.sort()
        run.step(flags=B.PL_FUSE_DEPOSIT | B.PL_ZERO_FIRST | B.PL_SUMS)
        assert run.sync() == B.PL_OK
        sums = run.sums()
        for i, it in enumerate(wl.items):
            sp = wl.species[it.species]
            if sp.kind == "tracer":
                continue
            g, p = sums[i][:8], sums[i][8:]
            npart = it.particles.n
            expect_rho = (sp.q if sp.kind == "lorentz" else sp.m) * npart
            assert abs(g[0] - expect_rho) <= tol * expect_rho
            assert abs(p[0] - expect_rho) <= tol * expect_rho
            chans = range(1, 8) if sp.kind == "lorentz" else range(4, 7)
            ab = ref[i]["abs"]
            flat = [ab["rho"], *(ab["J"] or [None] * 3), *ab["F"], ab["eng"]]
            for ch in chans:
                scale = float(flat[ch].sum())
                assert abs(g[ch] - p[ch]) <= tol * scale, (prec, i, ch, g[ch], p[ch], scale)
        run.close()


# ---------------------------------------------------------------- edge cases

def test_edge_cases(mods):
    oracle, driver, inputs, B = mods
    say("[parity] edge cases: empty item, single particle on faces and at the seam")
    wl = _small_batch(inputs)
    # item 3 becomes empty, item 4 a single particle exactly on a cell face at the seam
    wl.items[3].particles = inputs.make_particles(np.zeros((3, 0)), np.zeros((3, 0)))
    x = np.array([[0.0], [7.5], [3.0]])
    u = np.array([[-0.03], [0.02], [0.01]])
    wl.items[4].particles = inputs.make_particles(x, u)
    ores = oracle.run_workload(wl)
    for prec, algo in ((B.PL_F64, B.PL_ALGO_PLAIN), (B.PL_F64, B.PL_ALGO_TILED), (B.PL_F32_OFFSET, B.PL_ALGO_TILED),
                       (B.PL_F64, B.PL_ALGO_RUNS), (B.PL_F32_OFFSET, B.PL_ALGO_RUNS)):
        run, st = _run_gpu(driver, wl, wl.steps, algo != B.PL_ALGO_PLAIN, prec=prec, algo=algo)
        assert st == B.PL_OK
        f64 = prec == B.PL_F64
        for i in (3, 4):
            _check_item(run, i, ores[i], wl, X_TOL if f64 else 1e-5, U_TOL if f64 else 2e-5,
                        M_TOL if f64 else 2e-5, eng=f64)
        run.close()


def test_latched_conditions(mods):
    """A step that moves particles a full cell is reported as PL_ECFL by the
    next sync; a non-finite coordinate as PL_ENONFINITE; both still leave
    every index in range."""
    oracle, driver, inputs, B = mods
    say("[parity] latched CFL / non-finite conditions")
    n = (8, 8, 8)
    x = np.array([[1.5, 2.5], [1.5, 2.5], [1.5, 2.5]])
    u = np.zeros((3, 2))
    wl = inputs.Workload(name="cfl", boxes=[inputs.Box(3, n, inputs.uniform_fields(n, vg=(3.0, 0.0, 0.0)))],
                         species=[inputs.Species("tracer")], items=[inputs.Item(0, 0, inputs.make_particles(x, u))],
                         dt=0.5, steps=1)
    for prec in (B.PL_F64, B.PL_F32_OFFSET):
        run = driver.Run(wl, prec=prec, algo=B.PL_ALGO_PLAIN)
        run.step(flags=0)
        assert run.sync() == B.PL_ECFL
        assert run.sync() == B.PL_OK            # cleared
        gx, _, _, _ = run.state(0)
        assert ((gx >= 0) & (gx < 8)).all()
        run.close()
    xbad = np.array([[np.nan, 2.5], [1.5, 2.5], [1.5, 2.5]])
    wl.items[0].particles = inputs.make_particles(xbad, u)
    wl.boxes[0].fields = inputs.uniform_fields(n, vg=(0.1, 0.0, 0.0))
    for prec in (B.PL_F64, B.PL_F32_OFFSET):
        run = driver.Run(wl, prec=prec, algo=B.PL_ALGO_PLAIN)
        assert run.load_status == B.PL_ENONFINITE      # reported by pl_part_pack
        run.step(flags=0)
        assert run.sync() == B.PL_OK                  # the stored coordinate was replaced by 0
        gx, _, _, _ = run.state(0)
        assert np.isfinite(gx).all() and ((gx >= 0) & (gx < 8)).all()
        run.close()


def test_invalid_items_rejected(mods):
    oracle, driver, inputs, B = mods
    say("[parity] invalid items rejected before device work")
    wl = _small_batch(inputs)
    run = driver.Run(wl, prec=B.PL_F64, algo=B.PL_ALGO_PLAIN)
    items = run.items
    saved = B.pl_item()
    import ctypes as C
    C.pointer(saved)[0] = items[1]
    # dust item with a current channel
    items[1].m.J[0] = items[0].m.J[0]
    items[1].m.J[1] = items[0].m.J[1]
    items[1].m.J[2] = items[0].m.J[2]
    assert B.pl_part_gather_push(run.ctx, items, 0.05, B.PL_FUSE_DEPOSIT, check=False) == B.PL_EINVAL
    items[1] = saved
    # misaligned particle pointer
    items[0].p.u[0][1] = items[0].p.u[0][1] + 4
    assert B.pl_part_gather_push(run.ctx, items, 0.05, 0, check=False) == B.PL_EINVAL
    items[0].p.u[0][1] = items[0].p.u[0][1] - 4
    # bad dt, bad cur, unknown flag
    assert B.pl_part_gather_push(run.ctx, items, float("nan"), 0, check=False) == B.PL_EINVAL
    assert B.pl_part_gather_push(run.ctx, items, 0.05, 1 << 7, check=False) == B.PL_EINVAL
    items[0].p.cur = 2
    assert B.pl_part_gather_push(run.ctx, items, 0.05, 0, check=False) == B.PL_EINVAL
    items[0].p.cur = 0
    # graph on the null stream
    B.pl_part_set_stream(run.ctx, None)
    assert B.pl_part_gather_push(run.ctx, items, 0.05, B.PL_GRAPH, check=False) == B.PL_EINVAL
    B.pl_part_set_stream(run.ctx, run.stream.cuda_stream)
    # the valid call still works afterwards
    assert B.pl_part_gather_push(run.ctx, items, 0.05, B.PL_FUSE_DEPOSIT | B.PL_ZERO_FIRST, check=False) == B.PL_OK
    assert run.sync() == B.PL_OK
    run.close()


# ---------------------------------------------------------------- full size, bench configuration

def _sampled_cells_check(oracle, wl, gm, steps, ncells=48, seed=12, margin=2.0):
    """Deposits at sampled cells against the oracle: the particles whose
    initial position lies within `margin` cells of a sampled cell (every
    particle that can reach its stencil in `steps` steps at the workload's
    speeds) are advanced by the oracle; the last step deposits.  Returns the
    largest error per channel relative to the oracle's A_c at that cell."""
    box = wl.boxes[0]
    n = box.n[0]
    rng = np.random.default_rng(seed)
    cells = rng.integers(0, n, size=(ncells, 3))
    it = wl.items[0].particles
    x = it.x
    mark = np.zeros((n, n, n), dtype=bool)
    r = int(np.ceil(margin))
    off = np.arange(-r, r + 1)
    for c in cells:
        mark[np.ix_((c[2] + off) % n, (c[1] + off) % n, (c[0] + off) % n)] = True
    ci = np.floor(x).astype(np.int64) % n
    near = mark[ci[2], ci[1], ci[0]]
    xs = np.ascontiguousarray(x[:, near])
    us = np.ascontiguousarray(it.u[:, near])
    ws = np.ascontiguousarray(it.w[near])
    sp = (oracle.LORENTZ, 1.0, 1.0, 0.0)
    for _ in range(steps - 1):
        oracle.step(3, box.n, oracle.TSC, sp, xs, us, ws, box.fields, wl.dt)
    mom = oracle.new_moments(box.n, oracle.LORENTZ)
    ab = oracle.new_moments(box.n, oracle.LORENTZ)
    oracle.step(3, box.n, oracle.TSC, sp, xs, us, ws, box.fields, wl.dt, moments=mom, abs_moments=ab)
    worst = {}
    for name in ("rho", "J", "F"):
        ref = mom[name] if name == "rho" else np.stack(mom[name])
        scale = ab[name] if name == "rho" else np.stack(ab[name])
        got = np.asarray(gm[name]) if name == "rho" else np.stack(gm[name])
        e = 0.0
        for c in cells:
            idx = (..., c[2], c[1], c[0])
            e = max(e, float((np.abs(got[idx] - ref[idx]) / np.maximum(scale[idx], 1e-300)).max()))
        worst[name] = e
    return worst


@pytest.mark.parametrize("path", ["f32_runs", "f32_tiled", "f64_plain", "f64_tiled"])
def test_fullsize_sampled(mods, path):
    """128^3 turbulent box, 2^24 particles, 20 steps, in the launch
    configuration the benchmark times (sorted paths re-sort every
    SORT_EVERY steps).  The oracle advances a sample of 2048 particles (a
    particle's update reads only the fields) and they are compared per id;
    the deposit is compared at 48 sampled cells (the oracle advances every
    particle that can reach them) and through conservation: total charge
    equals the particle count, and the grid sums of J and F equal the
    particle-side sums."""
    oracle, driver, inputs, B = mods
    from paper_2602_23434_amd import benchcfg as BC
    say(f"[parity] full size 128^3, 2^24 particles, 20 steps, {path} (bench configuration)")
    wl = inputs.turbulent_box(n=BC.TURB_N, npart=BC.TURB_NP, steps=20)
    cfg = {"f32_runs": BC.headline(), "f32_tiled": dict(BC.F32_TILED, sort_every=BC.SORT_EVERY),
           "f64_plain": BC.F64_PLAIN, "f64_tiled": dict(BC.F64_TILED, sort_every=BC.SORT_EVERY)}[path]
    run = driver.Run(wl, **BC.run_kwargs(cfg))
    sorted_path = cfg["algo"] != B.PL_ALGO_PLAIN
    for s in range(wl.steps):
        # the benchmark's sequence: a sorting step is one graph (sort, zero, step)
        fl = BC.STEP_FLAGS | (B.PL_SUMS if s == wl.steps - 1 else 0)
        if sorted_path and s % cfg["sort_every"] == 0:
            fl |= B.PL_SORT_FIRST
        run.step(flags=fl)
    assert run.sync() == B.PL_OK
    if path == "f32_runs":
        st = B.pl_part_stats(run.ctx)
        assert st[4] > 0 and st[5] == 0, st
    gx, gu, gid, _ = run.state(0)
    gm = run.moments(0)
    sums = run.sums()[0]
    run.close()
    rng = np.random.default_rng(11)
    sample = np.sort(rng.choice(BC.TURB_NP, 2048, replace=False))
    it = wl.items[0].particles
    x = np.ascontiguousarray(it.x[:, sample])
    u = np.ascontiguousarray(it.u[:, sample])
    w = np.ascontiguousarray(it.w[sample])
    box = wl.boxes[0]
    for _ in range(wl.steps):
        oracle.step(3, box.n, oracle.TSC, (oracle.LORENTZ, 1.0, 1.0, 0.0), x, u, w, box.fields, wl.dt)
    order = np.argsort(gid)
    gxs, gus = gx[:, order][:, sample], gu[:, order][:, sample]
    dx = np.abs(_cmp.min_image(gxs - x, 128)).max()
    du = (np.sqrt(((gus - u) ** 2).sum(axis=0)) / np.maximum(np.sqrt((u * u).sum(axis=0)), 0.05)).max()
    say(f"  sampled max |dx| {dx:.3e} cells, max |du|/max(|u|,sigma) {du:.3e}")
    f64 = path.startswith("f64")
    if f64:
        assert dx <= X_TOL and du <= U_TOL
    else:
        assert dx <= 2e-5 and du <= 2e-5
    worst = _sampled_cells_check(oracle, wl, gm, wl.steps)
    say("  sampled cells, max error / A_c: " + " ".join(f"{k} {v:.2e}" for k, v in worst.items()))
    for k, v in worst.items():
        assert v <= (M_TOL if f64 else 2e-5), k
    tol = 1e-12 if f64 else 1e-6
    assert abs(sums[0] - BC.TURB_NP) <= tol * BC.TURB_NP
    for ch in range(1, 7):
        assert abs(sums[ch] - sums[8 + ch]) <= tol * max(abs(sums[8 + ch]), 1e-3 * BC.TURB_NP * 0.05), ch
