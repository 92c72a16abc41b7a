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


def expected_order(counts):
    """Tiles with more than twice the mean run count first (by decreasing
    count, ties by index; at most 1024 of them, the first in index order),
    then the others in index order."""
    ntiles = len(counts)
    thr = 2 * (int(counts.sum()) // max(ntiles, 1)) + 1
    heavy = [t for t in range(ntiles) if counts[t] > thr][:1024]
    hs = set(heavy)
    ranked = sorted(heavy, key=lambda t: (-counts[t], t))
    return np.array(ranked + [t for t in range(ntiles) if t not in hs], dtype=np.int64)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_runs_table_exact(mods, prec):
    oracle, driver, inputs, B = mods
    for n, npart, tile in ((32, 8 * 32 ** 3 - 37, (8, 8, 8)), (16, 1, (4, 4, 4)), (16, 3001, (16, 8, 2)),
                           (16, 20000, (4, 4, 4)), (32, -1, (4, 4, 4))):
        say(f"[runs] run table {prec} n={n} np={npart} tile={tile}")
        if npart < 0:
            # clumped: crowded tiles that go first in the order
            wl = inputs.clumped_box(n=n, npart=60000, nclumps=3, sigma=1.5, steps=0)
            npart = wl.items[0].particles.n
        else:
            wl = inputs.turbulent_box(n=n, npart=npart, steps=0)
        p = B.PL_F64 if prec == "f64" else B.PL_F32_OFFSET
        run = driver.Run(wl, prec=p, algo=B.PL_ALGO_RUNS, tile=tile)
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
        perm = oracle.stable_sort_perm(keys.astype(np.uint32))
        assert np.array_equal(raw["id"].astype(np.int64), perm)
        ntiles = (n // tile[0]) * (n // tile[1]) * (n // tile[2])
        per_tile = tile[0] * tile[1] * tile[2]
        exp, tstart = expected_runs(keys[perm], per_tile, ntiles)
        assert np.array_equal(raw["tile_start"][: ntiles + 1], tstart)
        got = raw["runs"][: npart + 2 * ntiles].astype(np.int64)
        for t in range(ntiles):
            beg = tstart[t]
            nr = exp[npart + t]
            assert got[npart + t] == nr, (t, got[npart + t], nr)
            assert np.array_equal(got[beg:beg + nr], exp[beg:beg + nr]), t
        assert np.array_equal(got[npart + ntiles:], expected_order(exp[npart:npart + ntiles]))
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
    for a in range(3):
        assert table[f"x{a}"][0] <= 2e-5 and table[f"x{a}"][1] <= 2e-6
        assert table[f"u{a}"][0] <= 2e-5 and table[f"u{a}"][1] <= 2e-6
    for k, (mx, rms, rel) in merr.items():
        assert mx <= 2e-5 and rms <= 2e-6, k
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
@pytest.mark.parametrize("tile", [(4, 4, 4), (8, 8, 4)])
def test_runs_states_match_tiled_under_drift(mods, prec, tile):
    """No re-sort for 10 fast steps: queues fill and overflow on the 4^3
    tiles.  Per-id states bit-identical to the tiled kernel; deposits within
    the precision's tolerance of it."""
    oracle, driver, inputs, B = mods
    say(f"[runs] drift {prec} tile {tile}: runs vs tiled, 10 steps without re-sort")
    wl = _hot_box(inputs)
    p = B.PL_F64 if prec == "f64" else B.PL_F32_OFFSET
    res = {}
    for algo in (B.PL_ALGO_TILED, B.PL_ALGO_RUNS):
        run, st = _run_gpu(driver, wl, wl.steps, True, prec=p, algo=algo, tile=tile, key_mode=1)
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
    _check_item(run, 0, ores[0], wl, X_TOL, 1e-11, M_TOL)
    run.close()


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
    oracle, driver, inputs, B = mods
    say(f"[runs] batched species {prec} (tracers take the tiled kernel)")
    wl = _small_batch(inputs)
    ores = oracle.run_workload(wl)
    p = B.PL_F64 if prec == "f64" else B.PL_F32_OFFSET
    run, st = _run_gpu(driver, wl, wl.steps, True, prec=p, algo=B.PL_ALGO_RUNS)
    assert st == B.PL_OK
    _assert_runs_kernel(run, B)
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
