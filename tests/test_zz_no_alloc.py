"""pl_sort_noalloc (the sort for callers that cannot allocate) against
pl_part_sort: bit-identical permutation, particle arrays, tile offsets and run
table, on two calls in a row through the C ABI, the second with fewer
particles (the fixed scratch keeps the first call's contents)."""

import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mods():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_23434_amd import binding, driver, inputs
    binding.lib()
    return driver, inputs, binding


def _arrays(run, n, ntiles, B):
    raw = run.raw(0)
    out = {}
    for k in ("cell", "x", "u", "w", "id"):
        if k in raw:
            v = raw[k]
            out[k] = (np.stack(v) if isinstance(v, list) else v)[..., :n].copy()
    out["tile_start"] = raw["tile_start"][: ntiles + 1].copy()
    if "runs" in raw:
        out["runs"] = raw["runs"][: B.runs_len(n, ntiles)].copy()
    return out


@pytest.mark.parametrize("prec,algo,key", [("f32", "runs", "run"), ("f64", "tiled", "cell"),
                                           ("f32", "tiled", "tile")])
def test_sort_noalloc_matches_sort(mods, prec, algo, key):
    driver, inputs, B = mods
    p = B.PL_F64 if prec == "f64" else B.PL_F32_OFFSET
    a = B.PL_ALGO_RUNS if algo == "runs" else B.PL_ALGO_TILED
    km = {"run": B.PL_KEY_TILE_RUN, "cell": B.PL_KEY_TILE_CELL, "tile": B.PL_KEY_TILE}[key]
    n_box = 32
    tile = (8, 8, 8) if prec == "f32" else (8, 8, 4)
    ntiles = (n_box // tile[0]) * (n_box // tile[1]) * (n_box // tile[2])
    wl = inputs.turbulent_box(n=n_box, npart=8 * n_box ** 3 - 37, steps=0)
    ref = driver.Run(wl, prec=p, algo=a, key_mode=km, tile=tile)
    new = driver.Run(wl, prec=p, algo=a, key_mode=km, tile=tile)
    n_full = wl.items[0].particles.n
    for call, n in enumerate((n_full, 100003)):
        say(f"[noalloc] {prec} {algo} key {key}: call {call + 1}, {n} particles")
        ref.items[0].p.n = n
        new.items[0].p.n = n
        B.pl_part_sort(ref.ctx, ref.items)
        B.pl_sort_noalloc(new.desc, new.items)
        assert ref.sync() == B.PL_OK
        new.stream.synchronize()
        assert new.items[0].p.cur == ref.items[0].p.cur == (call + 1) % 2
        ga, gb = _arrays(ref, n, ntiles, B), _arrays(new, n, ntiles, B)
        assert set(ga) == set(gb)
        for k in ga:
            assert np.array_equal(ga[k], gb[k]), (call, k)
        # the sort really reordered: ids are a permutation, not the identity
        assert not np.array_equal(ga["id"], np.sort(ga["id"]))
    ref.close()
    new.close()


def test_sort_noalloc_limits(mods):
    driver, inputs, B = mods
    say("[noalloc] limits: size, rank key")
    wl = inputs.turbulent_box(n=16, npart=1000, steps=0)
    run = driver.Run(wl, prec=B.PL_F32_OFFSET, algo=B.PL_ALGO_TILED, key_mode=B.PL_KEY_TILE_CELL, tile=(4, 4, 4))
    n = run.items[0].p.n
    run.items[0].p.n = B.PL_NOALLOC_MAX_NP + 1
    assert B.pl_sort_noalloc(run.desc, run.items, check=False) == B.PL_ENOSPACE
    run.items[0].p.n = n
    run.desc.key_mode = B.PL_KEY_TILE_RANK
    assert B.pl_sort_noalloc(run.desc, run.items, check=False) == B.PL_EUNSUPPORTED
    run.desc.key_mode = B.PL_KEY_TILE_CELL
    assert run.items[0].p.cur == 0
    assert B.pl_sort_noalloc(run.desc, run.items, check=False) == B.PL_OK
    assert run.items[0].p.cur == 1
    run.stream.synchronize()
    run.close()
