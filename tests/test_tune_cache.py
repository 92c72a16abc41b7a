"""The autotuner's cache file on the CPU: what write_cache stores,
read_cache returns, and the benchmark's configurations take from the files
shipped beside the package."""

from paper_2602_23434_amd import benchcfg, tune
from paper_2602_23434_amd import binding as B


def test_write_read_roundtrip(tmp_path):
    path = tmp_path / "t.txt"
    best = {"algo": B.PL_ALGO_RUNS, "key": B.PL_KEY_TILE_RUN, "block": 512, "tile": (8, 8, 4), "sort_every": 16,
            "one_launch": 0, "ms": 1.23456}
    tune.write_cache(str(path), best, "a test workload")
    text = path.read_text()
    assert text.startswith("# autotuned on MI355X: a test workload\n")
    got = tune.read_cache(str(path))
    assert got == {"algo": 2, "key": 3, "runs_block": 512, "tile": (8, 8, 4), "sort_every": 16, "one_launch": 0,
                   "ms_per_step": 1.2346}
    # the tiled kernel's block goes under its own key
    best2 = dict(best, algo=B.PL_ALGO_TILED, key=B.PL_KEY_TILE_RANK, block=256)
    best2.pop("one_launch")
    tune.write_cache(str(path), best2, "x")
    got = tune.read_cache(str(path))
    assert got["block"] == 256 and "runs_block" not in got and "one_launch" not in got


def test_shipped_caches_drive_the_benchmark():
    """The shipped caches name the run-based kernel in run order; the
    benchmark's headline and batched configurations take tile, key, block
    and cadence from them."""
    for batched in (False, True):
        t = tune.read_cache(tune.tune_file(B.PL_F32_OFFSET, batched=batched))
        cfg = benchcfg.batched_cfg() if batched else benchcfg.headline()
        assert t["algo"] == B.PL_ALGO_RUNS and cfg["algo"] == B.PL_ALGO_RUNS
        assert cfg["key_mode"] == t["key"] == B.PL_KEY_TILE_RUN
        assert tuple(cfg["tile"]) == tuple(t["tile"])
        assert cfg["block"] == t["runs_block"] == 512
        assert cfg["sort_every"] == t["sort_every"]
    assert benchcfg.batched_cfg()["tune_cache"] == tune.tune_file(B.PL_F32_OFFSET, batched=True)
    assert benchcfg.batched_cfg()["channels"] is None


def test_candidates_divide_the_box():
    for n in (128, 96, 24, 20):
        for algo, tile, block, key, every in tune.candidates(n, B.PL_F32_OFFSET):
            assert all(n % t == 0 for t in tile)
            assert every in tune.CADENCES


def test_no_candidate_is_an_error():
    import pytest
    assert list(tune.candidates(20, B.PL_F32_OFFSET)) == []
    with pytest.raises(ValueError):
        tune.tune(n=20, steps=1)
