"""The C-ABI library loads, exports every symbol include/pl.h declares, and its
ctypes structures match the C layout.  Host-side argument validation is
exercised on paths that return before any HIP call (no GPU needed)."""

import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

from paper_2602_23434_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pl.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pl_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        from paper_2602_23434_amd import build
        build.build()
    return B.lib()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert "pl_part_init" in names and "pl_part_sort" in names
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(B.EXPORTS) == names


def test_status_strings(lib):
    for s in range(9):
        assert B.pl_status_string(s) not in ("", "unknown status")
    assert "sort" in B.pl_status_string(B.PL_ENOTSORTED)
    assert B.pl_status_string(99) == "unknown status"


_PROBE = r"""
#include <stdio.h>
#include <stddef.h>
#include "pl.h"
#define S(t) printf(#t " %zu\n", sizeof(t));
#define O(t, f) printf(#t "." #f " %zu\n", offsetof(t, f));
int main(void) {
  S(pl_box_desc) O(pl_box_desc, dx) O(pl_box_desc, tile)
  S(pl_species_desc) O(pl_species_desc, q) O(pl_species_desc, t_stop)
  S(pl_init_desc) O(pl_init_desc, c) O(pl_init_desc, boxes) O(pl_init_desc, species) O(pl_init_desc, max_np)
  O(pl_init_desc, block) O(pl_init_desc, stream) O(pl_init_desc, tune_cache)
  S(pl_particles) O(pl_particles, cur) O(pl_particles, cell) O(pl_particles, x) O(pl_particles, u)
  O(pl_particles, w) O(pl_particles, id) O(pl_particles, fp) O(pl_particles, tile_start)
  O(pl_particles, runs) O(pl_particles, nbins) O(pl_particles, eng) O(pl_particles, chi)
  S(pl_fields) O(pl_fields, B) O(pl_fields, vg) O(pl_fields, divu)
  S(pl_spectra_desc) O(pl_spectra_desc, u_rad) O(pl_spectra_desc, ub)
  S(pl_boundary_desc) O(pl_boundary_desc, ghost)
  S(pl_moments) O(pl_moments, J) O(pl_moments, F) O(pl_moments, eng)
  S(pl_item) O(pl_item, p) O(pl_item, f) O(pl_item, m)
  printf("runs_len %lld\n", (long long)PL_RUNS_LEN(1000, 64));
  return 0;
}
"""


def test_struct_layout_matches_c():
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "probe.c")
        exe = os.path.join(d, "probe")
        open(src, "w").write(_PROBE)
        subprocess.run(["gcc", "-I" + os.path.join(ROOT, "include"), src, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    for line in out.strip().splitlines():
        name, val = line.split()
        val = int(val)
        if name == "runs_len":
            assert B.runs_len(1000, 64) == val
        elif "." in name:
            t, f = name.split(".")
            assert getattr(getattr(B, t), f).offset == val, name
        else:
            assert C.sizeof(getattr(B, name)) == val, name


def _desc(**kw):
    boxes = (B.pl_box_desc * 1)()
    for a in range(3):
        boxes[0].n[a] = 8
        boxes[0].dx[a] = 1.0
        boxes[0].tile[a] = 4
    sp = (B.pl_species_desc * 1)()
    sp[0].kind = B.PL_LORENTZ
    sp[0].q = sp[0].m = sp[0].weight = 1.0
    d = B.pl_init_desc()
    d.ndim, d.prec, d.shape, d.algo, d.key_mode = 3, B.PL_F64, B.PL_TSC, B.PL_ALGO_PLAIN, B.PL_KEY_TILE
    d.c = 1.0
    d.nboxes, d.boxes, d.nspecies, d.species = 1, boxes, 1, sp
    d.max_items, d.max_np, d.block = 1, 100, 0
    d._keep = (boxes, sp)
    for k, v in kw.items():
        if k in ("n", "tile", "dx"):
            for a in range(3):
                getattr(boxes[0], k)[a] = v[a]
        elif k in ("kind", "m", "t_stop", "q", "rk_stages"):
            setattr(sp[0], k, v)
        else:
            setattr(d, k, v)
    return d


@pytest.mark.parametrize("bad", [
    dict(ndim=4), dict(prec=7), dict(shape=0), dict(algo=5), dict(key_mode=5), dict(c=0.0),
    dict(c=float("inf")), dict(max_items=0), dict(max_np=-1), dict(max_np=1 << 31), dict(block=100),
    dict(block=1024), dict(n=(8, 8, 2000)), dict(n=(0, 8, 8)), dict(tile=(3, 4, 4)), dict(tile=(0, 4, 4)),
    dict(dx=(1.0, -1.0, 1.0)), dict(kind=9), dict(m=0.0), dict(kind=B.PL_DUST, t_stop=0.0),
    dict(ndim=2),          # 2D with n[2] = 8
    dict(nboxes=0),
    dict(algo=2),                                   # run-based kernel needs the tile+cell key
    dict(algo=2, key_mode=1, block=256),            # run-based block is 512
    dict(algo=2, key_mode=1, block=1024),
    dict(algo=2, key_mode=1, max_np=1 << 29),       # run entries hold the first index in 30 bits
    dict(kind=B.PL_TRACER, rk_stages=4),            # tracers take 2 or 3 Runge-Kutta stages
    dict(key_mode=3),                               # run order only with the run-based kernel
    dict(algo=1, key_mode=3),
])
def test_init_rejects_bad_descriptions(lib, bad):
    d = _desc(**bad)
    ctx = C.c_void_p()
    st = lib.pl_part_init(C.byref(ctx), C.byref(d))
    assert st == B.PL_EINVAL
    assert not ctx.value


def test_runs_tile_limit(lib):
    """The run table build keeps per-cell counts of one tile in LDS: at most
    1024 cells per tile."""
    d = _desc(algo=2, key_mode=1, n=(64, 64, 64), tile=(16, 16, 8))
    ctx = C.c_void_p()
    assert lib.pl_part_init(C.byref(ctx), C.byref(d)) == B.PL_EUNSUPPORTED
    assert not ctx.value


def test_null_context_calls_are_rejected(lib):
    item = B.pl_item()
    assert lib.pl_part_gather_push(None, C.byref(item), 1, 0.05, 0) == B.PL_EINVAL
    assert lib.pl_part_deposit(None, C.byref(item), 1, 0) == B.PL_EINVAL
    assert lib.pl_part_sort(None, C.byref(item), 1) == B.PL_EINVAL
    assert lib.pl_part_sync(None) == B.PL_EINVAL
    sd = B.pl_spectra_desc(1.0, 0.0, 0.5)
    assert lib.pl_part_spectra(None, C.byref(item), 1, 0.05, C.byref(sd)) == B.PL_EINVAL
    bc = B.pl_boundary_desc((C.c_int * 3)(1, 0, 0), 2)
    assert lib.pl_part_boundary(None, C.byref(item), 1, C.byref(bc), None) == B.PL_EINVAL
    x3 = (C.c_void_p * 3)()
    assert lib.pl_part_inject(None, C.byref(item), 1, x3, x3, None, None, None, None, 1) == B.PL_EINVAL
    assert lib.pl_sort_noalloc(None, C.byref(item), 1) == B.PL_EINVAL
    out = (C.c_int64 * B.PL_NSTATS)()
    assert lib.pl_part_stats(None, out, B.PL_NSTATS) == B.PL_EINVAL
    assert lib.pl_part_init(None, None) == B.PL_EINVAL
    lib.pl_part_finalize(None)
