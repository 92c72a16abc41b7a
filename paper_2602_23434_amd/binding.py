"""ctypes binding of libpl.so: the C ABI of include/pl.h under the same names.

Argument marshalling only; every step of the particle update runs in the HIP
kernels of libpl.so.  Loading fails loudly when the library has not been
built (``python -m paper_2602_23434_amd.build``): there is no fallback.
"""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpl.so")

PL_OK, PL_EINVAL, PL_ENOMEM, PL_EHIP, PL_EUNSUPPORTED, PL_ECFL, PL_ENONFINITE, PL_ENOTSORTED, PL_ENOSPACE = range(9)
PL_NOALLOC_MAX_NP = 1 << 20
PL_NSTATS = 8
PL_F64, PL_F32_OFFSET = 0, 1
PL_CIC, PL_TSC = 1, 2
PL_LORENTZ, PL_DUST, PL_TRACER = 0, 1, 2
PL_ALGO_PLAIN, PL_ALGO_TILED, PL_ALGO_RUNS = 0, 1, 2
PL_KEY_TILE, PL_KEY_TILE_CELL, PL_KEY_TILE_RANK, PL_KEY_TILE_RUN = 0, 1, 2, 3
PL_RUNS_SPLIT_UNITS = 1024


def runs_len(n, ntiles):
    """PL_RUNS_LEN: entries of the run table of n particles over ntiles tiles."""
    return n + 3 * ntiles + 2 * PL_RUNS_SPLIT_UNITS + 1
PL_FUSE_DEPOSIT, PL_ZERO_FIRST, PL_GRAPH, PL_SUMS, PL_SORT_FIRST = 1, 2, 4, 8, 16

EXPORTS = ["pl_part_init", "pl_part_gather_push", "pl_part_deposit", "pl_part_sort", "pl_part_pack",
           "pl_part_unpack", "pl_part_sums", "pl_part_sync", "pl_part_set_stream", "pl_part_stats",
           "pl_part_finalize", "pl_status_string", "pl_sort_noalloc", "pl_part_spectra", "pl_part_boundary",
           "pl_part_inject"]

_vp = C.c_void_p


class pl_box_desc(C.Structure):
    _fields_ = [("n", C.c_int * 3), ("dx", C.c_double * 3), ("tile", C.c_int * 3)]


class pl_species_desc(C.Structure):
    _fields_ = [("kind", C.c_int), ("q", C.c_double), ("m", C.c_double), ("weight", C.c_double),
                ("t_stop", C.c_double), ("rk_stages", C.c_int)]


class pl_init_desc(C.Structure):
    _fields_ = [("ndim", C.c_int), ("prec", C.c_int), ("shape", C.c_int), ("algo", C.c_int),
                ("key_mode", C.c_int), ("c", C.c_double), ("nboxes", C.c_int),
                ("boxes", C.POINTER(pl_box_desc)), ("nspecies", C.c_int),
                ("species", C.POINTER(pl_species_desc)), ("max_items", C.c_int), ("max_np", C.c_int64),
                ("block", C.c_int), ("stream", _vp), ("tune_cache", C.c_char_p)]


class pl_particles(C.Structure):
    _fields_ = [("n", C.c_int64), ("cur", C.c_int), ("cell", _vp * 2), ("x", (_vp * 3) * 2),
                ("u", (_vp * 3) * 2), ("w", _vp * 2), ("id", _vp * 2), ("fp", _vp * 3), ("tile_start", _vp),
                ("runs", _vp), ("nbins", C.c_int), ("eng", _vp * 2), ("chi", _vp * 2)]


class pl_fields(C.Structure):
    _fields_ = [("E", _vp * 3), ("B", _vp * 3), ("vg", _vp * 3), ("divu", _vp)]


class pl_moments(C.Structure):
    _fields_ = [("rho", _vp), ("J", _vp * 3), ("F", _vp * 3), ("eng", _vp)]


class pl_item(C.Structure):
    _fields_ = [("box", C.c_int), ("species", C.c_int), ("p", pl_particles), ("f", pl_fields),
                ("m", pl_moments)]


class pl_spectra_desc(C.Structure):
    _fields_ = [("cr", C.c_double), ("u_rad", C.c_double), ("ub", C.c_double)]


class pl_boundary_desc(C.Structure):
    _fields_ = [("open", C.c_int * 3), ("ghost", C.c_int)]


class PLError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: {pl_status_string(status)} (status {status})")


_LIB = None


def lib():
    """Load libpl.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2602_23434_amd.build`")
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        L.pl_part_init.argtypes = [P(_vp), P(pl_init_desc)]
        L.pl_part_gather_push.argtypes = [_vp, P(pl_item), C.c_int, C.c_double, C.c_uint32]
        L.pl_part_deposit.argtypes = [_vp, P(pl_item), C.c_int, C.c_uint32]
        L.pl_part_sort.argtypes = [_vp, P(pl_item), C.c_int]
        L.pl_sort_noalloc.argtypes = [P(pl_init_desc), P(pl_item), C.c_int]
        L.pl_part_spectra.argtypes = [_vp, P(pl_item), C.c_int, C.c_double, P(pl_spectra_desc)]
        L.pl_part_boundary.argtypes = [_vp, P(pl_item), C.c_int, P(pl_boundary_desc), P(C.c_int64)]
        L.pl_part_inject.argtypes = [_vp, P(pl_item), C.c_int64, P(_vp), P(_vp), _vp, _vp, _vp, _vp, C.c_int64]
        L.pl_part_pack.argtypes = [_vp, P(pl_item), P(_vp), P(_vp)]
        L.pl_part_unpack.argtypes = [_vp, P(pl_item), P(_vp), P(_vp)]
        L.pl_part_sums.argtypes = [_vp, P(pl_item), C.c_int, P(C.c_double)]
        L.pl_part_sync.argtypes = [_vp]
        L.pl_part_set_stream.argtypes = [_vp, _vp]
        L.pl_part_stats.argtypes = [_vp, P(C.c_int64), C.c_int]
        L.pl_part_finalize.argtypes = [_vp]
        L.pl_part_finalize.restype = None
        L.pl_status_string.argtypes = [C.c_int]
        L.pl_status_string.restype = C.c_char_p
        for name in EXPORTS:
            if name not in ("pl_part_finalize", "pl_status_string"):
                getattr(L, name).restype = C.c_int
        _LIB = L
    return _LIB


def _check(status, where):
    if status != PL_OK:
        raise PLError(status, where)
    return status


def pl_status_string(status):
    return lib().pl_status_string(int(status)).decode()


def pl_part_init(desc):
    ctx = _vp()
    _check(lib().pl_part_init(C.byref(ctx), C.byref(desc)), "pl_part_init")
    return ctx


def _items_arg(items):
    if isinstance(items, pl_item):
        return C.pointer(items), 1
    return items, len(items)


def pl_part_gather_push(ctx, items, dt, flags=0, check=True):
    arr, n = _items_arg(items)
    st = lib().pl_part_gather_push(ctx, arr, n, float(dt), int(flags))
    return _check(st, "pl_part_gather_push") if check else st


def pl_part_deposit(ctx, items, flags=0, check=True):
    arr, n = _items_arg(items)
    st = lib().pl_part_deposit(ctx, arr, n, int(flags))
    return _check(st, "pl_part_deposit") if check else st


def pl_part_sort(ctx, items, check=True):
    arr, n = _items_arg(items)
    st = lib().pl_part_sort(ctx, arr, n)
    return _check(st, "pl_part_sort") if check else st


def pl_part_spectra(ctx, items, dt, cr, u_rad=0.0, ub=0.5, check=True):
    arr, n = _items_arg(items)
    sd = pl_spectra_desc(float(cr), float(u_rad), float(ub))
    st = lib().pl_part_spectra(ctx, arr, n, float(dt), C.byref(sd))
    return _check(st, "pl_part_spectra") if check else st


def pl_part_boundary(ctx, items, open_dims, ghost, check=True):
    """Returns (status, removed per item); items' p.n are updated in place."""
    arr, n = _items_arg(items)
    bc = pl_boundary_desc((C.c_int * 3)(*[int(v) for v in open_dims]), int(ghost))
    removed = (C.c_int64 * n)()
    st = lib().pl_part_boundary(ctx, arr, n, C.byref(bc), removed)
    if check:
        _check(st, "pl_part_boundary")
    return st, list(removed)


def pl_part_inject(ctx, item, k, x, u, w=None, id=None, eng=None, chi=None, cap=None, check=True):
    """x, u: three device pointers each (x[2] may be None in 2D)."""
    st = lib().pl_part_inject(ctx, C.byref(item), int(k), _ptr3(x), _ptr3(u), w, id, eng, chi,
                              int(cap if cap is not None else item.p.n + k))
    return _check(st, "pl_part_inject") if check else st


def pl_sort_noalloc(desc, items, check=True):
    """pl_part_sort without a context, its scratch in the library's fixed array."""
    arr, n = _items_arg(items)
    st = lib().pl_sort_noalloc(C.byref(desc), arr, n)
    return _check(st, "pl_sort_noalloc") if check else st


def _ptr3(ptrs):
    a = (_vp * 3)()
    for k in range(3):
        a[k] = ptrs[k] if k < len(ptrs) and ptrs[k] else None
    return a


def pl_part_pack(ctx, item, x, u, check=True):
    st = lib().pl_part_pack(ctx, C.byref(item), _ptr3(x), _ptr3(u))
    return _check(st, "pl_part_pack") if check else st


def pl_part_unpack(ctx, item, x, u, check=True):
    st = lib().pl_part_unpack(ctx, C.byref(item), _ptr3(x), _ptr3(u))
    return _check(st, "pl_part_unpack") if check else st


def pl_part_sums(ctx, items):
    arr, n = _items_arg(items)
    out = (C.c_double * (16 * n))()
    _check(lib().pl_part_sums(ctx, arr, n, out), "pl_part_sums")
    return [list(out[16 * i:16 * i + 16]) for i in range(n)]


def pl_part_sync(ctx):
    """Returns the status (PL_OK, PL_ECFL, PL_ENONFINITE, ...) without raising."""
    return lib().pl_part_sync(ctx)


def pl_part_set_stream(ctx, stream):
    _check(lib().pl_part_set_stream(ctx, stream), "pl_part_set_stream")


def pl_part_stats(ctx):
    """The PL_NSTATS counters of pl_part_stats (see pl.h)."""
    out = (C.c_int64 * PL_NSTATS)()
    _check(lib().pl_part_stats(ctx, out, PL_NSTATS), "pl_part_stats")
    return list(out)


def runs_variant(stats):
    """(ts, chs, hf) of the last run-based launch from pl_part_stats' out[7]
    (bit 12, a launch over several species kinds, is not part of it)."""
    v = int(stats[7])
    return v & 15, (v >> 4) & 15, (v >> 8) & 15


def pl_part_finalize(ctx):
    lib().pl_part_finalize(ctx)
