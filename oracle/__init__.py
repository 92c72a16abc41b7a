"""Reference CPU implementation ("oracle") of the per-step particle update.

TEST INFRASTRUCTURE ONLY.  It is imported by ``tests/``, by the smoke check
and by the benchmark's CPU-baseline leg, never by the GPU library.  The
arithmetic lives in ``orc.c`` (plain C, float64, built with
``-ffp-contract=off``); this module only marshals numpy arrays through ctypes.

Grid coordinates are in cell units (cell i spans [i, i+1)), grid arrays are
float64 (nz, ny, nx) in C order, particles are structure-of-arrays float64.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# ORC_LIB names another build of orc.c to load instead (the mutation tests
# load copies with a planted mistake this way)
LIB_PATH = os.environ.get("ORC_LIB") or os.path.join(HERE, "liborc.so")

CIC, TSC = 1, 2
LORENTZ, DUST, TRACER = 0, 1, 2
KEY_TILE, KEY_TILE_CELL, KEY_TILE_RANK = 0, 1, 2
KINDS = {"lorentz": LORENTZ, "dust": DUST, "tracer": TRACER}
SHAPES = {"cic": CIC, "tsc": TSC}


def build(verbose=False):
    """Compile liborc.so from orc.c (gcc, OpenMP, no fused multiply-add)."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c99",
           "-Wall", "-Wextra", "-o", LIB_PATH + ".tmp", os.path.join(HERE, "orc.c"), "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    global _LIB
    _LIB = None


class _Box(C.Structure):
    _fields_ = [("ndim", C.c_int), ("n", C.c_int * 3), ("dx", C.c_double * 3)]


class _Species(C.Structure):
    _fields_ = [("kind", C.c_int), ("q", C.c_double), ("m", C.c_double), ("t_stop", C.c_double),
                ("rk", C.c_int)]


_P = C.POINTER(C.c_double)


class _Fields(C.Structure):
    _fields_ = [("E", _P * 3), ("B", _P * 3), ("vg", _P * 3)]


class _Moments(C.Structure):
    _fields_ = [("rho", _P), ("J", _P * 3), ("F", _P * 3), ("eng", _P)]


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        L.orc_weights_1d.restype = C.c_int
        L.orc_weights_1d.argtypes = [C.c_int, C.c_double, C.POINTER(C.c_long), _P]
        L.orc_gather.restype = C.c_double
        L.orc_gather.argtypes = [C.POINTER(_Box), C.c_int, _P, _P]
        L.orc_deposit_one.restype = None
        L.orc_deposit_one.argtypes = [C.POINTER(_Box), C.c_int, _P, _P, C.c_double]
        L.orc_step.restype = C.c_long
        L.orc_step.argtypes = [C.POINTER(_Box), C.c_int, C.c_double, C.POINTER(_Species), C.c_long,
                               _P * 3, _P * 3, _P, C.c_double, C.POINTER(_Fields), C.c_double,
                               C.POINTER(_Moments), C.POINTER(_Moments), C.c_void_p]
        L.orc_tile_key.restype = C.c_uint32
        L.orc_tile_key.argtypes = [C.POINTER(_Box), C.c_int * 3, C.c_int, C.c_long, C.c_long, C.c_long]
        L.orc_split_position.restype = None
        L.orc_split_position.argtypes = [C.POINTER(_Box), _P, C.POINTER(C.c_long), C.POINTER(C.c_float)]
        L.orc_rank_keys.restype = C.c_int
        L.orc_rank_keys.argtypes = [C.POINTER(_Box), C.c_int * 3, C.c_long, C.POINTER(C.c_long),
                                    C.POINTER(C.c_long), C.POINTER(C.c_long), C.POINTER(C.c_uint32)]
        L.orc_num_threads.restype = C.c_int
        L.orc_num_threads.argtypes = []
        L.orc_set_threads.restype = None
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_stable_sort_perm.restype = None
        L.orc_stable_sort_perm.argtypes = [C.c_long, C.POINTER(C.c_uint32), C.POINTER(C.c_long)]
        L.orc_spectra_step.restype = None
        L.orc_spectra_step.argtypes = [C.POINTER(_Box), C.c_int, C.c_double, C.c_long, _P * 3,
                                       C.POINTER(_Fields), _P, C.c_int, _P, _P, C.c_double,
                                       C.POINTER(_SpectraPar)]
        L.orc_outside.restype = C.c_int
        L.orc_outside.argtypes = [C.POINTER(_Box), C.c_int * 3, C.c_int, _P]
        L.orc_compact.restype = C.c_long
        L.orc_compact.argtypes = [C.c_long, C.POINTER(C.c_ubyte), C.c_int, C.POINTER(C.c_void_p),
                                  C.POINTER(C.c_size_t), C.POINTER(C.c_long), C.POINTER(C.c_long),
                                  C.POINTER(C.c_long)]
        _LIB = L
    return _LIB


class _SpectraPar(C.Structure):
    _fields_ = [("cr", C.c_double), ("u_rad", C.c_double), ("ub", C.c_double)]


def _dp(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_P)


def _box(ndim, n, dx=(1.0, 1.0, 1.0)):
    b = _Box()
    b.ndim = ndim
    for d in range(3):
        b.n[d] = int(n[d])
        b.dx[d] = float(dx[d])
    return b


def weights_1d(shape, x):
    first = C.c_long()
    w = np.zeros(3)
    cnt = lib().orc_weights_1d(shape, float(x), C.byref(first), _dp(w))
    return first.value, w[:cnt].copy()


def gather(ndim, n, shape, f, x, dx=(1.0, 1.0, 1.0)):
    b = _box(ndim, n, dx)
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
    xx = np.zeros(3)
    xx[: len(x)] = x
    return lib().orc_gather(C.byref(b), shape, _dp(f), _dp(xx))


def deposit_one(ndim, n, shape, g, x, mu, dx=(1.0, 1.0, 1.0)):
    b = _box(ndim, n, dx)
    assert g.dtype == np.float64 and g.flags.c_contiguous
    xx = np.zeros(3)
    xx[: len(x)] = x
    lib().orc_deposit_one(C.byref(b), shape, _dp(g), _dp(xx), float(mu))


def new_moments(n, kind):
    """Zeroed moment grids for one item: the channels its species deposits."""
    nx, ny, nz = n
    z = lambda: np.zeros((nz, ny, nx))
    if kind == LORENTZ:
        return {"rho": z(), "J": [z(), z(), z()], "F": [z(), z(), z()], "eng": z()}
    if kind == DUST:
        return {"rho": z(), "J": None, "F": [z(), z(), z()], "eng": None}
    return None


def _moments_struct(m):
    s = _Moments()
    if m is None:
        return None
    s.rho = _dp(m["rho"]) if m.get("rho") is not None else None
    for d in range(3):
        s.J[d] = _dp(m["J"][d]) if m.get("J") is not None else None
        s.F[d] = _dp(m["F"][d]) if m.get("F") is not None else None
    s.eng = _dp(m["eng"]) if m.get("eng") is not None else None
    return s


def step(ndim, n, shape, species, x, u, w, fields, dt, c=1.0, dx=(1.0, 1.0, 1.0),
         moments=None, abs_moments=None, fp=None, wdef=1.0):
    """Advance particle arrays x, u (3, np) float64 in place by one step.

    ``species`` is (kind, q, m, t_stop[, rk]) with rk the tracers' Runge-Kutta
    stages (2, the default, or 3).  ``fields`` maps "E","B","vg" to
    (3, nz, ny, nx) arrays (only what the kind needs).  ``moments`` and
    ``abs_moments`` are dicts from :func:`new_moments` (added to).  Returns the
    number of particles whose displacement reached one cell.
    """
    kind, q, m, t_stop = species[:4]
    rk = species[4] if len(species) > 4 else 2
    b = _box(ndim, n, dx)
    sp = _Species(kind, q, m, t_stop, rk)
    npart = x.shape[1]
    assert x.shape == (3, npart) and u.shape == (3, npart)
    xs = (_P * 3)(*[_dp(x[d]) for d in range(3)])
    us = (_P * 3)(*[_dp(u[d]) for d in range(3)])
    f = _Fields()
    keep = []
    for name in ("E", "B", "vg"):
        arr = fields.get(name) if fields else None
        for d in range(3):
            if arr is not None:
                a = np.ascontiguousarray(arr[d], dtype=np.float64)
                keep.append(a)
                getattr(f, name)[d] = _dp(a)
            else:
                getattr(f, name)[d] = None
    ms = _moments_struct(moments)
    am = _moments_struct(abs_moments)
    fpp = None
    if fp is not None:
        fpa = (_P * 3)(*[_dp(fp[d]) for d in range(3)])
        fpp = C.cast(fpa, C.c_void_p)
    wp = _dp(w) if w is not None else None
    return lib().orc_step(C.byref(b), shape, float(c), C.byref(sp), npart, xs, us, wp, float(wdef),
                          C.byref(f), float(dt), C.byref(ms) if ms is not None else None,
                          C.byref(am) if am is not None else None, fpp)


def tile_key(ndim, n, tile, key_mode, i, j, k):
    b = _box(ndim, n)
    t = (C.c_int * 3)(*tile)
    return lib().orc_tile_key(C.byref(b), t, key_mode, i, j, k)


def rank_keys(ndim, n, tile, cells):
    """Rank-interleaved sort keys from integer cells (3, np); returns (keys, rank_bits)."""
    b = _box(ndim, n)
    t = (C.c_int * 3)(*tile)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    npart = cells.shape[1]
    keys = np.zeros(npart, dtype=np.uint32)
    lp = C.POINTER(C.c_long)
    c = [np.ascontiguousarray(cells[d]) for d in range(3)]
    rb = lib().orc_rank_keys(C.byref(b), t, npart, c[0].ctypes.data_as(lp), c[1].ctypes.data_as(lp),
                             c[2].ctypes.data_as(lp), keys.ctypes.data_as(C.POINTER(C.c_uint32)))
    return keys, rb


def cells_of_positions(ndim, n, x):
    """Integer cells floor(x) of float64 grid positions (after the periodic wrap)."""
    cells = np.zeros((3, x.shape[1]), dtype=np.int64)
    for d in range(ndim):
        v = np.mod(x[d], n[d])
        v = np.where(v >= n[d], 0.0, v)
        cells[d] = np.floor(v).astype(np.int64)
    return cells


def split_positions(ndim, n, x):
    """Cell index (3, np) int64 and float32 offsets (3, np) for each particle."""
    b = _box(ndim, n)
    npart = x.shape[1]
    cells = np.zeros((3, npart), dtype=np.int64)
    offs = np.zeros((3, npart), dtype=np.float32)
    xx = np.zeros(3)
    cc = (C.c_long * 3)()
    oo = (C.c_float * 3)()
    L = lib()
    for p in range(npart):
        xx[:] = x[:, p]
        L.orc_split_position(C.byref(b), _dp(xx), cc, oo)
        cells[:, p] = cc[:]
        offs[:, p] = oo[:]
    return cells, offs


def num_threads():
    return lib().orc_num_threads()


def set_threads(n):
    lib().orc_set_threads(int(n))


def stable_sort_perm(keys):
    keys = np.ascontiguousarray(keys, dtype=np.uint32)
    perm = np.zeros(keys.shape[0], dtype=np.int64)
    lib().orc_stable_sort_perm(keys.shape[0], keys.ctypes.data_as(C.POINTER(C.c_uint32)),
                               perm.ctypes.data_as(C.POINTER(C.c_long)))
    return perm


def run_workload(wl, steps=None, c=1.0, abs_sums=True, fp=False):
    """Advance every item of a workload (see ``paper_2602_23434_amd.inputs``).

    Moments are zeroed at the start of every step and deposited at the new
    positions, so on return they hold the last step's deposit.  Returns a list
    of per-item dicts with the final x, u and moments (and |mu| W sums).
    """
    steps = wl.steps if steps is None else steps
    shape = SHAPES[wl.shape]
    out = []
    for it in wl.items:
        box = wl.boxes[it.box]
        sp = wl.species[it.species]
        kind = KINDS[sp.kind]
        x = it.particles.x.copy()
        u = it.particles.u.copy()
        w = it.particles.w.copy()
        mom = am = None
        fpa = np.zeros((3, x.shape[1])) if fp else None
        viol = 0
        for _ in range(steps):
            mom = new_moments(box.n, kind)
            am = new_moments(box.n, kind) if abs_sums else None
            viol += step(box.ndim, box.n, shape, (kind, sp.q, sp.m, sp.t_stop, sp.rk_stages), x, u, w, box.fields,
                         wl.dt, c=c, dx=box.dx, moments=mom, abs_moments=am, fp=fpa)
        out.append({"x": x, "u": u, "w": w, "moments": mom, "abs": am, "violations": viol, "fp": fpa})
    return out


def spectra_step(ndim, n, shape, x, fields, divu, eng, chi, dt, cr, u_rad=0.0, ub=0.5, c=1.0,
                 dx=(1.0, 1.0, 1.0)):
    """One step of the particles' energy distributions in place.

    ``x`` (3, np) grid positions; ``fields`` maps "B" and "vg" to
    (3, nz, ny, nx) arrays; ``divu`` (nz, ny, nx) the four-divergence of the
    fluid velocity; ``eng``, ``chi`` (np, nb) particle-major float64.
    Loss coefficient c_r = cr (ub |B|^2 + u_rad)."""
    b = _box(ndim, n, dx)
    npart = x.shape[1]
    assert eng.shape == chi.shape and eng.shape[0] == npart
    assert eng.flags.c_contiguous and chi.flags.c_contiguous
    xs = (_P * 3)(*[_dp(x[d]) for d in range(3)])
    f = _Fields()
    keep = []
    for name in ("B", "vg"):
        for d in range(3):
            a = np.ascontiguousarray(fields[name][d], dtype=np.float64)
            keep.append(a)
            getattr(f, name)[d] = _dp(a)
    dv = np.ascontiguousarray(divu, dtype=np.float64)
    par = _SpectraPar(float(cr), float(u_rad), float(ub))
    lib().orc_spectra_step(C.byref(b), shape, float(c), npart, xs, C.byref(f), _dp(dv), eng.shape[1],
                           _dp(eng), _dp(chi), float(dt), C.byref(par))


def outside(ndim, n, open_dims, ghost, x):
    """Per particle: 1 if grid position x[:, p] lies outside the active cells of
    an open dimension."""
    b = _box(ndim, n)
    od = (C.c_int * 3)(*[int(v) for v in open_dims])
    out = np.zeros(x.shape[1], dtype=np.uint8)
    xx = np.zeros(3)
    for p in range(x.shape[1]):
        xx[:] = x[:, p]
        out[p] = lib().orc_outside(C.byref(b), od, int(ghost), _dp(xx))
    return out


def compact(flag, arrays):
    """Holes-and-fillers compaction (in place) of the 1-D numpy arrays in
    ``arrays`` (the same length, any dtypes); returns (new count, holes,
    fillers) with the copied pairs in order."""
    flag = np.ascontiguousarray(flag, dtype=np.uint8)
    npart = flag.shape[0]
    for a in arrays:
        assert a.shape[0] == npart and a.flags.c_contiguous
    ptrs = (C.c_void_p * max(1, len(arrays)))(*[a.ctypes.data for a in arrays])
    esz = (C.c_size_t * max(1, len(arrays)))(*[a.itemsize * (a.size // max(npart, 1)) for a in arrays])
    holes = np.zeros(max(npart, 1), dtype=np.int64)
    fills = np.zeros(max(npart, 1), dtype=np.int64)
    nc = C.c_long()
    keep = lib().orc_compact(npart, flag.ctypes.data_as(C.POINTER(C.c_ubyte)), len(arrays), ptrs, esz,
                             holes.ctypes.data_as(C.POINTER(C.c_long)), fills.ctypes.data_as(C.POINTER(C.c_long)),
                             C.byref(nc))
    return int(keep), holes[: nc.value].copy(), fills[: nc.value].copy()

