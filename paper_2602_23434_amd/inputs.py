"""Seeded synthetic inputs for the particle update.

This module is shared by the CPU oracle's tests, the GPU parity tests and the
benchmark.  It draws random numbers and assembles the workloads' inputs
(grids, fields, particle positions and velocities); it computes no step of
the particle update itself (no weights, gather, push, deposit or sort).

Layout conventions (the same everywhere in this repository):

* Grid coordinates are in cell units: cell ``i`` spans ``[i, i+1)`` and its
  centre is at ``i + 1/2``; the domain is ``[0, N)`` per dimension, periodic.
* Grid arrays are float64 of shape ``(nz, ny, nx)`` in C order, so the flat
  index of cell ``(i, j, k)`` is ``i + nx*(j + ny*k)`` (x fastest).  A 2D box
  has ``nz == 1``.
* Particle arrays are structure-of-arrays: ``x`` and ``u`` of shape ``(3, np)``
  float64 (``u`` is the spatial part of the four-velocity, ``gamma*v``, in
  units of c = 1), weights ``w`` of shape ``(np,)`` and ids ``(np,)`` uint64
  equal to the initial index.

The turbulent-field recipe follows the standard Fourier synthesis of a
Kolmogorov spectrum: integer wave vectors ``m`` with ``1 <= |m| <= N/4``,
per-mode amplitude ``|m|**(-11/6)`` (shell spectrum ``E(k) ~ k**(-5/3)``),
complex Gaussian coefficients (uniform random phases), projection onto the
divergence-free subspace, and an RMS rescaling.  The electric field is the
ideal-MHD field ``E = -v x B`` of a velocity field drawn with the same recipe.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Seeds per workload k: fields B 1000+k, velocity 2000+k, particles 3000+k;
# small box b of the batched workload: 10000 + 100*b (+0 B, +1 v, +2 particles).
SEED_B, SEED_V, SEED_P = 1000, 2000, 3000


def _solenoidal_modes(n, seed, kmax_frac=0.25, slope=-11.0 / 6.0):
    """Random divergence-free vector field on an nx x ny x nz periodic grid (rms not set)."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = n
    kx = np.fft.rfftfreq(nx, 1.0 / nx)
    ky = np.fft.fftfreq(ny, 1.0 / ny)
    kz = np.fft.fftfreq(nz, 1.0 / nz)
    KZ, KY, KX = np.meshgrid(kz, ky, kx, indexing="ij")
    k2 = KX * KX + KY * KY + KZ * KZ
    kmag = np.sqrt(k2)
    kmax = kmax_frac * min(v for v in n if v > 1)     # a 2D grid (nz = 1) keeps its in-plane modes
    live = (kmag >= 1.0) & (kmag <= kmax)
    amp = np.zeros_like(kmag)
    amp[live] = kmag[live] ** slope
    shape = (3,) + kmag.shape
    coef = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * (amp / math.sqrt(2.0))
    # divergence-free projection  a <- a - m (m.a)/|m|^2
    kvec = np.stack([KX, KY, KZ])
    safe = np.where(k2 > 0, k2, 1.0)
    kdota = (kvec * coef).sum(axis=0)
    coef = coef - kvec * (kdota / safe)
    coef[:, ~live] = 0.0
    out = np.empty((3, nz, ny, nx))
    for c in range(3):
        out[c] = np.fft.irfftn(coef[c], s=(nz, ny, nx), axes=(0, 1, 2))
    return out


def _rescale_rms(f, rms):
    cur = math.sqrt(float(np.mean((f * f).sum(axis=0))))
    return f * (rms / cur)


def turbulent_fields(n, seed_b, seed_v, b0=(0.0, 0.0, 1.0), db_rms=0.5, v_rms=0.1):
    """E, B and gas velocity on an n^3 grid.

    ``B = B0 + dB`` with ``rms(|dB|) = db_rms``; ``v`` with ``rms(|v|) = v_rms``
    (same spectrum, its own seed); ``E = -v x B`` cell by cell.
    Returns a dict of float64 arrays of shape ``(3, nz, ny, nx)``.
    """
    n = tuple(int(a) for a in n)
    db = _rescale_rms(_solenoidal_modes(n, seed_b), db_rms)
    vg = _rescale_rms(_solenoidal_modes(n, seed_v), v_rms)
    B = db
    for c in range(3):
        B[c] += b0[c]
    E = -np.cross(vg, B, axis=0)
    return {"E": np.ascontiguousarray(E), "B": np.ascontiguousarray(B), "vg": np.ascontiguousarray(vg)}


def uniform_fields(n, E=(0.0, 0.0, 0.0), B=(0.0, 0.0, 1.0), vg=(0.0, 0.0, 0.0)):
    """Spatially uniform fields on a grid of shape n = (nx, ny, nz)."""
    nx, ny, nz = n
    out = {}
    for name, val in (("E", E), ("B", B), ("vg", vg)):
        a = np.empty((3, nz, ny, nx))
        for c in range(3):
            a[c] = val[c]
        out[name] = a
    return out


def _inside(x, n):
    """Clamp draws that rounded up to the upper domain edge back inside [0, n)."""
    return np.minimum(x, np.nextafter(float(n), 0.0))


def uniform_positions(rng, npart, n, ndim):
    x = np.zeros((3, npart))
    for d in range(ndim):
        x[d] = _inside(rng.random(npart) * n[d], n[d])
    return x


def clumped_positions(rng, npart_clumps, nclumps, sigma, n):
    """Gaussian clumps with uniformly drawn centres, wrapped periodically (3D)."""
    per = npart_clumps // nclumps
    centres = rng.random((nclumps, 3)) * np.asarray(n, dtype=np.float64)
    x = np.empty((3, per * nclumps))
    for c in range(nclumps):
        blk = rng.standard_normal((3, per)) * sigma
        for d in range(3):
            v = np.mod(centres[c, d] + blk[d], float(n[d]))
            x[d, c * per:(c + 1) * per] = _inside(v, n[d])
    return x


def gamma_of_v(v):
    return 1.0 / np.sqrt(1.0 - (v * v).sum(axis=0))


def maxwellian_u(rng, npart, sigma):
    """u = gamma v with each component of v drawn from N(0, sigma^2)."""
    v = rng.standard_normal((3, npart)) * sigma
    return v * gamma_of_v(v)


def isotropic_u(rng, npart, speed):
    """u = gamma v with |v| = speed exactly and direction uniform on the sphere."""
    g = rng.standard_normal((3, npart))
    v = g * (speed / np.sqrt((g * g).sum(axis=0)))
    return v * gamma_of_v(v)


@dataclass
class Species:
    kind: str            # "lorentz" | "dust" | "tracer"
    q: float = 1.0
    m: float = 1.0
    weight: float = 1.0
    t_stop: float = 0.0
    rk_stages: int = 2   # tracers: Runge-Kutta stages per step (2 or 3)


@dataclass
class Particles:
    x: np.ndarray        # (3, np) float64 grid coordinates
    u: np.ndarray        # (3, np) float64
    w: np.ndarray        # (np,) float64
    id: np.ndarray       # (np,) uint64

    @property
    def n(self):
        return int(self.x.shape[1])


@dataclass
class Box:
    ndim: int
    n: tuple             # (nx, ny, nz)
    fields: dict         # "E","B","vg" -> (3, nz, ny, nx) float64
    dx: tuple = (1.0, 1.0, 1.0)


@dataclass
class Item:
    box: int
    species: int
    particles: Particles


@dataclass
class Workload:
    name: str
    boxes: list
    species: list
    items: list
    dt: float
    steps: int
    shape: str = "tsc"
    sort_every: int = 0
    notes: dict = field(default_factory=dict)


def make_particles(x, u, weight=1.0):
    npart = x.shape[1]
    return Particles(x=np.ascontiguousarray(x), u=np.ascontiguousarray(u),
                     w=np.full(npart, float(weight)), id=np.arange(npart, dtype=np.uint64))


def turbulent_2d(n=(48, 16), npart=6000, steps=6, k=7, sigma_v=0.05):
    """2D periodic box (n[0] x n[1] cells) with turbulent in-plane fields and
    uniformly placed Maxwellian particles (a non-square grid, so that a
    swapped dimension shows)."""
    nn = (int(n[0]), int(n[1]), 1)
    flds = turbulent_fields(nn, SEED_B + k, SEED_V + k)
    rng = np.random.default_rng(SEED_P + k)
    x = uniform_positions(rng, npart, nn, 2)
    u = maxwellian_u(rng, npart, sigma_v)
    box = Box(ndim=2, n=nn, fields=flds)
    return Workload(name=f"turbulent 2D {nn[0]}x{nn[1]}, {npart} particles", boxes=[box],
                    species=[Species("lorentz")], items=[Item(0, 0, make_particles(x, u))],
                    dt=0.05, steps=steps)


def gyration_2d(npart=4096, n=32, steps=10, seed=SEED_P + 0):
    """2D 32x32 periodic grid, E=0, B=z, 4096 charged particles with |v| = 0.1c."""
    rng = np.random.default_rng(seed)
    nn = (n, n, 1)
    x = uniform_positions(rng, npart, nn, 2)
    u = isotropic_u(rng, npart, 0.1)
    box = Box(ndim=2, n=nn, fields=uniform_fields(nn))
    return Workload(name=f"gyration 2D {n}^2, {npart} particles", boxes=[box],
                    species=[Species("lorentz")], items=[Item(0, 0, make_particles(x, u))],
                    dt=0.05, steps=steps)


def turbulent_box(n=128, npart=1 << 24, steps=20, k=1, sigma_v=0.05):
    """3D periodic box with turbulent E, B and uniformly placed Maxwellian
    particles; n is the cell count per dimension, or three counts."""
    nn = tuple(int(v) for v in n) if isinstance(n, (tuple, list)) else (n, n, n)
    flds = turbulent_fields(nn, SEED_B + k, SEED_V + k)
    rng = np.random.default_rng(SEED_P + k)
    x = uniform_positions(rng, npart, nn, 3)
    u = maxwellian_u(rng, npart, sigma_v)
    box = Box(ndim=3, n=nn, fields=flds)
    shape = f"{n}^3" if nn[0] == nn[1] == nn[2] else "x".join(str(v) for v in nn)
    return Workload(name=f"turbulent {shape}, {npart} particles", boxes=[box],
                    species=[Species("lorentz")], items=[Item(0, 0, make_particles(x, u))],
                    dt=0.05, steps=steps)


def clumped_box(n=256, npart=1 << 26, nclumps=32, sigma=4.0, steps=20, k=3, sigma_v=0.05,
                sort_every=4):
    """Half the particles in Gaussian clumps, half uniform, turbulent fields."""
    nn = (n, n, n)
    flds = turbulent_fields(nn, SEED_B + k, SEED_V + k)
    rng = np.random.default_rng(SEED_P + k)
    half = npart // 2
    xc = clumped_positions(rng, half, nclumps, sigma, nn)
    xu = uniform_positions(rng, npart - xc.shape[1], nn, 3)
    x = np.concatenate([xc, xu], axis=1)
    u = maxwellian_u(rng, x.shape[1], sigma_v)
    box = Box(ndim=3, n=nn, fields=flds)
    return Workload(name=f"clumped {n}^3, {x.shape[1]} particles", boxes=[box],
                    species=[Species("lorentz")], items=[Item(0, 0, make_particles(x, u))],
                    dt=0.05, steps=steps, sort_every=sort_every)


def batched(n_main=192, n_cr=40_000_000, n_dust=8_000_000, n_tracer=1_000_000,
            n_small=64, n_boxes=16, small_lo=50_000, small_hi=2_000_000, steps=20, k=4,
            sigma_v=0.05, t_stop=0.1):
    """One large box with three species plus independent small boxes of charged particles.

    Species 0: charged (q/m = 1); species 1: dust (drag towards the gas velocity,
    stopping time t_stop, initially at rest); species 2: passive tracers.
    Small-box particle counts are log-uniform in [small_lo, small_hi].
    """
    boxes, items = [], []
    nn = (n_main,) * 3
    boxes.append(Box(ndim=3, n=nn, fields=turbulent_fields(nn, SEED_B + k, SEED_V + k)))
    rng = np.random.default_rng(SEED_P + k)
    species = [Species("lorentz"), Species("dust", t_stop=t_stop), Species("tracer")]
    x = uniform_positions(rng, n_cr, nn, 3)
    items.append(Item(0, 0, make_particles(x, maxwellian_u(rng, n_cr, sigma_v))))
    x = uniform_positions(rng, n_dust, nn, 3)
    items.append(Item(0, 1, make_particles(x, np.zeros((3, n_dust)))))
    x = uniform_positions(rng, n_tracer, nn, 3)
    items.append(Item(0, 2, make_particles(x, np.zeros((3, n_tracer)))))
    crng = np.random.default_rng(SEED_P + k + 100)
    counts = np.round(np.exp(crng.uniform(math.log(small_lo), math.log(small_hi), n_boxes))).astype(np.int64)
    ns = (n_small,) * 3
    for b in range(n_boxes):
        sb = 10000 + 100 * b
        boxes.append(Box(ndim=3, n=ns, fields=turbulent_fields(ns, sb, sb + 1)))
        prng = np.random.default_rng(sb + 2)
        npb = int(counts[b])
        x = uniform_positions(prng, npb, ns, 3)
        items.append(Item(b + 1, 0, make_particles(x, maxwellian_u(prng, npb, sigma_v))))
    return Workload(name="batched: main box with charged, dust and tracer species + small boxes",
                    boxes=boxes, species=species, items=items, dt=0.05, steps=steps,
                    notes={"small_counts": counts.tolist()})


def powerlaw_spectrum(nb=128, emin=1e2, emax=1e4, p=9.0, n0=1e-6):
    """The initial particle spectrum of the paper's shock test (Sec. 4.2):
    nb energies log-spaced from emin to emax and the power law
    chi = n0 (1 - p) / (emax^(1-p) - emin^(1-p)) * eps^(-p), whose integral
    over [emin, emax] is n0.  Returns (eng, chi), each of shape (nb,)."""
    eng = np.geomspace(emin, emax, nb)
    norm = n0 * (1.0 - p) / (emax ** (1.0 - p) - emin ** (1.0 - p))
    return eng, norm * eng ** (-p)


def scalar_field(n, seed, rms, kmax_frac=0.25, slope=-11.0 / 6.0):
    """Random scalar field on an n^3 periodic grid with the turbulent recipe's
    mode amplitudes (no projection), rescaled to the given rms.  Stands in for
    the fluid's four-velocity divergence (compressions and expansions)."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = n
    kx = np.fft.rfftfreq(nx, 1.0 / nx)
    ky = np.fft.fftfreq(ny, 1.0 / ny)
    kz = np.fft.fftfreq(nz, 1.0 / nz)
    KZ, KY, KX = np.meshgrid(kz, ky, kx, indexing="ij")
    kmag = np.sqrt(KX * KX + KY * KY + KZ * KZ)
    live = (kmag >= 1.0) & (kmag <= kmax_frac * min(nx, ny, nz))
    amp = np.zeros_like(kmag)
    amp[live] = kmag[live] ** slope
    coef = (rng.standard_normal(kmag.shape) + 1j * rng.standard_normal(kmag.shape)) * (amp / math.sqrt(2.0))
    f = np.fft.irfftn(coef, s=(nz, ny, nx), axes=(0, 1, 2))
    return f * (rms / math.sqrt(float(np.mean(f * f))))


def per_cell_positions(rng, ppc, n):
    """ppc particles in every cell of an n^3 grid, each uniform inside its
    cell, stored cell by cell (x fastest): how a grid code seeds a fixed
    number of particles per cell."""
    nx, ny, nz = n
    ncell = nx * ny * nz
    cell = np.repeat(np.arange(ncell, dtype=np.int64), ppc)
    base = np.stack([cell % nx, (cell // nx) % ny, cell // (nx * ny)]).astype(np.float64)
    x = base + rng.random((3, cell.shape[0]))
    for d in range(3):
        x[d] = _inside(x[d], n[d])
    return x


def spectra_box(n=160, ppc=4, nb=128, steps=10, k=5, divu_rms=0.1, dt=0.05):
    """The paper's Lagrangian-particle workload shape (Sec. 4.2, Table 1): n^3
    cells with ppc particles per cell (160^3 x 4 = 16 384 000 per GPU), seeded
    cell by cell, each carrying nb spectral points initialised to the power
    law of powerlaw_spectrum; turbulent B and gas velocity, and a random
    four-divergence field (rms divu_rms) for the adiabatic term.  The spectra
    are returned as one (nb,) template (every particle starts with it).  n is
    the cell count per dimension, or three counts."""
    nn = tuple(int(v) for v in n) if isinstance(n, (tuple, list)) else (n, n, n)
    flds = turbulent_fields(nn, SEED_B + k, SEED_V + k)
    flds["divu"] = scalar_field(nn, SEED_V + 100 + k, divu_rms)
    rng = np.random.default_rng(SEED_P + k)
    npart = ppc * nn[0] * nn[1] * nn[2]
    x = per_cell_positions(rng, ppc, nn)
    box = Box(ndim=3, n=nn, fields=flds)
    eng, chi = powerlaw_spectrum(nb)
    shape = f"{n}^3" if nn[0] == nn[1] == nn[2] else "x".join(str(v) for v in nn)
    return Workload(name=f"spectra {shape}, {npart} particles, {nb} bins", boxes=[box],
                    species=[Species("tracer")], items=[Item(0, 0, make_particles(x, np.zeros((3, npart))))],
                    dt=dt, steps=steps, notes={"eng0": eng, "chi0": chi})


def scaled(kind, scale):
    """Smaller versions of the workloads with the same recipe (for tests).

    ``scale`` divides the grid edge; particle counts keep the particles-per-cell.
    """
    if kind == "turbulent":
        n = 128 // scale
        return turbulent_box(n=n, npart=8 * n ** 3)
    if kind == "clumped":
        n = 256 // scale
        npart = 4 * n ** 3
        return clumped_box(n=n, npart=npart, nclumps=max(2, 32 // scale ** 3), sigma=4.0)
    raise ValueError(kind)
