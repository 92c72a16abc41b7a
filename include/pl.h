/*
 * pl.h -- C ABI of libpl.so, the MI355X (gfx950) particle-update library.
 *
 * One step of the update, for every particle of every item passed in:
 *   1. locate the particle's cell and TSC/CIC weights and gather the grid
 *      fields there (the particles sample the fluid at their position, Sec. 2
 *      after Eq. 1; the weights are the textbook CIC/TSC assignment functions);
 *   2. advance it: relativistic Boris push for charged particles, exact
 *      exponential drag towards the gas velocity for dust, a two- or
 *      three-stage Runge-Kutta step on the sampled gas velocity for passive
 *      tracers (Eq. 1, the paper's Lagrangian particles; two RK sub-steps per
 *      step in Sec. 3.3 and Table 1, second and third order in Sec. 4.1.1;
 *      pl_species_desc.rk_stages);
 *   3. deposit its moments (charge or mass density, current, force, energy
 *      change) onto the grid at the new position with the same weights.
 * A stable cell-tile counting sort groups particles by tile so the tiled
 * kernels can stage fields and deposits in LDS.
 *
 * Conventions
 * - Grid coordinates are in cell units: cell i spans [i, i+1), its centre is
 *   i + 1/2, the box is [0, n) per dimension and periodic.  Grid arrays are
 *   float64, cell-centred, flat index i + n[0]*(j + n[1]*k).
 * - Equations of motion (code units, speed of light c):
 *     charged:  du/dt = (q/m)(E + (u/gamma) x B),  gamma = sqrt(1 + |u|^2/c^2),
 *               dx/dt = u/gamma
 *     dust:     dv/dt = -(v - v_gas(x)) / t_stop,   dx/dt = v
 *     tracer:   dx/dt = v_gas(x)                    (Eq. 1)
 *   Positions advance by dt*v/dx per dimension.  The velocity passed in is
 *   the one at the previous half step (leapfrog).
 * - Deposited channels per unit cell volume dV = dx*dy(*dz), at the new
 *   position:  rho = q w (dust: m w);  J = q w v;  F = m w du/dt (the momentum
 *   change over the step divided by dt);  eng = m w c^2 dgamma/dt.
 *
 * Ownership and streams
 * - Every particle, field and moment array is caller-owned DEVICE memory
 *   (e.g. torch tensors' data_ptr()).  The library owns only the context and
 *   the scratch it allocates in pl_part_init; no other call allocates.
 * - All work is queued on the context's stream and is asynchronous; results
 *   are ready after pl_part_sync() (or any later stream synchronisation).
 * - One context per stream; calls on one context must not overlap.
 *
 * Errors
 * - Every call returns a pl_status.  Argument errors are detected on the host
 *   before any device work is queued and leave all data untouched.
 * - Device-side conditions (a particle that moved a full cell or more in one
 *   step, a non-finite or out-of-range particle coordinate, an item whose
 *   tile offsets do not describe its particles) are latched in the context
 *   and returned by the next pl_part_sync() as PL_ECFL / PL_ENONFINITE /
 *   PL_ENOTSORTED; particles with a bad coordinate are still processed with
 *   wrapped, in-range indices, the particles of an unsorted item are left
 *   untouched and deposit nothing.
 */
#ifndef PL_H
#define PL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int pl_status;
#define PL_OK            0
#define PL_EINVAL        1   /* invalid argument (null/misaligned pointer, bad size or enum) */
#define PL_ENOMEM        2   /* device or pinned-host allocation failed in pl_part_init */
#define PL_EHIP          3   /* a HIP runtime call failed */
#define PL_EUNSUPPORTED  4   /* valid request the library does not implement */
#define PL_ECFL          5   /* a particle moved a full cell or more in one step */
#define PL_ENONFINITE    6   /* a particle coordinate was non-finite or outside the grid */
#define PL_ENOTSORTED    7   /* PL_ALGO_TILED / PL_ALGO_RUNS met an item whose p.tile_start (or run
                                table) does not cover its p.n particles: never sorted, sorted by a
                                context of another algorithm, or its count changed since the sort.
                                That item's particles were left untouched and nothing was
                                deposited for them */
#define PL_ENOSPACE      8   /* pl_sort_noalloc: an item holds more than PL_NOALLOC_MAX_NP particles */

/* Storage / arithmetic form of the particles. */
#define PL_F64         0   /* float64 absolute grid coordinates and velocities */
#define PL_F32_OFFSET  1   /* packed uint32 cell + float32 offsets from the cell centre, float32 u */

#define PL_CIC 1
#define PL_TSC 2

#define PL_LORENTZ 0       /* charged particle, relativistic Boris */
#define PL_DUST    1       /* dust grain, drag towards the gas velocity */
#define PL_TRACER  2       /* passive tracer of the gas velocity (Eq. 1) */

#define PL_ALGO_PLAIN 0    /* one thread per particle, fields and deposits straight from/to HBM */
#define PL_ALGO_TILED 1    /* per-tile LDS field stage and LDS deposit (needs pl_part_sort) */
#define PL_ALGO_RUNS  2    /* per-tile LDS kernel in which each thread advances a run of up to
                              four particles of one cell in register batches (four float32 or two
                              float64 particles): each batch particle gathers its fields from the
                              LDS field tile, and the batch's deposits into a stencil point are
                              summed in registers before one LDS atomic per channel (3D/2D,
                              TSC/CIC; charged, dust and, from the same field tile, tracer
                              species; push-only and deposit-only calls run the PL_ALGO_TILED
                              kernel).
                              Needs pl_part_sort with PL_KEY_TILE_CELL or PL_KEY_TILE_RUN,
                              which writes p.runs */

/* Work units beyond one per tile that pl_part_sort may create by splitting
 * crowded tiles (PL_ALGO_RUNS), and the length of the run table. */
#define PL_RUNS_SPLIT_UNITS 1024
#define PL_RUNS_LEN(n, ntiles) ((int64_t)(n) + 3 * (int64_t)(ntiles) + 2 * PL_RUNS_SPLIT_UNITS + 1)

#define PL_KEY_TILE       0  /* sort by tile */
#define PL_KEY_TILE_CELL  1  /* sort by tile, then by cell inside the tile (x fastest) */
#define PL_KEY_TILE_RANK  2  /* sort by tile, then by rank among the particles of the same cell
                                (0 for the first in array order, ...), then by cell: consecutive
                                particles lie in distinct cells.  Ranks of 2^rb - 1 and above share
                                one level, rb = min(10, 32 - tile bits - cell-in-tile bits) >= 3 */
#define PL_KEY_TILE_RUN   3  /* PL_ALGO_RUNS only: sort by tile, then by (rank in cell) / 4, then by
                                cell, then by (rank in cell) % 4, ranks in stable tile+cell order:
                                each run of the run table is contiguous and the runs of a tile
                                lie in table order, so the lanes of a wave read and write one
                                contiguous stretch of every particle array.  Cells are numbered
                                x fastest, with the rows y of every group of eight taken in the
                                order 0, 2, 4, 6, 1, 3, 5, 7 when the tile's y size is a multiple
                                of 8, else those of every group of four in the order 0, 2, 1, 3
                                when it is a multiple of 4 */

/* flags of pl_part_gather_push / pl_part_deposit */
#define PL_FUSE_DEPOSIT  (1u << 0)  /* gather_push also deposits at the new positions */
#define PL_ZERO_FIRST    (1u << 1)  /* zero the items' moment grids before depositing */
#define PL_GRAPH         (1u << 2)  /* record the call's launches once as a hipGraph, replay afterwards */
#define PL_SUMS          (1u << 3)  /* accumulate particle-side conservation sums (see pl_part_sums) */
#define PL_SORT_FIRST    (1u << 4)  /* gather_push: sort every item first, exactly as pl_part_sort (tiled
                                       and run-based algorithms); with PL_GRAPH the sort's launches are
                                       recorded in the same graph as the zeroing and the step */

typedef struct pl_ctx pl_ctx;

typedef struct {
    int n[3];         /* cells per dimension (n[2] == 1 in 2D); each 1..1024 */
    double dx[3];     /* cell size per dimension (> 0) */
    int tile[3];      /* tile edge in cells (sort key, LDS tile); must divide n; tile[2] == 1 in 2D */
} pl_box_desc;

typedef struct {
    int kind;         /* PL_LORENTZ, PL_DUST or PL_TRACER */
    double q, m;      /* charge and mass per unit weight (m > 0) */
    double weight;    /* weight of every particle when an item passes no weights */
    double t_stop;    /* dust stopping time (> 0 for PL_DUST) */
    int rk_stages;    /* PL_TRACER: Runge-Kutta stages per step with the gas velocity frozen over the
                         step (Eq. 1): 2 (Heun; also 0) or 3 (the three-stage strong-stability-preserving
                         scheme of Shu and Osher, the paper's third-order option, Sec. 4.1.1); ignored
                         by the other kinds */
} pl_species_desc;

typedef struct {
    int ndim;                        /* 2 or 3, for every box of the context */
    int prec;                        /* PL_F64 or PL_F32_OFFSET */
    int shape;                       /* PL_CIC or PL_TSC */
    int algo;                        /* PL_ALGO_PLAIN, PL_ALGO_TILED or PL_ALGO_RUNS */
    int key_mode;                    /* PL_KEY_TILE, PL_KEY_TILE_CELL, PL_KEY_TILE_RANK or
                                        PL_KEY_TILE_RUN */
    double c;                        /* speed of light in code units (> 0) */
    int nboxes;
    const pl_box_desc *boxes;        /* host array, copied */
    int nspecies;
    const pl_species_desc *species;  /* host array, copied */
    int max_items;                   /* most items any one call passes (>= 1) */
    int64_t max_np;                  /* most particles in any one item (sizes the sort scratch) */
    int block;                       /* threads per block of the particle kernels (64..512, multiple of 64;
                                        with PL_ALGO_RUNS: 512, the run-based kernel's block);
                                        0 = default */
    void *stream;                    /* hipStream_t for all work; NULL = the null stream */
    const char *tune_cache;          /* nullable: file written by the autotuner ("key value" lines: block,
                                        runs_block, tile, and one_launch 0 to give each species kind its
                                        own launch in fused run-based steps) */
} pl_init_desc;

/*
 * Particles of one item, structure of arrays, two buffer sets: the sort reads
 * set `cur` and writes set 1-cur, then flips `cur`.  Set 1-cur may be left
 * NULL by callers that never sort.  Pointers are device pointers aligned to
 * their element size.
 */
typedef struct {
    int64_t n;              /* particle count, 0 <= n <= max_np, n < 2^31 */
    int cur;                /* 0 or 1: the set holding the current state */
    uint32_t *cell[2];      /* PL_F32_OFFSET: cell i | j<<10 | k<<20;  PL_F64: unused */
    void *x[2][3];          /* PL_F64: double grid coordinates; PL_F32_OFFSET: float offsets in [-1/2, 1/2) */
    void *u[2][3];          /* velocity (u = gamma v for charged particles), double or float */
    void *w[2];             /* nullable: per-particle weights (double or float) */
    uint64_t *id[2];        /* nullable: particle ids, carried through the sort */
    void *fp[3];            /* nullable: per-particle force m w du/dt, written by gather_push, read by deposit */
    int32_t *tile_start;    /* ntiles+1 first-particle offsets per tile, written by pl_part_sort;
                               required by PL_ALGO_TILED and PL_ALGO_RUNS */
    int32_t *runs;          /* nullable: PL_RUNS_LEN(n, ntiles) run-table entries written by
                               pl_part_sort with PL_ALGO_RUNS: the runs of tile t at
                               [tile_start[t], ...), their count at runs[n + t], the work units
                               in processing order as pairs (tile, piece | npieces << 16) at
                               runs[n + ntiles + 2g], and the number of units at
                               runs[n + ntiles + 2 * (ntiles + PL_RUNS_SPLIT_UNITS)]; required by
                               PL_ALGO_RUNS, n < 2^29 */
    int nbins;              /* spectral points per particle for pl_part_spectra (0: none) */
    double *eng[2];         /* nullable: energies of each particle's spectral points, particle-major
                               (eng[s][p * nbins + i]), both buffer sets like x and u: the sort and
                               the compaction move a particle's row with it */
    double *chi[2];         /* nullable: number fraction chi = N / n at those energies (Eq. chi),
                               same layout */
} pl_particles;

typedef struct {
    const double *E[3];     /* charged particles: electric field (the E of du/dt above) */
    const double *B[3];     /* charged particles: magnetic field */
    const double *vg[3];    /* dust and tracers: gas velocity */
    const double *divu;     /* pl_part_spectra: four-divergence of the fluid velocity, div_mu u^mu */
} pl_fields;

typedef struct {
    double *rho;            /* charge density (charged) or mass density (dust) */
    double *J[3];           /* current density, charged only */
    double *F[3];           /* force density m w du/dt, charged and dust */
    double *eng;            /* energy-change density, charged only */
} pl_moments;               /* NULL channels are skipped; tracers deposit nothing */

typedef struct {
    int box;                /* index into pl_init_desc.boxes */
    int species;            /* index into pl_init_desc.species */
    pl_particles p;
    pl_fields f;
    pl_moments m;
} pl_item;

/*
 * pl_part_init: validate the description, allocate every piece of scratch the
 * library will ever use (sort buffers for max_np particles, item tables for
 * max_items, work counters, latched-error flags, pinned staging) and create
 * the context.  Reads tune_cache when given.  On error *out is NULL.
 * Source: the paper's two memory rules for the particle module (Sec. 3.2):
 * data stay resident on the device for the whole run, and allocation is kept
 * out of the time step; here every device buffer the library needs exists
 * from this call on, and the caller owns all particle and grid storage.
 */
pl_status pl_part_init(pl_ctx **out, const pl_init_desc *d);

/*
 * pl_part_gather_push: advance every particle of items[0..nitems) by one step
 * of length dt (finite, non-zero): gather at x^n, push, new position x^{n+1}
 * (periodic wrap).  Kinds, fields and channels are described above.
 * Sources: the particles sample the fluid at their own position and tracers
 * move with it (Sec. 2, Eq. 1; two Runge-Kutta sub-steps per step, Sec. 3.3,
 * Table 1; second- and third-order schemes, Sec. 4.1.1).  The weights are the
 * cloud-in-cell and triangular-shaped-cloud assignment functions of Hockney &
 * Eastwood (Computer Simulation Using Particles, 1988, ch. 5), the same at
 * gather and deposit.  Charged particles take the relativistic Boris push
 * (Boris 1970: half electric kick, magnetic rotation, half kick, u^{n-1/2} ->
 * u^{n+1/2}); dust takes the exact solution of linear drag with the gas
 * velocity frozen over the step.  With PL_FUSE_DEPOSIT every channel is
 * deposited at x^{n+1}, J with u^{n+1/2}, F = m w (u^{n+1/2} - u^{n-1/2})/dt.
 * When p.fp is given it receives F of each particle, in the particle order of
 * this call.  With PL_ALGO_RUNS and PL_FUSE_DEPOSIT every item of the call,
 * of every species kind, goes to one persistent launch whose blocks claim
 * (item, tile piece) work units from one counter and run each with its
 * item's kind (unless the tune cache says one_launch 0); otherwise the items
 * of each kind share one launch.
 *   PL_FUSE_DEPOSIT  deposit the items' non-NULL moment channels at x^{n+1}
 *                    in the same pass (added to the grids' contents);
 *   PL_ZERO_FIRST    zero those channels first;
 *   PL_SUMS          accumulate per-item particle-side sums (pl_part_sums);
 *   PL_GRAPH         record the launches as a hipGraph keyed by the call's
 *                    arguments and replay it on later identical calls
 *                    (the stream must not be the null stream);
 *   PL_SORT_FIRST    sort every item first (pl_part_sort's result, cur
 *                    flipped), then zero and step: with PL_GRAPH the whole
 *                    sequence is one graph, a separate one per buffer set.
 * Items must not share particle arrays; items sharing a moment grid add into
 * it.
 */
pl_status pl_part_gather_push(pl_ctx *ctx, pl_item *items, int nitems, double dt, uint32_t flags);

/*
 * pl_part_deposit: deposit the current state of every item (no push): rho and
 * J from the particles, F from p.fp (required when m.F is set), eng is not
 * available here (must be NULL).  PL_ZERO_FIRST zeroes the channels first.
 * Source: charge assignment with the same cloud-in-cell / triangular-shaped-
 * cloud weights as the gather (Hockney & Eastwood 1988, ch. 5), so deposit
 * is the adjoint of gather and total charge is conserved exactly; the
 * particles are taken at their current positions.  p.fp is in the particle
 * order of the gather_push that wrote it and a sort does not move it, so an
 * F deposit must come before the next pl_part_sort: a deposit with m.F set
 * after a sort of the item, with no gather_push writing p.fp in between,
 * returns PL_EINVAL.
 */
pl_status pl_part_deposit(pl_ctx *ctx, const pl_item *items, int nitems, uint32_t flags);

/*
 * pl_part_sort: stable sort of each item's particles by cell-tile key (the
 * context's key_mode and the box's tile), moving every SoA array (cell, x, u,
 * w, id) from set cur into set 1-cur, writing p.tile_start, and flipping
 * items[i].p.cur.  p.fp is not moved (see pl_part_deposit).
 * Source: the paper stores its particles in no particular order and only
 * compacts them (Sec. 3.2); this sort is the library's own locality step, the
 * cell-tile sort that particle-in-cell codes use so a tile's particles are
 * contiguous and its fields and deposits fit in on-chip memory.  It is a least
 * significant digit radix sort (8-bit digits, stable scatter), so the
 * permutation equals a stable comparison sort on the same keys.  Equal keys keep their order (bit-identical to a stable
 * sort).  Requires the 1-cur set for every non-NULL array of set cur.
 * With PL_ALGO_RUNS it also writes p.runs: the particles of every cell are
 * cut into runs of up to four consecutive sorted particles, and the runs of a
 * tile are listed by (index of the run inside its cell, cell in tile), each
 * entry holding (first particle << 2) | (length - 1).  It then lists the
 * work units of the run kernel: with P = max(ceil(total runs / 1024), 1024)
 * runs, a tile of c runs becomes ceil(c / P) pieces of equal run count (an
 * empty tile none).  Tiles cut into several pieces or holding more than twice
 * the mean run count come first (the first 1024 such tiles in index order,
 * by decreasing runs per piece, ties by tile index), each with its pieces in
 * order, then the other non-empty tiles in index order.  Piece k of a tile
 * takes runs [c*k/npieces, c*(k+1)/npieces).  With PL_KEY_TILE_RUN the
 * particles of every tile are stored in run order (the runs one after another
 * in table order from tile_start[t]) and the entries point there.
 */
pl_status pl_part_sort(pl_ctx *ctx, pl_item *items, int nitems);

/*
 * pl_sort_noalloc: pl_part_sort for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  It needs no context: d is validated as by
 * pl_part_init (ndim, prec, algo, key_mode, boxes with their tiles given,
 * species, max_items, max_np; block and tune_cache are ignored) and the work
 * is queued on d->stream.  The result is exactly that of pl_part_sort with a
 * context made from d: same permutation, tile offsets, run table and flip of
 * items[i].p.cur.  The sort's own scratch (keys, indices, digit histograms)
 * is a fixed array inside the library, about 17 MB, which every GPU the
 * library runs on holds until the process ends; nothing is allocated, and
 * the array is set up on the first call on each device.
 * Limits and errors: an item with more than PL_NOALLOC_MAX_NP particles
 * returns PL_ENOSPACE, PL_KEY_TILE_RANK (per-cell scratch) and devices
 * numbered 64 and above return PL_EUNSUPPORTED, a box without a tile
 * returns PL_EINVAL; all of them before any device work.  All calls on one
 * GPU share the array: calls that overlap on one GPU (several streams or
 * threads) race; calls queued on one stream are ordered and safe.
 */
#define PL_NOALLOC_MAX_NP (1 << 20)
pl_status pl_sort_noalloc(const pl_init_desc *d, pl_item *items, int nitems);

/*
 * pl_part_spectra: advance the energy distribution of every particle of
 * every item with nbins > 0 by one step dt (finite, non-zero): Sec. 2,
 * Eqs. cr_N to cr_chi with the losses of Eq. rad_losses.  At the particle's
 * current position the fluid's B, gas velocity vg and four-divergence divu
 * are sampled with the box's CIC/TSC weights; then, with a = divu / 3,
 * c_r = s->cr (s->ub |B|^2 + s->u_rad), d tau = dt / gamma_g
 * (gamma_g = 1 / sqrt(1 - |vg|^2 / c^2)), E = exp(-a d tau) and
 * phi = (1 - E) / a (d tau when a = 0), each spectral point moves on its
 * characteristic d eps / d tau = -a eps - c_r eps^2, solved exactly:
 *     den = 1 + c_r eps phi,  eps <- eps E / den,  chi <- chi den^2 / E,
 * so chi d eps (the number between neighbouring points) is conserved.
 * Arithmetic is float64 in both particle forms.  Any species kind; the item
 * needs f.B, f.vg and f.divu, and p.eng / p.chi of its current set.  One
 * launch for all items.  Errors: a null or misaligned array, nbins outside
 * 1..4096, a non-finite or negative coefficient: PL_EINVAL.  A gas speed at
 * or above c latches PL_ENONFINITE (that particle's spectrum is left as it
 * was).
 */
typedef struct {
    double cr;        /* loss coefficient per unit energy density (Eq. rad_losses prefactor) */
    double u_rad;     /* radiation energy density U_rad */
    double ub;        /* magnetic energy density per |B|^2: U_B = ub |B|^2 (1/2 in Heaviside-Lorentz units) */
} pl_spectra_desc;
pl_status pl_part_spectra(pl_ctx *ctx, const pl_item *items, int nitems, double dt, const pl_spectra_desc *s);

/*
 * pl_part_boundary: delete the particles that left through open boundaries
 * and compact every item's current set (Sec. 3.2).  A dimension d with
 * bc->open[d] != 0 keeps bc->ghost (>= 2) layers of boundary cells on each
 * side: a particle whose cell lies outside the active cells
 * [ghost, n[d] - ghost) is deleted.  (With a push of less than a cell per
 * step and this call after every step, no stencil of an active particle
 * reaches across the periodic seam of an open dimension.)  The compaction is
 * the paper's holes-and-fillers algorithm: with ndel particles deleted, the
 * k-th deleted particle below n - ndel (in index order) is overwritten by the
 * k-th surviving particle at or above n - ndel (in index order), every array
 * of the set moving together (cell, x, u, w, id and the spectral rows); the
 * other survivors keep their index.  O(n) work, scratch from pl_part_init.
 * Synchronous: waits for the stream, then sets items[i].p.n to the new count
 * and, when removed is not NULL, removed[i] to the number deleted.  An item
 * that lost particles has its tile offsets marked unsorted (PL_ENOTSORTED
 * until the next pl_part_sort); p.fp is not moved.  Errors: bad arguments,
 * ghost < 2 or 2 * ghost >= n[d] in an open dimension: PL_EINVAL.
 */
typedef struct {
    int open[3];      /* nonzero: outflow boundaries on both sides of dimension d */
    int ghost;        /* boundary cells on each open side (>= 2) */
} pl_boundary_desc;
pl_status pl_part_boundary(pl_ctx *ctx, pl_item *items, int nitems, const pl_boundary_desc *bc, int64_t *removed);

/*
 * pl_part_inject: append k particles to item->p's current set at indices
 * [n, n + k) (the paper's particles can be injected at run time, Sec. 3.2):
 * x[3] grid coordinates and u[3] velocities as float64 device arrays
 * (converted to the storage form as pl_part_pack does), w (nullable: set to
 * the species weight when the set has weights), id (nullable), eng / chi
 * (nullable; k * nbins float64, particle-major, when the set has spectra).
 * cap is the capacity of the caller's arrays (in particles); n + k must not
 * exceed cap or max_np.  Sets item->p.n to n + k and marks the item unsorted
 * (PL_ENOTSORTED until the next pl_part_sort).  Asynchronous.  Errors: a null
 * context, item, x or u, k < 0, n + k above cap or max_np, a null or
 * misaligned array the set needs (eng and chi when it has spectra), or an
 * item the context rejects: PL_EINVAL, before any device work; a failed
 * launch: PL_EHIP.  k = 0 is a no-op.
 */
pl_status pl_part_inject(pl_ctx *ctx, pl_item *item, int64_t k, const double *x[3], const double *u[3],
                         const double *w, const uint64_t *id, const double *eng, const double *chi, int64_t cap);

/*
 * pl_part_pack: write item->p's current set from float64 device arrays
 * x[3] (grid coordinates, wrapped into the box) and u[3]; for PL_F32_OFFSET
 * this splits each coordinate into the packed cell and the float32 offset
 * (an offset that rounds to +1/2 moves to the next cell at -1/2).
 * pl_part_unpack writes the current state back as float64 grid coordinates
 * and velocities.  x[2] may be NULL in 2D.
 */
pl_status pl_part_pack(pl_ctx *ctx, const pl_item *item, const double *x[3], const double *u[3]);
pl_status pl_part_unpack(pl_ctx *ctx, const pl_item *item, double *x[3], double *u[3]);

/*
 * pl_part_sums: synchronous.  For each item writes 16 doubles to host array
 * out: [0..8) grid sums of rho, J[3], F[3], eng times dV (0 for NULL
 * channels), [8..16) the matching particle-side sums accumulated by the last
 * gather_push called with PL_SUMS (sum q w (dust: m w), sum q w v, sum m w
 * du/dt, sum m w c^2 dgamma/dt).  Conservation means the halves agree.
 */
pl_status pl_part_sums(pl_ctx *ctx, const pl_item *items, int nitems, double *out);

/* Wait for the context's stream; return and clear latched device errors. */
pl_status pl_part_sync(pl_ctx *ctx);

/* Change the stream later work is queued on (drops recorded graphs). */
pl_status pl_part_set_stream(pl_ctx *ctx, void *stream);

/* Diagnostics, counted since pl_part_init; writes min(n, PL_NSTATS) entries:
 * out[0] kernel launches, out[1] graph replays, out[2] graph recordings,
 * out[3] sorts, out[4] launches of the run-based kernel, out[5] PL_ALGO_RUNS
 * launch groups that took the tiled kernel because the run-based kernel's
 * LDS footprint exceeds the device's, out[6] launches of a run-based kernel
 * compiled for a fixed tile shape and channel set, out[7] the variant of the
 * last run-based launch: ts | chs << 4 | hf << 8 | mixed << 12, with mixed = 1
 * when the launch took items of several kinds (or tracers), ts the fixed tile
 * (1: 8x8x8, 2: 8x8x4, 0: taken at run time), chs the fixed channel set
 * (1: rho J F of charged particles, 2: rho F of dust, 0: taken at run time;
 * a mixed launch reports its charged items' set)
 * and hf the field halo in cells (1 or 2). */
#define PL_NSTATS 8
pl_status pl_part_stats(pl_ctx *ctx, int64_t *out, int n);

/* Free the context and its scratch (synchronises first).  NULL is a no-op. */
void pl_part_finalize(pl_ctx *ctx);

/* Static text for a status code. */
const char *pl_status_string(pl_status s);

#ifdef __cplusplus
}
#endif

#endif /* PL_H */
