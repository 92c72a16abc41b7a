// Internal declarations shared by the HIP sources of libpl.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/pl.h"

namespace pl {

constexpr int kMaxCh = 8;            // rho, J0, J1, J2, F0, F1, F2, eng
constexpr int kCellBits = 10;        // packed cell: 10 bits per dimension
constexpr int kMaxN = 1 << kCellBits;
constexpr int kMaxDigitBits = 8;     // radix digit of the sort (256 counters per block and wave)
constexpr int kRunLen = 4;           // particles per run of the run table (PL_ALGO_RUNS)
constexpr int kRunsMaxTileCells = 1024;
constexpr int kRunsSplit = PL_RUNS_SPLIT_UNITS;   // work units beyond one per tile
constexpr int kQueues = 8;          // run kernels: chunks of the unit slots, one counter each
constexpr int kCounterStride = 16;  // counters per launch stage (kQueues + 1 used by the run kernels)
constexpr int kCounterSlots = 4 * kCounterStride;   // one stage per species kind, plus one
static_assert(kQueues + 1 <= kCounterStride, "a run-kernel stage needs kQueues + 1 counters");
constexpr int kRunsMinPiece = 1024;               // smallest run count worth a split

// Run table of an item (PL_ALGO_RUNS), offsets from runs[0]: unit g is the
// pair at units_at + 2g, the unit count at count_at.
__host__ __device__ inline int64_t runs_units_at(int64_t np, int ntiles) { return np + ntiles; }
__host__ __device__ inline int64_t runs_count_at(int64_t np, int ntiles)
{
    return np + ntiles + 2 * ((int64_t)ntiles + kRunsSplit);
}

enum Channel { CH_RHO = 0, CH_J0 = 1, CH_F0 = 4, CH_ENG = 7 };

// Latched device-side error bits.
enum ErrBit { ERR_CFL = 1, ERR_NONFINITE = 2, ERR_UNSORTED = 4 };

// Mode bits of the step kernels.
enum StepFlag : unsigned {
    SF_PUSH = 1u,       // advance particles (else: deposit the current state)
    SF_DEPOSIT = 2u,    // deposit moments
    SF_SUMS = 4u,       // particle-side conservation sums
    SF_RUNS = 8u,       // tiled: each thread takes a contiguous run of the tile's particles
    SF_FHALO2 = 16u,    // run-based: the LDS field tile carries a two-cell halo
};

// Everything a kernel needs to know about one item of a call.  Built on the
// host for every call, uploaded into the context's item table.
struct ItemDesc {
    // box
    int n[3];
    int tile[3];
    int ntile[3];
    int ntiles;
    double inv_dv;
    double dtdx[3];          // dt / dx per dimension
    float dtdx_f[3];
    // species
    int kind;
    int rk;                  // tracers: Runge-Kutta stages (2 or 3)
    double h;                // (q/m) dt / 2
    double q, m, wdef;
    double decay;            // dust: exp(-dt/t_stop)
    double one_m_decay;      // dust: 1 - exp(-dt/t_stop)
    double inv_dt;
    double c2, inv_c2;
    // particles, current buffer set
    int np;
    uint32_t *cell;
    void *x[3];
    void *u[3];
    void *w;
    void *fp[3];
    int32_t *tile_start;
    int32_t *runs;           // run table (PL_ALGO_RUNS)
    uint64_t *id;            // nullable: particle ids (current set)
    double dt;               // the call's time step
    int nb;                  // spectral points per particle (0: none)
    double *eng;             // spectral energies, particle-major (current set)
    double *chi;             // spectral number fractions, same layout
    // fields
    const double *E[3];
    const double *B[3];
    const double *vg[3];
    const double *divu;      // four-divergence of the fluid velocity (spectra)
    // moments
    double *M[kMaxCh];
    int slot[kMaxCh];        // LDS slot of each active channel, -1 if inactive
    int nslot;
    // work decomposition
    int unit_begin;          // first global work unit of this item
    int nunits;
    int chunk;               // particles per unit (plain algorithm)
    double *psum;            // particle-side sums, 8 doubles
};

struct GraphEntry {
    uint64_t key = 0;
    bool valid = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ItemDesc *table = nullptr;       // device table owned by this graph
    int nitems = 0;
    uint64_t last_use = 0;
};

struct Ctx {
    pl_init_desc d;
    std::vector<pl_box_desc> boxes;
    std::vector<pl_species_desc> species;
    hipStream_t stream = nullptr;
    int device = 0;
    int num_cu = 0;
    int block = 256;
    int lds_max = 65536;
    bool runs = false;               // tiled: contiguous per-thread particle runs (tune cache "runs 1")
    int runs_block = 512;            // block size of the run-based kernels (init block or tune cache "runs_block")
    bool one_launch = true;          // fused run-based steps over several kinds: one launch (tune cache
                                     // "one_launch 0": one launch per kind)

    // device scratch
    ItemDesc *table = nullptr;       // max_items descriptors for non-graph calls
    unsigned *counters = nullptr;    // work counters: kCounterStride per launch stage
    int *errflags = nullptr;         // latched error bits
    double *sums = nullptr;          // max_items * 16
    uint32_t *keys[2] = {nullptr, nullptr};
    uint32_t *idx[2] = {nullptr, nullptr};
    uint32_t *hist = nullptr;        // radix digit counts
    int32_t *cell_start = nullptr;   // rank-interleaved sort: first sorted position of every cell
    uint32_t *hist_scan = nullptr;
    int64_t hist_cap = 0;
    int64_t max_np = 0;
    int max_ntiles = 0;

    // pinned staging ring for item tables
    static constexpr int kRing = 8;
    ItemDesc *pinned = nullptr;      // kRing * max_items
    hipEvent_t ring_ev[kRing] = {};
    int ring_pos = 0;

    // graphs
    static constexpr int kGraphs = 8;
    GraphEntry graphs[kGraphs];
    uint64_t use_clock = 0;

    // launches, graph replays, graph captures, sorts, run-kernel launches, run
    // groups on the tiled kernel, fixed-shape run-kernel launches, variant of
    // the last run-kernel launch (pl.h, pl_part_stats)
    int64_t stats[PL_NSTATS] = {0, 0, 0, 0, 0, 0, 0, 0};

    // p.fp arrays whose particles a sort has reordered since a gather_push
    // last wrote them: a deposit of F from them is refused
    std::vector<const void *> fp_stale;
};

// Launch configuration of the run kernel for one launch's items: field halo,
// compile-time tile shape (0 generic, 1 8^3, 2 8x8x4), channel sets of the
// charged (1: rho J F) and dust (2: rho F) items, LDS bytes, and whether the
// items mix species kinds (one launch dispatching per unit).
struct RunsPlan {
    int hf = 0, ts = 0, chl = 0, chd = 0;
    size_t lds = 0;
    bool mixed = false;
};
bool runs_plan(const Ctx *c, const ItemDesc *host, int nitems, RunsPlan &pl);

// Kernel launchers (k_step.hip)
hipError_t launch_step(Ctx *c, const ItemDesc *table, const std::vector<ItemDesc> &host, int nitems,
                       int total_units, unsigned flags, bool deposit, bool push);
hipError_t launch_zero(Ctx *c, const ItemDesc *table, const std::vector<ItemDesc> &host);
hipError_t launch_zero_sums(Ctx *c, double *sums, int n);
hipError_t launch_grid_sums(Ctx *c, const ItemDesc &it, double *out8);
hipError_t launch_pack(Ctx *c, const ItemDesc &it, int prec, int ndim, const double *x[3], const double *u[3]);
hipError_t launch_unpack(Ctx *c, const ItemDesc &it, int prec, int ndim, double *x[3], double *u[3]);

// Lagrangian-particle extras (k_lp.hip)
constexpr int kMaxBins = 4096;
hipError_t launch_spectra(Ctx *c, const ItemDesc *table, const std::vector<ItemDesc> &host, double cr,
                          double u_rad, double ub);
// Deletion at open boundaries and compaction of one item; writes the new
// count and the number removed (int64) to host memory, synchronously.
hipError_t launch_boundary(Ctx *c, const ItemDesc &it, const pl_boundary_desc &bc, int ndim, int64_t *keep,
                           int64_t *removed);
// Weights, ids and spectral rows of k injected particles at [it.np, it.np + k)
// (positions and velocities go through launch_pack); marks the item unsorted.
hipError_t launch_inject_rest(Ctx *c, const ItemDesc &it, int64_t k, const double *w, bool has_w, double wdef,
                              const uint64_t *id, uint64_t *id_dst, const double *eng, const double *chi);

// Sort (k_sort.hip)
struct SortArgs {
    int prec, ndim, key_mode;
    int n[3], tile[3];
    int np;
    int ntiles;
    const uint32_t *cell;            // F32_OFFSET
    const double *x[3];              // F64
    // source and destination arrays (element sizes given): cell, 3 x, 3 u, w, id
    static constexpr int kMaxArrays = 12;
    const void *src[kMaxArrays];
    void *dst[kMaxArrays];
    int esize[kMaxArrays];
    int narrays;
    int32_t *tile_start;
    int32_t *runs;                   // nullable: run table to build (PL_ALGO_RUNS)
    // spectral rows (nb doubles per particle) moved with the particles
    int nb;
    const double *rsrc[2];
    double *rdst[2];
};
hipError_t launch_sort(Ctx *c, const SortArgs &a);
// The same sort with its scratch in the library's fixed device array (set up
// on the first call on each device); c supplies the stream only.
hipError_t launch_sort_noalloc(Ctx *c, const SortArgs &a);

}  // namespace pl
