/*
 * Reference CPU implementation ("oracle") of the per-step particle update:
 * gather of grid fields to particles with CIC/TSC weights, Boris / drag /
 * tracer advance, deposit of particle moments, the stable cell-tile sort, the
 * Lagrangian spectral update, and deletion with compaction at open
 * boundaries.
 *
 * TEST INFRASTRUCTURE ONLY.  The test-suite, the smoke check and the
 * benchmark's CPU-baseline leg call it; the GPU library never includes,
 * links or calls anything here, and nothing here includes GPU code.
 *
 * Everything is IEEE double precision, built with -ffp-contract=off so that no
 * multiply-add is fused behind the reader's back.  Grid coordinates are in
 * cell units: cell i spans [i, i+1), its centre is i + 1/2, the box is [0, N)
 * per dimension and periodic.  Grid arrays are flat, index i + nx*(j + ny*k).
 */
#ifndef ORC_H
#define ORC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_CIC = 1, ORC_TSC = 2 };
enum { ORC_LORENTZ = 0, ORC_DUST = 1, ORC_TRACER = 2 };
enum { ORC_KEY_TILE = 0, ORC_KEY_TILE_CELL = 1, ORC_KEY_TILE_RANK = 2 };

typedef struct {
    int ndim;        /* 2 or 3; in 2D n[2] == 1 and the z coordinate is ignored */
    int n[3];
    double dx[3];    /* cell size; positions stay in cell units, velocities in physical units */
} orc_box;

typedef struct {
    int kind;        /* ORC_LORENTZ, ORC_DUST, ORC_TRACER */
    double q, m;     /* charge and mass of one unit of weight */
    double t_stop;   /* dust stopping time */
    int rk;          /* tracers: Runge-Kutta stages per step, 2 (Heun) or 3 (SSP, Shu and Osher) */
} orc_species;

typedef struct { const double *E[3], *B[3], *vg[3]; } orc_fields;
typedef struct { double *rho, *J[3], *F[3], *eng; } orc_moments;

/* One-dimensional weights for grid coordinate x of a box of n cells.
 * Returns the number of stencil points (3 for TSC, 2 for CIC) and writes the
 * un-wrapped index of the first stencil cell into *first. */
int orc_weights_1d(int shape, double x, long *first, double w[3]);

/* Field value at grid position x (length 3; x[2] ignored in 2D). */
double orc_gather(const orc_box *b, int shape, const double *f, const double x[3]);

/* Add mu * W(c) / dV to grid g for every stencil cell c of position x. */
void orc_deposit_one(const orc_box *b, int shape, double *g, const double x[3], double mu);

/* Advance np particles of one species by one step of length dt and, when m is
 * not NULL, deposit their moments at the new positions into m (added to what
 * is there).  am, when not NULL, receives the sums of |mu| W per channel, used
 * for round-off tolerances.  fp, when not NULL, receives the per-particle force
 * m w du/dt.  w may be NULL (then every weight is wdef).
 * Returns the number of particles whose displacement reached a full cell in
 * some dimension (a time step beyond the method's stability bound); their
 * update is still carried out. */
long orc_step(const orc_box *b, int shape, double c, const orc_species *sp, long np,
              double *x[3], double *u[3], const double *w, double wdef,
              const orc_fields *f, double dt, orc_moments *m, orc_moments *am, double *fp[3]);

/* Sort key of the particle in cell (i, j, k) for tiles of tile[0..2] cells. */
uint32_t orc_tile_key(const orc_box *b, const int tile[3], int key_mode, long i, long j, long k);

/* Rank-interleaved keys from cells (i, j, k) given per particle: within a tile,
 * particles are ordered first by their rank among earlier particles of the same
 * cell (0 for the first particle of a cell in array order, 1 for the second,
 * ...; ranks above 2^rank_bits - 1 share the last level), then by the cell's
 * place in the tile (x fastest).  key = tile << (rank_bits + cell_bits)
 * | rank << cell_bits | local, cell_bits = bits to number the cells of a tile,
 * rank_bits = min(10, 32 - tile_bits - cell_bits).  Returns rank_bits, or -1
 * when fewer than 3 bits are left for the rank. */
int orc_rank_keys(const orc_box *b, const int tile[3], long np, const long *ci, const long *cj, const long *ck,
                  uint32_t *key);

/* Split grid position x into a cell index and a single-precision offset from
 * the cell centre in [-1/2, 1/2), per dimension (the compact position form). */
void orc_split_position(const orc_box *b, const double x[3], long cell[3], float off[3]);

/* Threads the particle loop uses (OpenMP), for reporting timings. */
int orc_num_threads(void);

/* Set the threads of the particle loops (n > 0), for single-thread timings. */
void orc_set_threads(int n);

/* Stable sort: perm[r] = index of the particle that lands at rank r. */
void orc_stable_sort_perm(long np, const uint32_t *key, long *perm);

/* Parameters of the spectral update: the loss coefficient is
 * c_r = cr * (ub * |B|^2 + u_rad) (Eq. rad_losses, U_B = ub |B|^2). */
typedef struct { double cr, u_rad, ub; } orc_spectra_par;

/* One step dt of the energy distributions of np particles (nb points each,
 * particle-major eng[p*nb+i], chi[p*nb+i]), fluid quantities B, vg and divu
 * (the four-divergence of the fluid velocity) sampled at positions x. */
void orc_spectra_step(const orc_box *b, int shape, double c, long np, double *x[3], const orc_fields *f,
                      const double *divu, int nb, double *eng, double *chi, double dt, const orc_spectra_par *par);

/* 1 when grid position x lies outside the active cells [ghost, n - ghost) of
 * an open dimension (open[d] != 0), else 0. */
int orc_outside(const orc_box *b, const int open[3], int ghost, const double x[3]);

/* Holes-and-fillers compaction of Sec. 3.2 (see orc.c); returns the new count. */
long orc_compact(long np, const unsigned char *flag, int narr, void *const arr[], const size_t esz[],
                 long *hole_out, long *filler_out, long *ncopied);

#ifdef __cplusplus
}
#endif

#endif
