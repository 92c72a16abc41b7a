/*
 * Reference CPU implementation of the per-step particle update.
 * TEST INFRASTRUCTURE ONLY: see orc.h.  Plain loops in the order the method
 * states them; no blocking, fusion or reordering.
 *
 * The paper's particles sample the fluid at their position (Sec. 2, after
 * Eq. 1) and move with it (Eq. 1).  The interpolation kernel, the charged
 * particle pusher, the drag law and the deposit are not spelled out in the
 * paper; they are the textbook definitions named at each function below.
 */
#include "orc.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads the particle loop runs on (for reporting timings). */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads for the particle loops from now on (for single-thread timings). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------ */
/* Grid conventions                                                   */
/* ------------------------------------------------------------------ */

static long wrap_index(long i, long n)
{
    long r = i % n;
    return r < 0 ? r + n : r;
}

/* Periodic wrap of a grid coordinate into [0, n). */
static double wrap_coord(double x, double n)
{
    double y = x - n * floor(x / n);
    if (y >= n) y = 0.0;      /* rounding can land exactly on the upper edge */
    if (y < 0.0) y = 0.0;
    return y;
}

static long flat_index(const orc_box *b, long i, long j, long k)
{
    return wrap_index(i, b->n[0]) + (long)b->n[0] * (wrap_index(j, b->n[1]) + (long)b->n[1] * wrap_index(k, b->n[2]));
}

static double cell_volume(const orc_box *b)
{
    double v = b->dx[0] * b->dx[1];
    if (b->ndim == 3) v *= b->dx[2];
    return v;
}

/* ------------------------------------------------------------------ */
/* Weights                                                            */
/* ------------------------------------------------------------------ */

/*
 * TSC (triangular-shaped cloud; the quadratic B-spline, Hockney & Eastwood
 * 1988, Birdsall & Langdon 1991): with the particle in cell i at offset
 * d = x - i - 1/2 from the cell centre, the weights of cells i-1, i, i+1 are
 * (1/2)(1/2 - d)^2, 3/4 - d^2, (1/2)(1/2 + d)^2.
 *
 * CIC (cloud-in-cell, linear): with b = floor(x - 1/2) and f = x - 1/2 - b,
 * the weights of cells b and b+1 are 1 - f and f.
 */
int orc_weights_1d(int shape, double x, long *first, double w[3])
{
    if (shape == ORC_TSC) {
        double i = floor(x);
        double d = x - i - 0.5;
        *first = (long)i - 1;
        w[0] = 0.5 * (0.5 - d) * (0.5 - d);
        w[1] = 0.75 - d * d;
        w[2] = 0.5 * (0.5 + d) * (0.5 + d);
        return 3;
    }
    double bb = floor(x - 0.5);
    double f = x - 0.5 - bb;
    *first = (long)bb;
    w[0] = 1.0 - f;
    w[1] = f;
    w[2] = 0.0;
    return 2;
}

typedef struct {
    long first[3];
    int cnt[3];
    double w[3][3];
} stencil;

static void make_stencil(const orc_box *b, int shape, const double x[3], stencil *s)
{
    for (int d = 0; d < 3; ++d) {
        if (d < b->ndim) {
            s->cnt[d] = orc_weights_1d(shape, x[d], &s->first[d], s->w[d]);
        } else {
            s->cnt[d] = 1;
            s->first[d] = 0;
            s->w[d][0] = 1.0;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Gather and deposit                                                 */
/* ------------------------------------------------------------------ */

/* F(x) = sum over stencil cells of Wz Wy Wx F[cell], z outermost. */
double orc_gather(const orc_box *b, int shape, const double *f, const double x[3])
{
    stencil s;
    make_stencil(b, shape, x, &s);
    double acc = 0.0;
    for (int k = 0; k < s.cnt[2]; ++k)
        for (int j = 0; j < s.cnt[1]; ++j)
            for (int i = 0; i < s.cnt[0]; ++i) {
                long c = flat_index(b, s.first[0] + i, s.first[1] + j, s.first[2] + k);
                acc += s.w[2][k] * s.w[1][j] * s.w[0][i] * f[c];
            }
    return acc;
}

/* Deposit: the same weights as the gather, amount mu per particle, density
 * per unit cell volume. */
void orc_deposit_one(const orc_box *b, int shape, double *g, const double x[3], double mu)
{
    stencil s;
    make_stencil(b, shape, x, &s);
    double inv_dv = 1.0 / cell_volume(b);
    for (int k = 0; k < s.cnt[2]; ++k)
        for (int j = 0; j < s.cnt[1]; ++j)
            for (int i = 0; i < s.cnt[0]; ++i) {
                long c = flat_index(b, s.first[0] + i, s.first[1] + j, s.first[2] + k);
                g[c] += mu * (s.w[2][k] * s.w[1][j] * s.w[0][i]) * inv_dv;
            }
}

/* ------------------------------------------------------------------ */
/* Pushers                                                            */
/* ------------------------------------------------------------------ */

static void cross(const double a[3], const double b[3], double r[3])
{
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/*
 * Relativistic Boris push (Boris 1970) of du/dt = (q/m)(E + (u/gamma) x B),
 * gamma = sqrt(1 + |u|^2/c^2), with h = (q/m) dt/2:
 *   u-  = u + h E
 *   t   = h B / gamma(u-)
 *   s   = 2 t / (1 + |t|^2)
 *   u'  = u- + u- x t
 *   u+  = u- + u' x s
 *   u   = u+ + h E
 */
static void boris(double u[3], const double E[3], const double B[3], double h, double c)
{
    double um[3], t[3], s[3], up[3], uc[3], tmp[3];
    for (int d = 0; d < 3; ++d) um[d] = u[d] + h * E[d];
    double g = sqrt(1.0 + dot(um, um) / (c * c));
    for (int d = 0; d < 3; ++d) t[d] = h * B[d] / g;
    double tt = dot(t, t);
    for (int d = 0; d < 3; ++d) s[d] = 2.0 * t[d] / (1.0 + tt);
    cross(um, t, tmp);
    for (int d = 0; d < 3; ++d) uc[d] = um[d] + tmp[d];
    cross(uc, s, tmp);
    for (int d = 0; d < 3; ++d) up[d] = um[d] + tmp[d];
    for (int d = 0; d < 3; ++d) u[d] = up[d] + h * E[d];
}

static int moves_a_cell(const orc_box *b, const double v[3], double dt)
{
    for (int d = 0; d < b->ndim; ++d)
        if (fabs(dt * v[d] / b->dx[d]) >= 1.0) return 1;
    return 0;
}

long orc_step(const orc_box *b, int shape, double c, const orc_species *sp, long np,
              double *x[3], double *u[3], const double *w, double wdef,
              const orc_fields *f, double dt, orc_moments *m, orc_moments *am, double *fp[3])
{
    /* per-particle amounts for the deposit, filled by the push loop */
    double *mu = (double *)malloc(sizeof(double) * (size_t)(np > 0 ? np : 1) * 8);
    long violations = 0;
    const double decay = (sp->kind == ORC_DUST) ? exp(-dt / sp->t_stop) : 0.0;

#pragma omp parallel for reduction(+ : violations) schedule(static)
    for (long p = 0; p < np; ++p) {
        double xp[3], un[3], uo[3], v[3];
        double wp = w ? w[p] : wdef;
        for (int d = 0; d < 3; ++d) {
            xp[d] = (d < b->ndim) ? wrap_coord(x[d][p], (double)b->n[d]) : 0.0;
            uo[d] = u[d][p];
            un[d] = uo[d];
        }
        double *mp = mu + 8 * p;
        for (int k = 0; k < 8; ++k) mp[k] = 0.0;

        if (sp->kind == ORC_LORENTZ) {
            double E[3], B[3];
            for (int d = 0; d < 3; ++d) {
                E[d] = orc_gather(b, shape, f->E[d], xp);
                B[d] = orc_gather(b, shape, f->B[d], xp);
            }
            double h = (sp->q / sp->m) * dt * 0.5;
            boris(un, E, B, h, c);
            double gn = sqrt(1.0 + dot(un, un) / (c * c));
            double go = sqrt(1.0 + dot(uo, uo) / (c * c));
            for (int d = 0; d < 3; ++d) v[d] = un[d] / gn;
            violations += moves_a_cell(b, v, dt);
            for (int d = 0; d < b->ndim; ++d)
                xp[d] = wrap_coord(xp[d] + dt * v[d] / b->dx[d], (double)b->n[d]);
            mp[0] = sp->q * wp;                                  /* charge */
            for (int d = 0; d < 3; ++d) mp[1 + d] = sp->q * wp * v[d];              /* current */
            for (int d = 0; d < 3; ++d) mp[4 + d] = sp->m * wp * (un[d] - uo[d]) / dt; /* force */
            mp[7] = sp->m * wp * c * c * (gn - go) / dt;        /* energy change rate */
        } else if (sp->kind == ORC_DUST) {
            /* Exponential (exact for a frozen gas velocity) integrator of
             * dv/dt = -(v - v_g(x)) / t_stop, non-relativistic. */
            double vg[3];
            for (int d = 0; d < 3; ++d) vg[d] = orc_gather(b, shape, f->vg[d], xp);
            for (int d = 0; d < 3; ++d) un[d] = vg[d] + (uo[d] - vg[d]) * decay;
            violations += moves_a_cell(b, un, dt);
            for (int d = 0; d < b->ndim; ++d)
                xp[d] = wrap_coord(xp[d] + dt * un[d] / b->dx[d], (double)b->n[d]);
            mp[0] = sp->m * wp;                                  /* dust mass */
            for (int d = 0; d < 3; ++d) mp[4 + d] = sp->m * wp * (un[d] - uo[d]) / dt;
        } else if (sp->rk == 3) {
            /* Passive tracer, Eq. 1 (dx/dt = v(x)), the three-stage
             * strong-stability-preserving Runge-Kutta scheme of Shu and Osher
             * with the gas velocity frozen over the step:
             *   x1 = x + dt v(x)
             *   x2 = 3/4 x + 1/4 (x1 + dt v(x1))
             *   x3 = 1/3 x + 2/3 (x2 + dt v(x2))
             * written as x3 = x + dt (k1 + k2 + 4 k3)/6 with k1 = v(x),
             * k2 = v(x + dt k1), k3 = v(x + dt (k1 + k2)/4). */
            double k1[3], k2[3], k3[3], xs[3], h[3];
            for (int d = 0; d < 3; ++d) k1[d] = orc_gather(b, shape, f->vg[d], xp);
            for (int d = 0; d < 3; ++d)
                xs[d] = (d < b->ndim) ? wrap_coord(xp[d] + dt * k1[d] / b->dx[d], (double)b->n[d]) : 0.0;
            for (int d = 0; d < 3; ++d) k2[d] = orc_gather(b, shape, f->vg[d], xs);
            for (int d = 0; d < 3; ++d) h[d] = 0.25 * (k1[d] + k2[d]);
            for (int d = 0; d < 3; ++d)
                xs[d] = (d < b->ndim) ? wrap_coord(xp[d] + dt * h[d] / b->dx[d], (double)b->n[d]) : 0.0;
            for (int d = 0; d < 3; ++d) k3[d] = orc_gather(b, shape, f->vg[d], xs);
            for (int d = 0; d < 3; ++d) un[d] = (k1[d] + k2[d] + 4.0 * k3[d]) / 6.0;
            violations += moves_a_cell(b, k1, dt) | moves_a_cell(b, un, dt);
            for (int d = 0; d < b->ndim; ++d)
                xp[d] = wrap_coord(xp[d] + dt * un[d] / b->dx[d], (double)b->n[d]);
        } else {
            /* Passive tracer, Eq. 1 (dx/dt = v(x)), two-stage Runge-Kutta
             * (Heun) with the gas velocity frozen over the step. */
            double k1[3], k2[3], xs[3];
            for (int d = 0; d < 3; ++d) k1[d] = orc_gather(b, shape, f->vg[d], xp);
            for (int d = 0; d < 3; ++d)
                xs[d] = (d < b->ndim) ? wrap_coord(xp[d] + dt * k1[d] / b->dx[d], (double)b->n[d]) : 0.0;
            for (int d = 0; d < 3; ++d) k2[d] = orc_gather(b, shape, f->vg[d], xs);
            for (int d = 0; d < 3; ++d) un[d] = 0.5 * (k1[d] + k2[d]);
            violations += moves_a_cell(b, k1, dt) | moves_a_cell(b, un, dt);
            for (int d = 0; d < b->ndim; ++d)
                xp[d] = wrap_coord(xp[d] + dt * un[d] / b->dx[d], (double)b->n[d]);
        }

        for (int d = 0; d < 3; ++d) {
            if (d < b->ndim) x[d][p] = xp[d];
            u[d][p] = un[d];
        }
        if (fp)
            for (int d = 0; d < 3; ++d) fp[d][p] = mp[4 + d];
    }

    /* Deposit at the new positions, particle by particle in index order. */
    if (m) {
        for (long p = 0; p < np; ++p) {
            double xp[3] = {x[0][p], x[1][p], b->ndim == 3 ? x[2][p] : 0.0};
            const double *mp = mu + 8 * p;
            double *g[8] = {m->rho, m->J[0], m->J[1], m->J[2], m->F[0], m->F[1], m->F[2], m->eng};
            double *a[8] = {0};
            if (am) {
                a[0] = am->rho; a[1] = am->J[0]; a[2] = am->J[1]; a[3] = am->J[2];
                a[4] = am->F[0]; a[5] = am->F[1]; a[6] = am->F[2]; a[7] = am->eng;
            }
            for (int ch = 0; ch < 8; ++ch) {
                if (g[ch]) orc_deposit_one(b, shape, g[ch], xp, mp[ch]);
                if (a[ch]) orc_deposit_one(b, shape, a[ch], xp, fabs(mp[ch]));
            }
        }
    }
    free(mu);
    return violations;
}

/* ------------------------------------------------------------------ */
/* Cell-tile sort                                                     */
/* ------------------------------------------------------------------ */

/*
 * Tiles of tile[0] x tile[1] x tile[2] cells, numbered x fastest.  Key mode
 * "tile" sorts by tile only; "tile+cell" by tile, then by the cell's place in
 * the tile (x fastest).
 */
uint32_t orc_tile_key(const orc_box *b, const int tile[3], int key_mode, long i, long j, long k)
{
    long ntx = b->n[0] / tile[0], nty = b->n[1] / tile[1];
    long t = i / tile[0] + ntx * (j / tile[1] + nty * (k / tile[2]));
    if (key_mode == ORC_KEY_TILE) return (uint32_t)t;
    long local = i % tile[0] + (long)tile[0] * (j % tile[1] + (long)tile[1] * (k % tile[2]));
    return (uint32_t)(t * (long)tile[0] * tile[1] * tile[2] + local);
}

static int bits_for(long count)
{
    int b = 0;
    while ((1L << b) < count) ++b;
    return b;
}

int orc_rank_keys(const orc_box *b, const int tile[3], long np, const long *ci, const long *cj, const long *ck,
                  uint32_t *key)
{
    long ntiles = (long)(b->n[0] / tile[0]) * (b->n[1] / tile[1]) * (b->n[2] / tile[2]);
    long per_tile = (long)tile[0] * tile[1] * tile[2];
    int tb = bits_for(ntiles), cb = bits_for(per_tile);
    int rb = 32 - tb - cb;
    if (rb > 10) rb = 10;
    if (rb < 3) return -1;
    long ncells = (long)b->n[0] * b->n[1] * b->n[2];
    long *seen = (long *)calloc((size_t)ncells, sizeof(long));
    long rmax = (1L << rb) - 1;
    for (long p = 0; p < np; ++p) {
        long c = ci[p] + (long)b->n[0] * (cj[p] + (long)b->n[1] * ck[p]);
        long rank = seen[c]++;
        if (rank > rmax) rank = rmax;
        uint32_t tk = orc_tile_key(b, tile, ORC_KEY_TILE, ci[p], cj[p], ck[p]);
        uint32_t full = orc_tile_key(b, tile, ORC_KEY_TILE_CELL, ci[p], cj[p], ck[p]);
        uint32_t local = full - tk * (uint32_t)per_tile;
        key[p] = (tk << (rb + cb)) | ((uint32_t)rank << cb) | local;
    }
    free(seen);
    return rb;
}

/*
 * Compact position: cell index plus the single-precision offset from the cell
 * centre.  If the offset rounds up to +1/2 the particle belongs to the next
 * cell at offset -1/2 (cells are half-open).
 */
void orc_split_position(const orc_box *b, const double x[3], long cell[3], float off[3])
{
    for (int d = 0; d < 3; ++d) {
        if (d >= b->ndim) { cell[d] = 0; off[d] = 0.0f; continue; }
        double y = wrap_coord(x[d], (double)b->n[d]);
        double i = floor(y);
        float o = (float)(y - i - 0.5);
        long ci = (long)i;
        if (o >= 0.5f) { o = -0.5f; ci = wrap_index(ci + 1, b->n[d]); }
        cell[d] = ci;
        off[d] = o;
    }
}

typedef struct { uint32_t key; long idx; } key_idx;

static int cmp_key_idx(const void *a, const void *b)
{
    const key_idx *p = (const key_idx *)a, *q = (const key_idx *)b;
    if (p->key != q->key) return p->key < q->key ? -1 : 1;
    if (p->idx != q->idx) return p->idx < q->idx ? -1 : 1;
    return 0;
}

/* Stable sort by key: ordering by (key, original index) is exactly the
 * stable order. */
void orc_stable_sort_perm(long np, const uint32_t *key, long *perm)
{
    key_idx *t = (key_idx *)malloc(sizeof(key_idx) * (size_t)(np > 0 ? np : 1));
    for (long p = 0; p < np; ++p) { t[p].key = key[p]; t[p].idx = p; }
    qsort(t, (size_t)np, sizeof(key_idx), cmp_key_idx);
    for (long p = 0; p < np; ++p) perm[p] = t[p].idx;
    free(t);
}

/* ------------------------------------------------------------------ */
/* Lagrangian spectral update (Sec. 2)                                 */
/* ------------------------------------------------------------------ */

/*
 * Each particle carries its energy distribution as nb points (eps_i, chi_i),
 * chi = N / n the number density per unit energy relative to the fluid's
 * (Eq. chi).  Away from shocks chi obeys Eq. cr_chi: it is carried in energy
 * with the rate
 *     d eps / d tau = -(eps / 3) div_mu u^mu - c_r eps^2          (Eq. cr_N)
 * (adiabatic term, and synchrotron plus inverse-Compton losses with
 * c_r = cr (U_B + U_rad), Eq. rad_losses; U_B = ub |B|^2), while
 * d chi / d tau = -chi d(d eps/d tau)/d eps along each characteristic.
 * Proper and laboratory time: d tau = dt / gamma_g (Sec. 2).
 *
 * With the fluid quantities frozen over the step (a = div u / 3, b = c_r)
 * both are solved exactly:
 *     eps(tau) = a eps0 e^{-a tau} / (a + b eps0 (1 - e^{-a tau})),
 * i.e. eps = eps0 E / den with E = e^{-a tau}, den = 1 + b eps0 phi,
 * phi = (1 - e^{-a tau}) / a (-> tau as a -> 0), and since
 * d eps / d eps0 = E / den^2 and chi d eps is conserved on a characteristic,
 *     chi(tau) = chi0 den^2 / E.
 * Each point of the spectrum moves on its own characteristic (a Lagrangian
 * grid in energy), so the number between two neighbouring points is
 * conserved.  The fluid quantities are sampled at the particle position with
 * the same CIC/TSC weights as orc_gather.  Arrays are particle-major:
 * eng[p * nb + i], chi[p * nb + i].
 */
void orc_spectra_step(const orc_box *b, int shape, double c, long np, double *x[3], const orc_fields *f,
                      const double *divu, int nb, double *eng, double *chi, double dt, const orc_spectra_par *par)
{
#pragma omp parallel for schedule(static)
    for (long p = 0; p < np; ++p) {
        double xp[3] = {x[0][p], x[1][p], b->ndim == 3 ? x[2][p] : 0.0};
        double Bp[3], vp[3];
        for (int d = 0; d < 3; ++d) {
            Bp[d] = orc_gather(b, shape, f->B[d], xp);
            vp[d] = orc_gather(b, shape, f->vg[d], xp);
        }
        double dv = orc_gather(b, shape, divu, xp);
        double gamma_g = 1.0 / sqrt(1.0 - dot(vp, vp) / (c * c));
        double dtau = dt / gamma_g;
        double a = dv / 3.0;
        double bb = par->cr * (par->ub * dot(Bp, Bp) + par->u_rad);
        double E = exp(-a * dtau);
        double phi = a != 0.0 ? -expm1(-a * dtau) / a : dtau;
        for (int i = 0; i < nb; ++i) {
            double eps0 = eng[p * nb + i];
            double den = 1.0 + bb * eps0 * phi;
            eng[p * nb + i] = eps0 * E / den;
            chi[p * nb + i] = chi[p * nb + i] * den * den / E;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Open boundaries: deletion and compaction (Sec. 3.2)                 */
/* ------------------------------------------------------------------ */

/*
 * A particle leaves through an open dimension d when its cell lies outside
 * the active cells [ghost, n_d - ghost): the grid keeps `ghost` layers of
 * boundary cells on each open side, so the stencils of the particles that
 * were active at the start of a step stay inside the grid arrays.
 */
int orc_outside(const orc_box *b, const int open[3], int ghost, const double x[3])
{
    for (int d = 0; d < b->ndim; ++d) {
        if (!open[d]) continue;
        double cell = floor(x[d]);
        if (cell < (double)ghost || cell >= (double)(b->n[d] - ghost)) return 1;
    }
    return 0;
}

/*
 * The compaction of Sec. 3.2, step by step:
 *   1. count the ndel flagged particles (the holes to be);
 *   2. save the indices of the flagged particles in a temporary array;
 *   3. collect the fillers: unflagged particles stored at i >= np - ndel;
 *   4. copy every array of the k-th filler into the k-th saved hole below
 *      np - ndel (both lists in increasing index order);
 *   5. shrink to np - ndel.
 * Arrays: narr arrays of np elements of esz[k] bytes each, moved together.
 * Returns the new count; hole_out / filler_out (nullable, np entries) receive
 * the pairs actually copied, and *ncopied their number.
 */
long orc_compact(long np, const unsigned char *flag, int narr, void *const arr[], const size_t esz[],
                 long *hole_out, long *filler_out, long *ncopied)
{
    long ndel = 0;
    for (long p = 0; p < np; ++p) ndel += flag[p] != 0;                 /* 1 */
    long *tmp = (long *)malloc(sizeof(long) * (size_t)(np > 0 ? np : 1));
    long nsaved = 0;
    for (long p = 0; p < np; ++p)                                       /* 2 */
        if (flag[p]) tmp[nsaved++] = p;
    long keep = np - ndel;
    long *fill = (long *)malloc(sizeof(long) * (size_t)(ndel > 0 ? ndel : 1));
    long nfill = 0;
    if (nsaved > 0)                                                     /* 3 */
        for (long p = keep; p < np; ++p)
            if (!flag[p]) fill[nfill++] = p;
    long k = 0;
    for (long h = 0; h < nsaved && tmp[h] < keep; ++h, ++k) {           /* 4 */
        for (int a = 0; a < narr; ++a) {
            unsigned char *base = (unsigned char *)arr[a];
            memcpy(base + (size_t)tmp[h] * esz[a], base + (size_t)fill[k] * esz[a], esz[a]);
        }
        if (hole_out) hole_out[k] = tmp[h];
        if (filler_out) filler_out[k] = fill[k];
    }
    if (ncopied) *ncopied = k;
    free(fill);
    free(tmp);
    return keep;                                                        /* 5 */
}
