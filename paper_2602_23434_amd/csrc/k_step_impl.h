// Gather -> push -> deposit kernels for gfx950 (template; instantiated per
// precision in k_step_f32.hip and k_step_f64.hip).
//
// One templated body serves both algorithms:
//  * PLAIN: one thread per particle; fields are read from HBM/L2 at the 27
//    (TSC) stencil cells and every deposit is a float64 global atomic.
//  * TILED: one work unit per (item, cell tile).  The block stages the tile's
//    fields plus a one-cell halo into LDS (converted to the arithmetic type),
//    processes the particles the last cell-tile sort assigned to the tile,
//    accumulates their deposits in an LDS tile, and flushes it with one
//    float64 global atomic per touched cell and channel.  A particle whose
//    stencil leaves the LDS tile (it drifted since the sort) takes the plain
//    route for that gather or deposit, so results never depend on the sort.
// Work units of all items of a call are claimed from one atomic counter by a
// persistent grid sized to the chip's resident capacity; items are ordered
// largest first on the host.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <vector>

#include "pl_device.h"

namespace pl {

template <int DIM> struct Stencil {
    static constexpr int SY = DIM >= 2 ? 3 : 1;
    static constexpr int SZ = DIM >= 3 ? 3 : 1;
};

// Work-unit claim shared by every persistent kernel: returns a wave-uniform
// unit index, or -1 when the work is exhausted.
__device__ __forceinline__ int claim_unit(unsigned *counter, int total, int *s_slot)
{
    __syncthreads();
    if (threadIdx.x == 0) *s_slot = (int)atomicAdd(counter, 1u);
    __syncthreads();
    int g = __builtin_amdgcn_readfirstlane(*s_slot);
    return g < total ? g : -1;
}

// The last block to finish resets the counter pair for the next launch.
__device__ __forceinline__ void release_counter(unsigned *counter)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        unsigned done = atomicAdd(counter + 1, 1u);
        if (done == gridDim.x - 1) {
            atomicExch(counter, 0u);
            atomicExch(counter + 1, 0u);
        }
    }
}

__device__ __forceinline__ int find_item(const ItemDesc *items, int nitems, int g)
{
    int it = 0;
    while (it + 1 < nitems && items[it + 1].unit_begin <= g) ++it;
    return it;
}

// Per-unit constants: read once from the item table into registers when a
// block claims a unit, so the particle loop never goes back to memory (or
// waits on the scalar cache) for them.
template <int PREC> struct UnitC {
    using R = typename RealOf<PREC>::T;
    int n[3];
    int np, kind, rk;
    R h, inv_c2, c2, q, m, wdef, inv_dt, decay, one_m_decay;
    R dtdx[3];
    double inv_dv;
    gptr<uint32_t> cell;
    gptr<R> x[3];
    gptr<R> u[3];
    gptr<const R> w;
    gptr<R> fp[3];
    gptr<const double> gf[6];
    gptr<double> M[kMaxCh];
    int soff[kMaxCh];      // offset of each active channel in the LDS deposit tile, -1 if inactive
};

template <int PREC>
__device__ __forceinline__ void load_unit(const ItemDesc &I, UnitC<PREC> &U, int L)
{
    using R = typename RealOf<PREC>::T;
    for (int a = 0; a < 3; ++a) {
        U.n[a] = I.n[a];
        U.dtdx[a] = (R)I.dtdx[a];
        U.x[a] = (gptr<R>)I.x[a];
        U.u[a] = (gptr<R>)I.u[a];
        U.fp[a] = (gptr<R>)I.fp[a];
    }
    U.np = I.np;
    U.kind = I.kind;
    U.rk = I.rk;
    U.h = (R)I.h;
    U.inv_c2 = (R)I.inv_c2;
    U.c2 = (R)I.c2;
    U.q = (R)I.q;
    U.m = (R)I.m;
    U.wdef = (R)I.wdef;
    U.inv_dt = (R)I.inv_dt;
    U.decay = (R)I.decay;
    U.one_m_decay = (R)I.one_m_decay;
    U.inv_dv = I.inv_dv;
    U.cell = (gptr<uint32_t>)I.cell;
    U.w = (gptr<const R>)I.w;
    if (I.kind == PL_LORENTZ) {
        for (int a = 0; a < 3; ++a) {
            U.gf[a] = (gptr<const double>)I.E[a];
            U.gf[3 + a] = (gptr<const double>)I.B[a];
        }
    } else {
        for (int a = 0; a < 3; ++a) {
            U.gf[a] = (gptr<const double>)I.vg[a];
            U.gf[3 + a] = nullptr;
        }
    }
    for (int ch = 0; ch < kMaxCh; ++ch) {
        U.M[ch] = (gptr<double>)I.M[ch];
        U.soff[ch] = I.slot[ch] >= 0 ? I.slot[ch] * L : -1;
    }
}

// Compile-time channel -> LDS slot maps for the common channel sets (CHS):
// 0 runtime (UnitC::soff), 1 charged rho, J, F (slots 0..6), 2 dust rho, F
// (slots 0..3).
__host__ __device__ constexpr int chs_slot(int CHS, int ch)
{
    return CHS == 1 ? (ch < 7 ? ch : -1) : CHS == 2 ? (ch == 0 ? 0 : (ch >= 4 && ch <= 6 ? ch - 3 : -1)) : -1;
}

// Compile-time tile shapes (TS): 0 runtime, 1 = 8x8x8, 2 = 8x8x4.
__host__ __device__ constexpr int ts_dim(int TS, int a) { return TS == 1 ? 8 : TS == 2 ? (a < 2 ? 8 : 4) : 0; }

// Tile geometry of one work unit in the LDS (one-cell halo on every side).
struct TileGeo {
    int lo[3];
    int T[3];
    int Lx, LxLy, L;
};

template <int DIM>
__device__ __forceinline__ bool in_tile(const TileGeo &tg, const int c[3], int &base)
{
    int l0 = c[0] - tg.lo[0], l1 = DIM >= 2 ? c[1] - tg.lo[1] : 0, l2 = DIM >= 3 ? c[2] - tg.lo[2] : 0;
    bool ok = (unsigned)l0 < (unsigned)tg.T[0];
    if (DIM >= 2) ok = ok && (unsigned)l1 < (unsigned)tg.T[1];
    if (DIM >= 3) ok = ok && (unsigned)l2 < (unsigned)tg.T[2];
    // LDS cell index of stencil offset (-1,-1,-1) relative to the particle's cell
    base = l0 + (DIM >= 2 ? l1 * tg.Lx : 0) + (DIM >= 3 ? l2 * tg.LxLy : 0);
    return ok;
}

// Interpolate NC field components at a particle in cell c with 1D weights
// wx, wy, wz: from the LDS tile (component-major, L cells per component) when
// the stencil lies inside it, otherwise from the float64 grids in HBM.  Both
// routes add the same terms in the same order with explicit fused
// multiply-adds, so the result does not depend on the route.
template <int PREC, int DIM, int NC>
__device__ __forceinline__ void gather(const UnitC<PREC> &U, const typename RealOf<PREC>::T *lds_f, int L, bool use_lds,
                                       int base, int Lx, int LxLy, const int c[3],
                                       const typename RealOf<PREC>::T wx[3], const typename RealOf<PREC>::T wy[3],
                                       const typename RealOf<PREC>::T wz[3], typename RealOf<PREC>::T out[NC])
{
    using R = typename RealOf<PREC>::T;
    constexpr int SY = Stencil<DIM>::SY, SZ = Stencil<DIM>::SZ;
#pragma unroll
    for (int q = 0; q < NC; ++q) out[q] = R(0);
    if (use_lds) {
#pragma unroll
        for (int k = 0; k < SZ; ++k)
#pragma unroll
            for (int j = 0; j < SY; ++j) {
                R wyz = wz[k] * wy[j];
                int row = base + k * LxLy + j * Lx;
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    R w = wyz * wx[i];
#pragma unroll
                    for (int q = 0; q < NC; ++q) out[q] = fma(w, lds_f[q * L + row + i], out[q]);
                }
            }
    } else {
        const int *n = U.n;
        int ix[3] = {wrap_cell(c[0] - 1, n[0]), c[0], wrap_cell(c[0] + 1, n[0])};
        int iy[3] = {wrap_cell(c[1] - 1, n[1]), c[1], wrap_cell(c[1] + 1, n[1])};
        int iz[3] = {DIM >= 3 ? wrap_cell(c[2] - 1, n[2]) : c[2], c[2], DIM >= 3 ? wrap_cell(c[2] + 1, n[2]) : c[2]};
#pragma unroll
        for (int k = 0; k < SZ; ++k)
#pragma unroll
            for (int j = 0; j < SY; ++j) {
                R wyz = wz[k] * wy[j];
                long row = (long)n[0] * (iy[j] + (long)n[1] * iz[k]);
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    R w = wyz * wx[i];
                    long g = row + ix[i];
#pragma unroll
                    for (int q = 0; q < NC; ++q) out[q] = fma(w, (R)U.gf[q][g], out[q]);
                }
            }
    }
}

// Deposit mu[ch] * W into the float64 LDS tile (or straight into the grids
// when the stencil leaves the tile).  LDS float64 adds are used because on
// gfx950 they run about ten times faster than float32 LDS atomic adds.
template <int PREC, int DIM, int CHS>
__device__ __forceinline__ void deposit(const UnitC<PREC> &U, double *lds_d, bool use_lds, int base, int Lx,
                                        int LxLy, int L, const int c[3], const typename RealOf<PREC>::T wx[3],
                                        const typename RealOf<PREC>::T wy[3], const typename RealOf<PREC>::T wz[3],
                                        const double mu[kMaxCh])
{
    using R = typename RealOf<PREC>::T;
    constexpr int SY = Stencil<DIM>::SY, SZ = Stencil<DIM>::SZ;
    if (use_lds) {
#pragma unroll
        for (int k = 0; k < SZ; ++k)
#pragma unroll
            for (int j = 0; j < SY; ++j) {
                R wyz = wz[k] * wy[j];
                int row = base + k * LxLy + j * Lx;
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    double w = (double)(wyz * wx[i]);
#pragma unroll
                    for (int ch = 0; ch < kMaxCh; ++ch) {
                        if constexpr (CHS != 0) {
                            const int sl = chs_slot(CHS, ch);
                            if (sl >= 0)
                                __hip_atomic_fetch_add(lds_d + sl * L + row + i, w * mu[ch], __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                        } else {
                            int so = U.soff[ch];
                            if (so >= 0)
                                __hip_atomic_fetch_add(lds_d + so + row + i, w * mu[ch], __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                        }
                    }
                }
            }
    } else {
        const int *n = U.n;
        int ix[3] = {wrap_cell(c[0] - 1, n[0]), c[0], wrap_cell(c[0] + 1, n[0])};
        int iy[3] = {wrap_cell(c[1] - 1, n[1]), c[1], wrap_cell(c[1] + 1, n[1])};
        int iz[3] = {DIM >= 3 ? wrap_cell(c[2] - 1, n[2]) : c[2], c[2], DIM >= 3 ? wrap_cell(c[2] + 1, n[2]) : c[2]};
#pragma unroll
        for (int k = 0; k < SZ; ++k)
#pragma unroll
            for (int j = 0; j < SY; ++j) {
                R wyz = wz[k] * wy[j];
                long row = (long)n[0] * (iy[j] + (long)n[1] * iz[k]);
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    double w = (double)(wyz * wx[i]) * U.inv_dv;
                    long g = row + ix[i];
#pragma unroll
                    for (int ch = 0; ch < kMaxCh; ++ch) {
                        bool on = CHS != 0 ? chs_slot(CHS, ch) >= 0 : U.soff[ch] >= 0;
                        if (on) global_add(U.M[ch] + g, w * mu[ch]);
                    }
                }
            }
    }
}

template <int PREC, int SHAPE, int DIM>
__device__ __forceinline__ void stencil_weights(const typename RealOf<PREC>::T d[3], typename RealOf<PREC>::T wx[3],
                                                typename RealOf<PREC>::T wy[3], typename RealOf<PREC>::T wz[3])
{
    using R = typename RealOf<PREC>::T;
    weights3<SHAPE>(d[0], wx);
    weights3<SHAPE>(d[1], wy);
    if (DIM >= 3) {
        weights3<SHAPE>(d[2], wz);
    } else {
        wz[0] = R(1); wz[1] = R(0); wz[2] = R(0);
    }
}

// LDS bytes of one work unit: field tile (when pushing) + float64 deposit tile
// + a 16-byte tail holding the claimed unit index.
__host__ __device__ inline size_t step_lds_bytes(int prec, int kind, int L, bool push, int nslot)
{
    size_t rs = prec == PL_F64 ? 8 : 4;
    int nf = kind == PL_LORENTZ ? 6 : 3;
    size_t f = push ? (size_t)L * nf * rs : 0;
    f = (f + 15) & ~(size_t)15;
    return f + (size_t)L * nslot * 8 + 16;
}

template <int PREC, int SHAPE, int DIM, bool TILED, int KIND, int TS, int CHS>
__global__ __launch_bounds__(512, (TILED && PREC == PL_F32_OFFSET && KIND != PL_TRACER) ? 4 : 1) void k_step(const ItemDesc *__restrict__ items, int nitems, int total_units,
                                               unsigned *counter, int *errflags, unsigned flags, int lds_bytes)
{
    using R = typename RealOf<PREC>::T;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    int *s_unit = reinterpret_cast<int *>(smem_raw + lds_bytes - 16);

    const bool do_push = flags & SF_PUSH;
    const bool do_dep = flags & SF_DEPOSIT;
    const bool do_sums = flags & SF_SUMS;
    int err = 0;

    for (;;) {
        int g = claim_unit(counter, total_units, s_unit);
        if (g < 0) break;
        const int iti = find_item(items, nitems, g);
        const ItemDesc &I = items[iti];
        const int unit = g - I.unit_begin;
        TileGeo tg;
        int pbeg, pend;
        if (TILED) {
            int t = unit;
            int tx = t % I.ntile[0];
            int ty = (t / I.ntile[0]) % I.ntile[1];
            int tz = t / (I.ntile[0] * I.ntile[1]);
            tg.T[0] = TS ? ts_dim(TS, 0) : I.tile[0];
            tg.T[1] = TS ? ts_dim(TS, 1) : I.tile[1];
            tg.T[2] = TS ? ts_dim(TS, 2) : I.tile[2];
            tg.lo[0] = tx * tg.T[0];
            tg.lo[1] = ty * tg.T[1];
            tg.lo[2] = tz * tg.T[2];
            tg.Lx = tg.T[0] + 2;
            tg.LxLy = tg.Lx * (tg.T[1] + 2);
            tg.L = tg.LxLy * (DIM >= 3 ? tg.T[2] + 2 : 1);
            // tile offsets must run from 0 to np: otherwise the item was never
            // sorted (or its count changed since): latch it, leave it alone
            if (I.tile_start[0] != 0 || I.tile_start[I.ntiles] != I.np) {
                if (threadIdx.x == 0) atomicOr(errflags, (int)ERR_UNSORTED);
                continue;                  // uniform
            }
            int a = I.tile_start[t], b = I.tile_start[t + 1];
            pbeg = min(max(a, 0), I.np);
            pend = min(max(b, pbeg), I.np);
        } else {
            tg.Lx = tg.LxLy = tg.L = 0;
            tg.lo[0] = tg.lo[1] = tg.lo[2] = 0;
            tg.T[0] = tg.T[1] = tg.T[2] = 0;
            pbeg = unit * I.chunk;
            pend = min(I.np, pbeg + I.chunk);
        }
        if (pbeg >= pend) continue;        // uniform: the whole block skips an empty unit

        UnitC<PREC> U;
        load_unit<PREC>(I, U, tg.L);
        constexpr int kind = KIND;
        const bool dep_here = KIND != PL_TRACER && do_dep && I.nslot > 0;
        const int nslot = I.nslot;
        constexpr int nf = KIND == PL_LORENTZ ? 6 : 3;
        R *lds_f = reinterpret_cast<R *>(smem_raw);
        size_t foff = do_push ? ((size_t)tg.L * nf * sizeof(R) + 15) & ~(size_t)15 : 0;
        double *lds_d = reinterpret_cast<double *>(smem_raw + foff);

        if (TILED) {
            const int Ly = tg.T[1] + 2;
            for (int e = threadIdx.x; e < tg.L; e += blockDim.x) {
                int lx = e % tg.Lx;
                int ly = (e / tg.Lx) % Ly;
                int lz = e / tg.LxLy;
                int gx = wrap_cell(tg.lo[0] + lx - 1, U.n[0]);
                int gy = wrap_cell(tg.lo[1] + ly - 1, U.n[1]);
                int gz = DIM >= 3 ? wrap_cell(tg.lo[2] + lz - 1, U.n[2]) : 0;
                long gc = gx + (long)U.n[0] * (gy + (long)U.n[1] * gz);
                if (do_push)
                    for (int q = 0; q < nf; ++q) lds_f[q * tg.L + e] = (R)U.gf[q][gc];
                if (dep_here)
                    for (int s = 0; s < nslot; ++s) lds_d[s * tg.L + e] = 0.0;
            }
            __syncthreads();
        }

        double ps[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) ps[k] = 0.0;

        // Default: consecutive lanes take consecutive particles (coalesced
        // loads and stores; with particles sorted by cell, lanes of one cell
        // read the same LDS words, which the LDS broadcasts).  With SF_RUNS
        // thread t takes the contiguous run [pbeg + t*run, +run) instead, so
        // the lanes of a wave sit in about 64 distinct consecutive cells.
        const bool runs = TILED && (flags & SF_RUNS);
        const int run = runs ? (pend - pbeg + (int)blockDim.x - 1) / (int)blockDim.x : 1;
        const int pfirst = runs ? pbeg + (int)threadIdx.x * run : pbeg + (int)threadIdx.x;
        const int plast = runs ? min(pend, pfirst + run) : pend;
        const int pstep = runs ? 1 : (int)blockDim.x;
        for (int p = pfirst; p < plast; p += pstep) {
            Pos<PREC, DIM> pos;
            pos.load(U, p, err);
            R u[3] = {U.u[0][p], U.u[1][p], U.u[2][p]};
            R w = U.w ? U.w[p] : U.wdef;
            double mu[kMaxCh];
#pragma unroll
            for (int ch = 0; ch < kMaxCh; ++ch) mu[ch] = 0.0;

            if (do_push) {
                R d0[3] = {(R)pos.d[0], (R)pos.d[1], (R)pos.d[2]};
                R wx[3], wy[3], wz[3];
                stencil_weights<PREC, SHAPE, DIM>(d0, wx, wy, wz);
                int base = 0;
                bool inl = TILED && in_tile<DIM>(tg, pos.c, base);
                R v[3];
                if constexpr (KIND == PL_LORENTZ) {
                    R EB[6];
                    gather<PREC, DIM, 6>(U, lds_f, tg.L, inl, base, tg.Lx, tg.LxLy, pos.c, wx, wy, wz, EB);
                    R du[3];
                    R uo[3] = {u[0], u[1], u[2]};
                    R u_old2 = fma(u[0], u[0], fma(u[1], u[1], u[2] * u[2]));
                    boris<R>(u, EB, EB + 3, U.h, U.inv_c2, du);
                    R u_new2 = fma(u[0], u[0], fma(u[1], u[1], u[2] * u[2]));
                    const R gn2 = fma(u_new2, U.inv_c2, R(1));
                    R gn = sqrt(gn2);
                    R go = sqrt(fma(u_old2, U.inv_c2, R(1)));
                    R ig = div_sqrt_ge1(R(1), gn2);
#pragma unroll
                    for (int a = 0; a < 3; ++a) v[a] = u[a] * ig;
                    R qw = U.q * w, mw = U.m * w;
                    mu[0] = (double)qw;
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        mu[1 + a] = (double)(qw * v[a]);
                        mu[4 + a] = (double)(mw * du[a] * U.inv_dt);
                    }
                    if constexpr (PREC == PL_F64) {
                        mu[7] = (double)(mw * U.c2 * (gn - go) * U.inv_dt);
                    } else {
                        // c^2 (gamma_new - gamma_old) without the cancellation:
                        // (|u_new|^2 - |u_old|^2) / (gamma_new + gamma_old)
                        R dd = fma(du[0], u[0] + uo[0], fma(du[1], u[1] + uo[1], du[2] * (u[2] + uo[2])));
                        mu[7] = (double)(mw * dd / (gn + go) * U.inv_dt);
                    }
                    if (U.fp[0]) {
#pragma unroll
                        for (int a = 0; a < 3; ++a) U.fp[a][p] = (R)mu[4 + a];
                    }
                } else if constexpr (KIND == PL_DUST) {
                    R vg[3];
                    gather<PREC, DIM, 3>(U, lds_f, tg.L, inl, base, tg.Lx, tg.LxLy, pos.c, wx, wy, wz, vg);
                    R du[3];
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        du[a] = (vg[a] - u[a]) * U.one_m_decay;
                        u[a] = vg[a] + (u[a] - vg[a]) * U.decay;
                        v[a] = u[a];
                    }
                    R mw = U.m * w;
                    mu[0] = (double)mw;
#pragma unroll
                    for (int a = 0; a < 3; ++a) mu[4 + a] = (double)(mw * du[a] * U.inv_dt);
                    if (U.fp[0]) {
#pragma unroll
                        for (int a = 0; a < 3; ++a) U.fp[a][p] = (R)mu[4 + a];
                    }
                } else {
                    // tracer on the frozen gas velocity: Heun's two-stage
                    // Runge-Kutta, or the three-stage SSP scheme of Shu and
                    // Osher, x + dt (k1 + k2 + 4 k3) / 6 with k1 = v(x),
                    // k2 = v(x + dt k1), k3 = v(x + dt (k1 + k2) / 4)
                    R k1[3], k2[3];
                    gather<PREC, DIM, 3>(U, lds_f, tg.L, inl, base, tg.Lx, tg.LxLy, pos.c, wx, wy, wz, k1);
                    // velocity of the stage after k, at x + dt * s (s in cells per unit time)
                    auto stage = [&](const R s[3], R k[3]) {
                        Pos<PREC, DIM> mid = pos;
                        R dd[3] = {R(0), R(0), R(0)};
#pragma unroll
                        for (int a = 0; a < DIM; ++a) dd[a] = s[a] * U.dtdx[a];
                        mid.advance(dd, U, err);
                        R dm[3] = {(R)mid.d[0], (R)mid.d[1], (R)mid.d[2]};
                        R sx[3], sy[3], sz[3];
                        stencil_weights<PREC, SHAPE, DIM>(dm, sx, sy, sz);
                        int base2 = 0;
                        bool inl2 = TILED && in_tile<DIM>(tg, mid.c, base2);
                        gather<PREC, DIM, 3>(U, lds_f, tg.L, inl2, base2, tg.Lx, tg.LxLy, mid.c, sx, sy, sz, k);
                    };
                    stage(k1, k2);
                    if (U.rk == 3) {
                        R hq[3], k3[3];
#pragma unroll
                        for (int a = 0; a < 3; ++a) hq[a] = R(0.25) * (k1[a] + k2[a]);
                        stage(hq, k3);
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            u[a] = (k1[a] + k2[a] + R(4) * k3[a]) / R(6);
                            v[a] = u[a];
                        }
                    } else {
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            u[a] = R(0.5) * (k1[a] + k2[a]);
                            v[a] = u[a];
                        }
                    }
                }
                R disp[3] = {R(0), R(0), R(0)};
#pragma unroll
                for (int a = 0; a < DIM; ++a) disp[a] = v[a] * U.dtdx[a];
                pos.advance(disp, U, err);
                pos.store(U, p);
#pragma unroll
                for (int a = 0; a < 3; ++a) U.u[a][p] = u[a];
            } else {
                // deposit of the current state
                if constexpr (KIND == PL_LORENTZ) {
                    R g2 = sqrt(fma(fma(u[0], u[0], fma(u[1], u[1], u[2] * u[2])), U.inv_c2, R(1)));
                    R qw = U.q * w;
                    mu[0] = (double)qw;
#pragma unroll
                    for (int a = 0; a < 3; ++a) mu[1 + a] = (double)(qw * u[a] / g2);
                } else {
                    mu[0] = (double)(U.m * w);
                }
                if (U.fp[0]) {
#pragma unroll
                    for (int a = 0; a < 3; ++a) mu[4 + a] = (double)U.fp[a][p];
                }
            }

            if (do_sums) {
#pragma unroll
                for (int k = 0; k < 8; ++k) ps[k] += mu[k];
            }

            if (dep_here) {
                R dn[3] = {(R)pos.d[0], (R)pos.d[1], (R)pos.d[2]};
                R wx[3], wy[3], wz[3];
                stencil_weights<PREC, SHAPE, DIM>(dn, wx, wy, wz);
                int base = 0;
                bool inl = TILED && in_tile<DIM>(tg, pos.c, base);
                deposit<PREC, DIM, CHS>(U, lds_d, inl, base, tg.Lx, tg.LxLy, tg.L, pos.c, wx, wy, wz, mu);
            }
        }

        if (KIND != PL_TRACER && do_sums) {
            for (int k = 0; k < 8; ++k) {
                double sw = wave_sum(ps[k]);
                if ((threadIdx.x & 63) == 0 && sw != 0.0) global_add(I.psum + k, sw);
            }
        }

        if (TILED && dep_here) {
            __syncthreads();
            const int Ly = tg.T[1] + 2;
            for (int e = threadIdx.x; e < tg.L; e += blockDim.x) {
                int lx = e % tg.Lx;
                int ly = (e / tg.Lx) % Ly;
                int lz = e / tg.LxLy;
                int gx = wrap_cell(tg.lo[0] + lx - 1, U.n[0]);
                int gy = wrap_cell(tg.lo[1] + ly - 1, U.n[1]);
                int gz = DIM >= 3 ? wrap_cell(tg.lo[2] + lz - 1, U.n[2]) : 0;
                long gc = gx + (long)U.n[0] * (gy + (long)U.n[1] * gz);
#pragma unroll
                for (int ch = 0; ch < kMaxCh; ++ch) {
                    int so = CHS != 0 ? (chs_slot(CHS, ch) >= 0 ? chs_slot(CHS, ch) * tg.L : -1) : U.soff[ch];
                    if (so < 0) continue;
                    double val = lds_d[so + e];
                    if (val != 0.0) global_add(U.M[ch] + gc, val * U.inv_dv);
                }
            }
        }
    }

    // latch device-side conditions
    unsigned long long any = __ballot(err != 0);
    if (any) {
        int e = err;
        for (int off = 32; off > 0; off >>= 1) e |= __shfl_xor(e, off, 64);
        if ((threadIdx.x & 63) == 0) atomicOr(errflags, e);
    }
    release_counter(counter);
}

// ---------------------------------------------------------------------------
// Host side: launch one persistent kernel over one group of items of the
// same species kind.
// ---------------------------------------------------------------------------

using StepKernel = void (*)(const ItemDesc *, int, int, unsigned *, int *, unsigned, int);

// Kernel variants: the 3D TSC tiled kernels also come with a compile-time tile
// shape (TS) and channel set (CHS) so LDS addresses become immediate offsets.
template <int PREC>
static StepKernel pick_kernel(int shape, int dim, bool tiled, int kind, int ts, int chs)
{
#define PL_K(S, D, T, K, TS_, CHS_) \
    if (shape == S && dim == D && tiled == T && kind == K && ts == TS_ && chs == CHS_) \
        return k_step<PREC, S, D, T, K, TS_, CHS_>;
#define PL_KIND_ALL(S, D, T) PL_K(S, D, T, PL_LORENTZ, 0, 0) PL_K(S, D, T, PL_DUST, 0, 0) PL_K(S, D, T, PL_TRACER, 0, 0)
#define PL_FAST(TS_) PL_K(PL_TSC, 3, true, PL_LORENTZ, TS_, 0) PL_K(PL_TSC, 3, true, PL_LORENTZ, TS_, 1) \
    PL_K(PL_TSC, 3, true, PL_DUST, TS_, 0) PL_K(PL_TSC, 3, true, PL_DUST, TS_, 2) PL_K(PL_TSC, 3, true, PL_TRACER, TS_, 0)
    PL_KIND_ALL(PL_TSC, 3, false) PL_KIND_ALL(PL_TSC, 2, false) PL_KIND_ALL(PL_TSC, 2, true)
    PL_KIND_ALL(PL_CIC, 3, false) PL_KIND_ALL(PL_CIC, 3, true) PL_KIND_ALL(PL_CIC, 2, false) PL_KIND_ALL(PL_CIC, 2, true)
    PL_FAST(0) PL_FAST(1) PL_FAST(2)
#undef PL_FAST
#undef PL_KIND_ALL
#undef PL_K
    return nullptr;
}

static inline int resident_blocks(Ctx *c, StepKernel k, int block, size_t lds)
{
    static std::map<std::pair<const void *, std::pair<int, size_t>>, int> cache;
    auto key = std::make_pair((const void *)k, std::make_pair(block, lds));
    auto f = cache.find(key);
    if (f != cache.end()) return f->second;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, block, lds) != hipSuccess || per_cu < 1) per_cu = 1;
    int r = per_cu * c->num_cu;
    cache[key] = r;
    return r;
}

template <int PREC>
hipError_t launch_group_impl(Ctx *c, const ItemDesc *table, const ItemDesc *host, int nitems, int total_units,
                             unsigned sf, bool push, bool deposit, unsigned *counter)
{
    if (total_units <= 0) return hipSuccess;
    const bool tiled = c->d.algo != PL_ALGO_PLAIN;
    const int kind = host[0].kind;
    // compile-time tile shape and channel set when every item of the group allows them
    int ts = 0, chs = 0;
    if (tiled && c->d.shape == PL_TSC && c->d.ndim == 3) {
        for (int cand = 1; cand <= 2 && ts == 0; ++cand) {
            bool all = true;
            for (int i = 0; i < nitems; ++i)
                for (int a = 0; a < 3; ++a) all = all && host[i].tile[a] == ts_dim(cand, a);
            if (all) ts = cand;
        }
        int want = kind == PL_LORENTZ ? 1 : kind == PL_DUST ? 2 : 0;
        bool all = want != 0 && deposit;
        for (int i = 0; i < nitems && all; ++i)
            for (int ch = 0; ch < kMaxCh; ++ch) all = all && host[i].slot[ch] == chs_slot(want, ch);
        chs = all ? want : 0;
    }
    StepKernel k = pick_kernel<PREC>(c->d.shape, c->d.ndim, tiled, kind, ts, chs);
    if (!k) return hipErrorInvalidValue;
    size_t lds = 16;
    if (tiled) {
        for (int i = 0; i < nitems; ++i) {
            const ItemDesc &it = host[i];
            int L = (it.tile[0] + 2) * (it.tile[1] + 2) * (c->d.ndim >= 3 ? it.tile[2] + 2 : 1);
            int ns = (deposit && it.kind != PL_TRACER) ? it.nslot : 0;
            lds = std::max(lds, step_lds_bytes(PREC, it.kind, L, push, ns));
        }
        if (lds > (size_t)c->lds_max) return hipErrorInvalidConfiguration;
    }
    int block = c->block;
    int grid = std::min(total_units, resident_blocks(c, k, block, lds));
    hipLaunchKernelGGL(k, dim3(grid), dim3(block), lds, c->stream, table, nitems, total_units, counter, c->errflags,
                       sf, (int)lds);
    c->stats[0]++;
    return hipGetLastError();
}

}  // namespace pl
