// Run-based gather -> push -> deposit kernel for gfx950 (template;
// instantiated per precision in k_runs_f32.hip and k_runs_f64.hip).
//
// Work unit: a piece of one cell tile of one item (the sort cuts a crowded
// tile into pieces of equal run count and lists the units largest first).
// The sort cuts the particles of every cell into runs of up to kRunLen
// consecutive particles and lists the runs of a tile by (index of the run
// inside its cell, cell), so the threads of a wave hold runs of distinct
// neighbouring cells; with the run-order key the runs also lie in memory in
// table order, so a wave's particle loads and stores are contiguous.  A
// thread advances its run in register batches of KR particles that share one
// cell:
//  * each batch particle interpolates its fields from the 27 (9 in 2D)
//    records of its own cell's stencil in the LDS field tile (one or two
//    16-byte reads per record in float32, three in float64);
//  * after the push, the batch's deposits are summed per stencil point and
//    channel before one float64 LDS atomic, cutting LDS atomics by the run
//    length;
//  * the LDS deposit tile carries a two-cell halo, so particles that drifted
//    up to one cell out of the tile since the sort still deposit into LDS;
//    the field tile does too where the LDS allows it (else one cell).
// A particle that moved since the sort is still gathered in its batch, from
// its own cell, while its stencil lies in the field tile; outside the tile it
// is queued in LDS for the single-particle path.  After the push, batch
// particles outside the batch's reference cell queue their deposit.  Queued
// work runs after the runs, or immediately when a queue is full.
// Per particle, gathers and pushes add the same terms in the same order as the
// tiled kernel (explicit fma), so particle states are bit-identical to it.
#pragma once

#include "k_step_impl.h"

namespace pl {

// Capacity of the queue of particles that need the HBM gather: with a
// two-cell field halo only particles two cells out of their tile land there.
__host__ __device__ constexpr int gq_cap(int hf) { return hf == 2 ? 64 : 256; }

template <int PREC> struct RunsQ { static constexpr int DQ = PREC == PL_F32_OFFSET ? 256 : 128; };

// LDS field records, read with 16-byte loads.  Lanes of a wave read
// records of neighbouring cells, so the record stride decides the bank
// pattern: float32 charged particles use two planes of 16-byte records
// (E0 E1 E2 0 | B0 B1 B2 0, the B plane Lf records after the E plane), so 16
// lanes of one pass cover all 64 banks; float64 charged: one 48-byte record
// E0 E1 E2 B0 B1 B2; three-component kinds: v0 v1 v2 0.
template <int PREC, int KIND> struct FieldRec {
    static constexpr int NC = KIND == PL_LORENTZ ? 6 : 3;
    static constexpr int FS = PREC == PL_F32_OFFSET ? (NC == 6 ? 8 : 4) : (NC == 6 ? 6 : 4);
    static constexpr bool PLANES = PREC == PL_F32_OFFSET && NC == 6;
    // position of component q of cell e in a tile of Lf records
    __host__ __device__ static constexpr int at(int e, int q, int Lf)
    {
        return PLANES ? (q < 3 ? 4 * e + q : 4 * Lf + 4 * e + (q - 3)) : FS * e + q;
    }
};

template <int PREC, int KIND>
__device__ __forceinline__ void load_rec(const typename RealOf<PREC>::T *lds_f, int cell, int Lf,
                                         typename RealOf<PREC>::T f[FieldRec<PREC, KIND>::NC])
{
    if constexpr (PREC == PL_F32_OFFSET) {
        const float4 *p = reinterpret_cast<const float4 *>(lds_f);
        if constexpr (KIND == PL_LORENTZ) {
            float4 a = p[cell], b = p[Lf + cell];
            f[0] = a.x; f[1] = a.y; f[2] = a.z; f[3] = b.x; f[4] = b.y; f[5] = b.z;
        } else {
            float4 a = p[cell];
            f[0] = a.x; f[1] = a.y; f[2] = a.z;
        }
    } else {
        const double2 *p = reinterpret_cast<const double2 *>(lds_f);
        if constexpr (KIND == PL_LORENTZ) {
            double2 a = p[3 * cell], b = p[3 * cell + 1], c = p[3 * cell + 2];
            f[0] = a.x; f[1] = a.y; f[2] = b.x; f[3] = b.y; f[4] = c.x; f[5] = c.y;
        } else {
            double2 a = p[2 * cell], b = p[2 * cell + 1];
            f[0] = a.x; f[1] = a.y; f[2] = b.x;
        }
    }
}

__device__ __forceinline__ int wrap_any(int i, int n)
{
    int r = i % n;
    return r < 0 ? r + n : r;
}

// Geometry of one tile: field tile with an hf-cell halo (1 or 2), deposit
// tile with a two-cell halo.
struct RunGeo {
    int lo[3], T[3];
    int hf;
    int fx, fxy, Lf;
    int dx, dxy, Ld;
};

// LDS index (field tile) of stencil point (-1,-1,-1) of a particle in cell c,
// when the whole stencil lies in the field tile (c at most hf - 1 cells
// outside the tile, periodically).
template <int DIM>
__device__ __forceinline__ bool field_base(const RunGeo &g, const int n[3], const int c[3], int &base)
{
    bool ok = true;
    int l[3] = {0, 0, 0};
    const int h = g.hf - 1;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        int v = c[a] - g.lo[a];
        if (v < -h) v += n[a];
        else if (v > g.T[a] - 1 + h) v -= n[a];
        ok = ok && v >= -h && v <= g.T[a] - 1 + h;
        l[a] = v + h;
    }
    base = l[0] + (DIM >= 2 ? l[1] * g.fx : 0) + (DIM >= 3 ? l[2] * g.fxy : 0);
    return ok;
}

// LDS index (deposit tile) of stencil point (-1,-1,-1), when the stencil lies
// in the deposit tile (c at most one cell outside the tile, periodically).
template <int DIM>
__device__ __forceinline__ bool dep_base(const RunGeo &g, const int n[3], const int c[3], int &base)
{
    bool ok = true;
    int l[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        int v = c[a] - g.lo[a];
        if (v < -1) v += n[a];
        else if (v > g.T[a]) v -= n[a];
        ok = ok && v >= -1 && v <= g.T[a];
        l[a] = v + 1;
    }
    base = l[0] + (DIM >= 2 ? l[1] * g.dx : 0) + (DIM >= 3 ? l[2] * g.dxy : 0);
    return ok;
}

template <int DIM>
__device__ __forceinline__ bool same_cell(const int a[3], const int b[3])
{
    bool s = a[0] == b[0];
    if (DIM >= 2) s = s && a[1] == b[1];
    if (DIM >= 3) s = s && a[2] == b[2];
    return s;
}

// Push of one particle with interpolated fields F (E, B or the gas velocity):
// updates u, returns the velocity v used for the position update and the
// deposit values mu (charge / mass, current, force, energy) per channel.
template <int PREC, int KIND>
__device__ __forceinline__ void push_particle(const UnitC<PREC> &U, typename RealOf<PREC>::T u[3],
                                              const typename RealOf<PREC>::T *F, typename RealOf<PREC>::T w,
                                              typename RealOf<PREC>::T v[3], typename RealOf<PREC>::T mu[kMaxCh])
{
    using R = typename RealOf<PREC>::T;
    if constexpr (KIND == PL_LORENTZ) {
        R du[3];
        R uo[3] = {u[0], u[1], u[2]};
        R u_old2 = fma(u[0], u[0], fma(u[1], u[1], u[2] * u[2]));
        boris<R>(u, F, F + 3, U.h, U.inv_c2, du);
        R u_new2 = fma(u[0], u[0], fma(u[1], u[1], u[2] * u[2]));
        const R gn2 = fma(u_new2, U.inv_c2, R(1));
        R gn = sqrt(gn2);
        R go = sqrt(fma(u_old2, U.inv_c2, R(1)));
        R ig = div_sqrt_ge1(R(1), gn2);
#pragma unroll
        for (int a = 0; a < 3; ++a) v[a] = u[a] * ig;
        R qw = U.q * w, mw = U.m * w;
        mu[0] = qw;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            mu[1 + a] = qw * v[a];
            mu[4 + a] = mw * du[a] * U.inv_dt;
        }
        if constexpr (PREC == PL_F64) {
            mu[7] = mw * U.c2 * (gn - go) * U.inv_dt;
        } else {
            R dd = fma(du[0], u[0] + uo[0], fma(du[1], u[1] + uo[1], du[2] * (u[2] + uo[2])));
            mu[7] = mw * dd / (gn + go) * U.inv_dt;
        }
    } else {
        R du[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            du[a] = (F[a] - u[a]) * U.one_m_decay;
            u[a] = F[a] + (u[a] - F[a]) * U.decay;
            v[a] = u[a];
        }
        R mw = U.m * w;
        mu[0] = mw;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            mu[1 + a] = R(0);
            mu[4 + a] = mw * du[a] * U.inv_dt;
        }
        mu[7] = R(0);
    }
}

// Offset of channel ch's plane in the LDS deposit tile (compile-time for
// CHS != 0), -1 when the channel is inactive.
template <int CHS, class U_>
__device__ __forceinline__ int ch_off(const U_ &U, int ch, int Ld)
{
    if constexpr (CHS != 0) return chs_slot(CHS, ch) >= 0 ? chs_slot(CHS, ch) * Ld : -1;
    else return U.soff[ch];
}

template <int PREC> struct RunShared {
    using R = typename RealOf<PREC>::T;
    const R *lds_f;
    double *lds_d;
    int *gq;
    uint32_t *dq_c;
    R *dq_d;      // 3 x DQ
    R *dq_mu;     // nslot x DQ
    int *ctl;     // [0] claimed unit, [1] queued particles, [2] queued deposits
    double *sums; // 8 particle-side sums of the unit
};

// Particle-side conservation sums (only with SF_SUMS): LDS accumulation per
// unit, one global add per unit.
template <int PREC>
__device__ __forceinline__ void add_sums(const RunShared<PREC> &S, const typename RealOf<PREC>::T mu[kMaxCh])
{
#pragma unroll
    for (int k = 0; k < 8; ++k)
        __hip_atomic_fetch_add(S.sums + k, (double)mu[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Interpolate the fields of the LDS field tile to a particle whose stencil
// starts at record `fb`: the 27 (9 in 2D) records are read kPrefetch points
// ahead of their use, so several LDS reads are in flight while the previous
// points are summed.  Terms are added in the order (k, j, i) with explicit
// fused multiply-adds, the order of the tiled kernel.
constexpr int kPrefetch = 4;

template <int PREC, int DIM, int KIND>
__device__ __forceinline__ void gather_rec(const RunGeo &G, const typename RealOf<PREC>::T *lds_f, int fb,
                                           const typename RealOf<PREC>::T wx[3], const typename RealOf<PREC>::T wy[3],
                                           const typename RealOf<PREC>::T wz[3],
                                           typename RealOf<PREC>::T F[FieldRec<PREC, KIND>::NC])
{
    using R = typename RealOf<PREC>::T;
    constexpr int NC = FieldRec<PREC, KIND>::NC;
    constexpr int SY = Stencil<DIM>::SY, SZ = Stencil<DIM>::SZ;
    constexpr int NPT = SZ * SY * 3;
    constexpr int NB = kPrefetch + 1;
    R buf[NB][NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) F[q] = R(0);
#pragma unroll
    for (int pt = 0; pt < kPrefetch && pt < NPT; ++pt)
        load_rec<PREC, KIND>(lds_f, fb + (pt / 9) * G.fxy + ((pt / 3) % 3) * G.fx + pt % 3, G.Lf, buf[pt % NB]);
    R wyz = R(0);
#pragma unroll
    for (int pt = 0; pt < NPT; ++pt) {
        const int nx = pt + kPrefetch;
        if (nx < NPT)
            load_rec<PREC, KIND>(lds_f, fb + (nx / 9) * G.fxy + ((nx / 3) % 3) * G.fx + nx % 3, G.Lf, buf[nx % NB]);
        const int k = pt / 9, j = (pt / 3) % 3, i = pt % 3;
        if (i == 0) wyz = wz[k] * wy[j];
        const R wt = wyz * wx[i];
#pragma unroll
        for (int q = 0; q < NC; ++q) F[q] = fma(wt, buf[pt % NB][q], F[q]);
    }
}

// Deposit one particle (cell c, offset d, values mu per channel) into the LDS
// deposit tile when its stencil fits, else into the grids.
template <int PREC, int SHAPE, int DIM, int CHS>
__device__ __forceinline__ void deposit_single(const UnitC<PREC> &U, const RunGeo &G, double *lds_d, const int c[3],
                                               const typename RealOf<PREC>::T d[3], const double mu[kMaxCh])
{
    using R = typename RealOf<PREC>::T;
    R wx[3], wy[3], wz[3];
    stencil_weights<PREC, SHAPE, DIM>(d, wx, wy, wz);
    int base = 0;
    bool inl = dep_base<DIM>(G, U.n, c, base);
    deposit<PREC, DIM, CHS>(U, lds_d, inl, base, G.dx, G.dxy, G.Ld, c, wx, wy, wz, mu);
}

// The whole step of one particle on its own: gather from the LDS field tile
// when its stencil fits, else from the grids; push; store; deposit.
template <int PREC, int SHAPE, int DIM, int KIND, int CHS>
__device__ __forceinline__ void particle_single(const UnitC<PREC> &U, const RunGeo &G, const RunShared<PREC> &S, int p,
                                             bool do_sums, int &err)
{
    using R = typename RealOf<PREC>::T;
    constexpr int NC = FieldRec<PREC, KIND>::NC;
    Pos<PREC, DIM> pos;
    pos.load(U, p, err);
    R u[3] = {U.u[0][p], U.u[1][p], U.u[2][p]};
    R w = U.w ? U.w[p] : U.wdef;
    R d0[3] = {(R)pos.d[0], (R)pos.d[1], (R)pos.d[2]};
    R wx[3], wy[3], wz[3];
    stencil_weights<PREC, SHAPE, DIM>(d0, wx, wy, wz);
    R F[NC];
    int fb = 0;
    if (field_base<DIM>(G, U.n, pos.c, fb)) {
        gather_rec<PREC, DIM, KIND>(G, S.lds_f, fb, wx, wy, wz, F);
    } else {
        gather<PREC, DIM, NC>(U, nullptr, 0, false, 0, 0, 0, pos.c, wx, wy, wz, F);
    }
    R v[3], mu[kMaxCh];
    push_particle<PREC, KIND>(U, u, F, w, v, mu);
    if (U.fp[0]) {
#pragma unroll
        for (int a = 0; a < 3; ++a) U.fp[a][p] = mu[4 + a];
    }
    R disp[3] = {R(0), R(0), R(0)};
#pragma unroll
    for (int a = 0; a < DIM; ++a) disp[a] = v[a] * U.dtdx[a];
    pos.advance(disp, U, err);
    pos.store(U, p);
#pragma unroll
    for (int a = 0; a < 3; ++a) U.u[a][p] = u[a];
    double mud[kMaxCh];
#pragma unroll
    for (int ch = 0; ch < kMaxCh; ++ch) mud[ch] = (double)mu[ch];
    if (do_sums) add_sums(S, mu);
    R dn[3] = {(R)pos.d[0], (R)pos.d[1], (R)pos.d[2]};
    deposit_single<PREC, SHAPE, DIM, CHS>(U, G, S.lds_d, pos.c, dn, mud);
}

// Deposit of a queued record.
template <int PREC, int SHAPE, int DIM, int CHS>
__device__ __forceinline__ void record_deposit(const UnitC<PREC> &U, const RunGeo &G, const RunShared<PREC> &S, int i)
{
    using R = typename RealOf<PREC>::T;
    constexpr int DQ = RunsQ<PREC>::DQ;
    int c[3];
    unpack_cell(S.dq_c[i], c[0], c[1], c[2]);
    R d[3] = {S.dq_d[i], S.dq_d[DQ + i], S.dq_d[2 * DQ + i]};
    double mu[kMaxCh];
#pragma unroll
    for (int ch = 0; ch < kMaxCh; ++ch) {
        int so = ch_off<CHS>(U, ch, G.Ld);
        mu[ch] = so >= 0 ? (double)S.dq_mu[(so / G.Ld) * DQ + i] : 0.0;
    }
    deposit_single<PREC, SHAPE, DIM, CHS>(U, G, S.lds_d, c, d, mu);
}

// Deposit of the batch particles in the reference cell (dco[j]): their values
// are summed per stencil point and channel before each LDS atomic.
template <int PREC, int SHAPE, int DIM, int CHS, int KR>
__device__ __forceinline__ void batch_deposit(const UnitC<PREC> &U, const RunGeo &G, const RunShared<PREC> &S, int db,
                                              const Pos<PREC, DIM> pos[KR], typename RealOf<PREC>::T mu[KR][kMaxCh],
                                              const bool dco[KR])
{
    using R = typename RealOf<PREC>::T;
    constexpr int SY = Stencil<DIM>::SY, SZ = Stencil<DIM>::SZ;
    R wx[KR][3], wy[KR][3], wz[KR][3];
#pragma unroll
    for (int j = 0; j < KR; ++j) {
        R dn[3] = {(R)pos[j].d[0], (R)pos[j].d[1], (R)pos[j].d[2]};
        stencil_weights<PREC, SHAPE, DIM>(dn, wx[j], wy[j], wz[j]);
#pragma unroll
        for (int ch = 0; ch < kMaxCh; ++ch) mu[j][ch] = dco[j] ? mu[j][ch] : R(0);
    }
#pragma unroll
    for (int k = 0; k < SZ; ++k)
#pragma unroll
        for (int jj = 0; jj < SY; ++jj) {
            R wyz[KR];
#pragma unroll
            for (int j = 0; j < KR; ++j) wyz[j] = wz[j][k] * wy[j][jj];
            const int row = db + k * G.dxy + jj * G.dx;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                R wt[KR];
#pragma unroll
                for (int j = 0; j < KR; ++j) wt[j] = wyz[j] * wx[j][i];
#pragma unroll
                for (int ch = 0; ch < kMaxCh; ++ch) {
                    const int so = ch_off<CHS>(U, ch, G.Ld);
                    if (so < 0) continue;
                    R s = wt[0] * mu[0][ch];
#pragma unroll
                    for (int j = 1; j < KR; ++j) s = fma(wt[j], mu[j][ch], s);
                    __hip_atomic_fetch_add(S.lds_d + so + row + i, (double)s, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
                }
            }
        }
}

// K consecutive elements of one particle array in one access.  The sort keeps
// a run's particles consecutive, and with the run order the runs of a wave
// follow one another, so these loads and stores cover contiguous stretches.
// Only element alignment is known (a batch starts at any particle), so the
// vector type declares exactly that; gfx950's multi-dword global accesses
// need dword alignment only.
template <class T, int K> struct Vec {
    typedef T V __attribute__((ext_vector_type(K), aligned(sizeof(T))));
    typedef __attribute__((address_space(1))) V *P;
    typedef const __attribute__((address_space(1))) V *CP;
};

template <class T, int K>
__device__ __forceinline__ void load_vec(gptr<const T> p, T (&out)[K])
{
    const typename Vec<T, K>::V v = *reinterpret_cast<typename Vec<T, K>::CP>(p);
#pragma unroll
    for (int k = 0; k < K; ++k) out[k] = v[k];
}

template <class T, int K>
__device__ __forceinline__ void store_vec(gptr<T> p, const T (&in)[K])
{
    typename Vec<T, K>::V v;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = in[k];
    *reinterpret_cast<typename Vec<T, K>::P>(p) = v;
}

// State of a whole batch (every slot handled in place) written back with one
// access per array.
template <int PREC, int DIM, int KR>
__device__ __forceinline__ void store_batch(const UnitC<PREC> &U, int start, const Pos<PREC, DIM> pos[KR],
                                            const typename RealOf<PREC>::T u[KR][3],
                                            const typename RealOf<PREC>::T mu[KR][kMaxCh])
{
    using R = typename RealOf<PREC>::T;
    R t[KR];
    if constexpr (PREC == PL_F32_OFFSET) {
        uint32_t cv[KR];
#pragma unroll
        for (int j = 0; j < KR; ++j)
            cv[j] = pack_cell(pos[j].c[0], DIM > 1 ? pos[j].c[1] : 0, DIM > 2 ? pos[j].c[2] : 0);
        store_vec<uint32_t, KR>(U.cell + start, cv);
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
#pragma unroll
            for (int j = 0; j < KR; ++j) t[j] = pos[j].d[a];
            store_vec<R, KR>(U.x[a] + start, t);
        }
    } else {
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
#pragma unroll
            for (int j = 0; j < KR; ++j) t[j] = pos[j].x[a];
            store_vec<R, KR>(U.x[a] + start, t);
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int j = 0; j < KR; ++j) t[j] = u[j][a];
        store_vec<R, KR>(U.u[a] + start, t);
    }
    if (U.fp[0]) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
#pragma unroll
            for (int j = 0; j < KR; ++j) t[j] = mu[j][4 + a];
            store_vec<R, KR>(U.fp[a] + start, t);
        }
    }
}

// Gather, push and deposit of the batch particles whose stencil lies in the
// LDS field tile (co[j]); fb[j] is the field record of stencil point
// (-1,-1,-1) of particle j.
template <int PREC, int SHAPE, int DIM, int KIND, int CHS, int KR>
__device__ __forceinline__ void batch_body(const UnitC<PREC> &U, const RunGeo &G, const RunShared<PREC> &S, int start,
                                           const int fb[KR], Pos<PREC, DIM> pos[KR], typename RealOf<PREC>::T u[KR][3],
                                           const typename RealOf<PREC>::T w[KR], const bool co[KR], bool do_sums, int &err)
{
    using R = typename RealOf<PREC>::T;
    constexpr int NC = FieldRec<PREC, KIND>::NC;
    constexpr int SY = Stencil<DIM>::SY, SZ = Stencil<DIM>::SZ;
    constexpr int DQ = RunsQ<PREC>::DQ;

    // a batch whose slots are all handled here is written back at the end with
    // one access per array; otherwise every slot is stored on its own
    bool whole = true;
#pragma unroll
    for (int j = 0; j < KR; ++j) whole = whole && co[j];

    // gather and push one particle at a time (each stencil point is one
    // interleaved LDS record read); keep what the batched deposit needs
    R mu[KR][kMaxCh];
#pragma unroll
    for (int j = 0; j < KR; ++j) {
        const int p = start + j;
        R wx[3], wy[3], wz[3];
        R d0[3] = {(R)pos[j].d[0], (R)pos[j].d[1], (R)pos[j].d[2]};
        stencil_weights<PREC, SHAPE, DIM>(d0, wx, wy, wz);
        R F[NC];
        gather_rec<PREC, DIM, KIND>(G, S.lds_f, fb[j], wx, wy, wz, F);
        R v[3];
        push_particle<PREC, KIND>(U, u[j], F, w[j], v, mu[j]);
        R disp[3] = {R(0), R(0), R(0)};
#pragma unroll
        for (int a = 0; a < DIM; ++a) disp[a] = v[a] * U.dtdx[a];
        int e2 = 0;
        pos[j].advance(disp, U, e2);
        if (co[j]) {
            err |= e2;
            if (!whole) {
                pos[j].store(U, p);
#pragma unroll
                for (int a = 0; a < 3; ++a) U.u[a][p] = u[j][a];
                if (U.fp[0]) {
#pragma unroll
                    for (int a = 0; a < 3; ++a) U.fp[a][p] = mu[j][4 + a];
                }
            }
            if (do_sums) add_sums(S, mu[j]);
        }
    }
    if (whole) store_batch<PREC, DIM, KR>(U, start, pos, u, mu);

    // deposit: the batch particles in the reference cell are summed before
    // each LDS atomic; the others are queued.  The reference is the new cell
    // of the first batch particle, or of the second when the first shares its
    // cell with no other batch particle.
    int f0 = -1, f1 = -1;
#pragma unroll
    for (int j = KR - 1; j >= 0; --j) {
        if (co[j]) {
            f1 = f0;
            f0 = j;
        }
    }
    int rc[3] = {0, 0, 0};
#pragma unroll
    for (int j = 0; j < KR; ++j)
        if (j == f0)
#pragma unroll
            for (int a = 0; a < 3; ++a) rc[a] = pos[j].c[a];
    bool alone = true;
#pragma unroll
    for (int j = 0; j < KR; ++j) alone = alone && (j == f0 || !(co[j] && same_cell<DIM>(pos[j].c, rc)));
    if (alone && f1 >= 0) {
#pragma unroll
        for (int j = 0; j < KR; ++j)
            if (j == f1)
#pragma unroll
                for (int a = 0; a < 3; ++a) rc[a] = pos[j].c[a];
    }
    int db = 0;
    const bool dep_in = dep_base<DIM>(G, U.n, rc, db);
    bool dco[KR];
    bool any_dco = false;
#pragma unroll
    for (int j = 0; j < KR; ++j) {
        dco[j] = co[j] && dep_in && same_cell<DIM>(pos[j].c, rc);
        any_dco = any_dco || dco[j];
    }
    unsigned ovf_d = 0;
#pragma unroll
    for (int j = 0; j < KR; ++j) {
        if (co[j] && !dco[j]) {
            int q = atomicAdd(&S.ctl[2], 1);
            if (q < DQ) {
                S.dq_c[q] = pack_cell(pos[j].c[0], DIM > 1 ? pos[j].c[1] : 0, DIM > 2 ? pos[j].c[2] : 0);
#pragma unroll
                for (int a = 0; a < 3; ++a) S.dq_d[a * DQ + q] = (R)pos[j].d[a];
#pragma unroll
                for (int ch = 0; ch < kMaxCh; ++ch) {
                    int so = ch_off<CHS>(U, ch, G.Ld);
                    if (so >= 0) S.dq_mu[(so / G.Ld) * DQ + q] = mu[j][ch];
                }
            } else {
                ovf_d |= 1u << j;
            }
        }
    }
    // deposits that found the queue full
#pragma unroll
    for (int j = 0; j < KR; ++j) {
        if (ovf_d & (1u << j)) {
            double mud[kMaxCh];
#pragma unroll
            for (int ch = 0; ch < kMaxCh; ++ch) mud[ch] = (double)mu[j][ch];
            R dn[3] = {(R)pos[j].d[0], (R)pos[j].d[1], (R)pos[j].d[2]};
            deposit_single<PREC, SHAPE, DIM, CHS>(U, G, S.lds_d, pos[j].c, dn, mud);
        }
    }
    if (any_dco) batch_deposit<PREC, SHAPE, DIM, CHS, KR>(U, G, S, db, pos, mu, dco);
}

// Stored state of one batch (up to KR consecutive particles), fetched from
// HBM one batch ahead of its use so the loads overlap the previous batch.
template <int PREC, int DIM, int KR> struct BatchRaw {
    using R = typename RealOf<PREC>::T;
    typename Pos<PREC, DIM>::Raw pr[KR];
    R u[KR][3], w[KR];
    int start, len;
};

template <int PREC, int DIM, int KR>
__device__ __forceinline__ void fetch_batch(const UnitC<PREC> &U, int start, int len, BatchRaw<PREC, DIM, KR> &B)
{
    using R = typename RealOf<PREC>::T;
    B.start = start;
    B.len = len;
    if (len == KR) {
        // a whole batch: one access per array
        R t[KR];
        if constexpr (PREC == PL_F32_OFFSET) {
            uint32_t cv[KR];
            load_vec<uint32_t, KR>((gptr<const uint32_t>)(U.cell + start), cv);
#pragma unroll
            for (int j = 0; j < KR; ++j) B.pr[j].cell = cv[j];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (a < DIM) load_vec<R, KR>((gptr<const R>)(U.x[a] + start), t);
#pragma unroll
                for (int j = 0; j < KR; ++j) B.pr[j].o[a] = a < DIM ? t[j] : 0.0f;
            }
        } else {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (a < DIM) load_vec<R, KR>((gptr<const R>)(U.x[a] + start), t);
#pragma unroll
                for (int j = 0; j < KR; ++j) B.pr[j].x[a] = a < DIM ? t[j] : 0.0;
            }
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            load_vec<R, KR>((gptr<const R>)(U.u[a] + start), t);
#pragma unroll
            for (int j = 0; j < KR; ++j) B.u[j][a] = t[j];
        }
        if (U.w) {
            load_vec<R, KR>(U.w + start, t);
#pragma unroll
            for (int j = 0; j < KR; ++j) B.w[j] = t[j];
        } else {
#pragma unroll
            for (int j = 0; j < KR; ++j) B.w[j] = U.wdef;
        }
        return;
    }
#pragma unroll
    for (int j = 0; j < KR; ++j) {
        const int p = start + j;
        const bool in = j < len;
        if (in) Pos<PREC, DIM>::fetch(U, p, B.pr[j]);
        else B.pr[j] = B.pr[0];
#pragma unroll
        for (int a = 0; a < 3; ++a) B.u[j][a] = in ? U.u[a][p] : R(0);
        B.w[j] = in ? (U.w ? U.w[p] : U.wdef) : R(0);
    }
}

// One batch of up to KR particles of one run.
template <int PREC, int SHAPE, int DIM, int KIND, int CHS, int KR>
__device__ __forceinline__ void run_batch(const UnitC<PREC> &U, const RunGeo &G, const RunShared<PREC> &S,
                                          const BatchRaw<PREC, DIM, KR> &Bt, bool do_sums, int &err)
{
    using R = typename RealOf<PREC>::T;
    const int start = Bt.start, len = Bt.len;
    Pos<PREC, DIM> pos[KR];
    R u[KR][3], w[KR];
#pragma unroll
    for (int j = 0; j < KR; ++j) {
        if (j < len) pos[j].set(Bt.pr[j], U, err);
        else pos[j] = pos[0];
#pragma unroll
        for (int a = 0; a < 3; ++a) u[j][a] = Bt.u[j][a];
        w[j] = Bt.w[j];
    }
    // every particle whose stencil lies in the LDS field tile is gathered in
    // the batch from its own cell (lanes read distinct records anyway)
    int fb[KR];
    bool co[KR];
#pragma unroll
    for (int j = 0; j < KR; ++j) {
        co[j] = field_base<DIM>(G, U.n, pos[j].c, fb[j]) && j < len;
        if (!co[j]) fb[j] = 0;       // computed but unused: keep its reads inside the field tile
    }
    // particles outside the tile: queue for the single-particle path (when
    // the queue is full they run on their own after the batch)
    unsigned ovf_g = 0;
#pragma unroll
    for (int j = 0; j < KR; ++j) {
        if (j < len && !co[j]) {
            int q = atomicAdd(&S.ctl[1], 1);
            if (q < gq_cap(G.hf)) S.gq[q] = start + j;
            else ovf_g |= 1u << j;
        }
    }
    bool any = false;
#pragma unroll
    for (int j = 0; j < KR; ++j) any = any || co[j];
    if (any) batch_body<PREC, SHAPE, DIM, KIND, CHS, KR>(U, G, S, start, fb, pos, u, w, co, do_sums, err);
    while (ovf_g) {
        const int j = __builtin_ctz(ovf_g);
        ovf_g &= ovf_g - 1u;
        particle_single<PREC, SHAPE, DIM, KIND, CHS>(U, G, S, start + j, do_sums, err);
    }
}

// LDS bytes of one work unit: field records, float64 deposit tile, queues,
// a 16-byte control tail.
__host__ __device__ inline size_t runs_section(size_t b) { return (b + 15) & ~(size_t)15; }

template <int PREC, int KIND>
__host__ __device__ inline size_t runs_lds_bytes(int Lf, int Ld, int nslot, int hf, size_t offs[6])
{
    using R = typename RealOf<PREC>::T;
    constexpr int DQ = RunsQ<PREC>::DQ;
    size_t o = 0;
    offs[0] = o; o += runs_section((size_t)Lf * FieldRec<PREC, KIND>::FS * sizeof(R));
    offs[1] = o; o += runs_section((size_t)Ld * nslot * sizeof(double));
    offs[2] = o; o += runs_section((size_t)gq_cap(hf) * sizeof(int));
    offs[3] = o; o += runs_section((size_t)DQ * sizeof(uint32_t));
    offs[4] = o; o += runs_section((size_t)DQ * (3 + nslot) * sizeof(R));
    offs[5] = o; o += 8 * sizeof(double);
    return o + 16;
}

// Threads per block of the run kernel.  One block per CU (the LDS tiles take
// most of the 160 KB), so two waves per SIMD: the compiler may spend registers
// on reads in flight.
constexpr int kRunsThreads = 512;

// Gas velocity at a position of the Runge-Kutta scheme: from the LDS field
// records when the stencil lies in the tile's field tile, else from the grid.
template <int PREC, int SHAPE, int DIM>
__device__ __forceinline__ void tracer_velocity(const UnitC<PREC> &U, const RunGeo &G,
                                                const typename RealOf<PREC>::T *lds_f, const Pos<PREC, DIM> &q,
                                                typename RealOf<PREC>::T k[3])
{
    using R = typename RealOf<PREC>::T;
    R dm[3] = {(R)q.d[0], (R)q.d[1], (R)q.d[2]};
    R sx[3], sy[3], sz[3];
    stencil_weights<PREC, SHAPE, DIM>(dm, sx, sy, sz);
    int fb = 0;
    if (field_base<DIM>(G, U.n, q.c, fb)) gather_rec<PREC, DIM, PL_TRACER>(G, lds_f, fb, sx, sy, sz, k);
    else gather<PREC, DIM, 3>(U, nullptr, 0, false, 0, 0, 0, q.c, sx, sy, sz, k);
}

// One passive tracer on the gas velocity frozen over the step (Eq. 1):
// Heun's two-stage scheme, or the three-stage SSP scheme of Shu and Osher,
// x + dt (k1 + k2 + 4 k3) / 6 with k1 = v(x), k2 = v(x + dt k1),
// k3 = v(x + dt (k1 + k2) / 4); the stored velocity is the step's mean.
// The same terms in the same order as the tiled kernel's tracer path.
template <int PREC, int SHAPE, int DIM>
__device__ __forceinline__ void tracer_particle(const UnitC<PREC> &U, const RunGeo &G,
                                                const typename RealOf<PREC>::T *lds_f, int p, int &err)
{
    using R = typename RealOf<PREC>::T;
    Pos<PREC, DIM> pos;
    pos.load(U, p, err);
    R k1[3], k2[3], v[3];
    tracer_velocity<PREC, SHAPE, DIM>(U, G, lds_f, pos, k1);
    // velocity of the stage at x + dt * s (s in cells per unit time)
    auto stage = [&](const R sv[3], R k[3]) {
        Pos<PREC, DIM> mid = pos;
        R dd[3] = {R(0), R(0), R(0)};
#pragma unroll
        for (int a = 0; a < DIM; ++a) dd[a] = sv[a] * U.dtdx[a];
        mid.advance(dd, U, err);
        tracer_velocity<PREC, SHAPE, DIM>(U, G, lds_f, mid, k);
    };
    stage(k1, k2);
    if (U.rk == 3) {
        R hq[3], k3[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) hq[a] = R(0.25) * (k1[a] + k2[a]);
        stage(hq, k3);
#pragma unroll
        for (int a = 0; a < 3; ++a) v[a] = (k1[a] + k2[a] + R(4) * k3[a]) / R(6);
    } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) v[a] = R(0.5) * (k1[a] + k2[a]);
    }
    R disp[3] = {R(0), R(0), R(0)};
#pragma unroll
    for (int a = 0; a < DIM; ++a) disp[a] = v[a] * U.dtdx[a];
    pos.advance(disp, U, err);
    pos.store(U, p);
#pragma unroll
    for (int a = 0; a < 3; ++a) U.u[a][p] = v[a];
}

// One work unit of the run kernel (a piece of tile t of item I): stage the
// tile's field records (and clear its deposit tile), advance the piece's
// runs, and flush the deposits; passive tracers are advanced one particle at
// a time from the same field records.  The next unit is claimed into ctl[0]
// before the flush (pre = true).
template <int PREC, int SHAPE, int DIM, int KIND, int HF, int TS, int CHS>
__device__ __forceinline__ void runs_unit(const ItemDesc &I, int t, int piece, int npieces, unsigned flags,
                                          int lds_bytes, unsigned char *smem_raw, unsigned *counter, bool &pre,
                                          int &err)
{
    using R = typename RealOf<PREC>::T;
    using FR = FieldRec<PREC, KIND>;
    constexpr int NC = FR::NC, FS = FR::FS;
    constexpr int KR = PREC == PL_F32_OFFSET ? 4 : 2;
    int *ctl = reinterpret_cast<int *>(smem_raw + lds_bytes - 16);
    const bool do_sums = flags & SF_SUMS;
    RunGeo G;
    G.T[0] = TS ? ts_dim(TS, 0) : I.tile[0];
    G.T[1] = TS ? ts_dim(TS, 1) : I.tile[1];
    G.T[2] = TS ? ts_dim(TS, 2) : I.tile[2];
    {
        int tx = t % I.ntile[0];
        int ty = (t / I.ntile[0]) % I.ntile[1];
        int tz = t / (I.ntile[0] * I.ntile[1]);
        G.lo[0] = tx * G.T[0];
        G.lo[1] = ty * G.T[1];
        G.lo[2] = tz * G.T[2];
    }
    G.hf = HF ? HF : ((flags & SF_FHALO2) ? 2 : 1);
    G.fx = G.T[0] + 2 * G.hf;
    G.fxy = G.fx * (G.T[1] + 2 * G.hf);
    G.Lf = G.fxy * (DIM >= 3 ? G.T[2] + 2 * G.hf : 1);
    G.dx = G.T[0] + 4;
    G.dxy = G.dx * (G.T[1] + 4);
    G.Ld = G.dxy * (DIM >= 3 ? G.T[2] + 4 : 1);
    const int pbeg = min(max(I.tile_start[t], 0), I.np);
    const int pend = min(max(I.tile_start[t + 1], pbeg), I.np);
    const int nruns = min(max(I.runs[I.np + t], 0), pend - pbeg);
    const int r_lo = (int)((long long)nruns * piece / npieces);
    const int r_hi = (int)((long long)nruns * (piece + 1) / npieces);
    if (r_hi <= r_lo) return;        // uniform: the whole block skips an empty piece

    UnitC<PREC> U;
    load_unit<PREC>(I, U, G.Ld);
    const int nslot = I.nslot;
    size_t offs[6];
    runs_lds_bytes<PREC, KIND>(G.Lf, G.Ld, nslot, G.hf, offs);
    RunShared<PREC> S;
    R *lds_f = reinterpret_cast<R *>(smem_raw + offs[0]);
    S.lds_f = lds_f;
    S.lds_d = reinterpret_cast<double *>(smem_raw + offs[1]);
    S.gq = reinterpret_cast<int *>(smem_raw + offs[2]);
    S.dq_c = reinterpret_cast<uint32_t *>(smem_raw + offs[3]);
    S.dq_d = reinterpret_cast<R *>(smem_raw + offs[4]);
    S.dq_mu = S.dq_d + 3 * RunsQ<PREC>::DQ;
    S.ctl = ctl;
    S.sums = reinterpret_cast<double *>(smem_raw + offs[5]);

    // stage the field records (hf-cell halo) and clear the deposit tile.
    // Float32 form: two-deep pipeline, a record's loads are issued before
    // the previous record is stored, and the first loads overlap the
    // clearing.
    {
        const int Ly = G.T[1] + 2 * G.hf;
        auto rec_cell = [&](int e) -> long {
            int lx = e % G.fx;
            int ly = (e / G.fx) % Ly;
            int lz = e / G.fxy;
            int gx = wrap_any(G.lo[0] + lx - G.hf, U.n[0]);
            int gy = DIM >= 2 ? wrap_any(G.lo[1] + ly - G.hf, U.n[1]) : 0;
            int gz = DIM >= 3 ? wrap_any(G.lo[2] + lz - G.hf, U.n[2]) : 0;
            return gx + (long)U.n[0] * (gy + (long)U.n[1] * gz);
        };
        auto rec_load = [&](int e, double (&v)[NC]) {
            const long gc = rec_cell(e);
#pragma unroll
            for (int q = 0; q < NC; ++q) v[q] = U.gf[q][gc];
        };
        // one 16-byte LDS store per 16 bytes of record (conflict-free:
        // consecutive threads write consecutive records)
        auto rec_store = [&](int e, const double (&v)[NC]) {
            if constexpr (FR::PLANES) {
                *reinterpret_cast<float4 *>(lds_f + FR::at(e, 0, G.Lf)) =
                    make_float4((R)v[0], (R)v[1], (R)v[2], 0.0f);
                *reinterpret_cast<float4 *>(lds_f + FR::at(e, 3, G.Lf)) =
                    make_float4((R)v[3], (R)v[4], (R)v[5], 0.0f);
            } else {
                R w[FS];
#pragma unroll
                for (int q = 0; q < FS; ++q) w[q] = q < NC ? (R)v[q] : R(0);
                if constexpr (PREC == PL_F32_OFFSET) {
                    *reinterpret_cast<float4 *>(lds_f + FS * e) = make_float4(w[0], w[1], w[2], w[3]);
                } else {
#pragma unroll
                    for (int k = 0; k < FS / 2; ++k)
                        *reinterpret_cast<double2 *>(lds_f + FS * e + 2 * k) = make_double2(w[2 * k], w[2 * k + 1]);
                }
            }
        };
        if constexpr (PREC == PL_F32_OFFSET) {
            double cur[NC];
            int e = threadIdx.x;
            if (e < G.Lf) rec_load(e, cur);
            for (int k = threadIdx.x; k < G.Ld * nslot; k += blockDim.x) S.lds_d[k] = 0.0;
            for (; e < G.Lf; e += blockDim.x) {
                double nxt[NC];
                const int en = e + (int)blockDim.x;
                if (en < G.Lf) rec_load(en, nxt);
                rec_store(e, cur);
#pragma unroll
                for (int q = 0; q < NC; ++q) cur[q] = nxt[q];
            }
        } else {
            // float64 records: one at a time (the pipeline's registers spill there)
            for (int e = threadIdx.x; e < G.Lf; e += blockDim.x) {
                double v[NC];
                rec_load(e, v);
                rec_store(e, v);
            }
            for (int k = threadIdx.x; k < G.Ld * nslot; k += blockDim.x) S.lds_d[k] = 0.0;
        }
        if (threadIdx.x == 0) {
            ctl[1] = 0;
            ctl[2] = 0;
        }
        if (threadIdx.x < 8) S.sums[threadIdx.x] = 0.0;
        __syncthreads();
    }

    // this thread's runs r = r_lo + tid, + blockDim, ..., each cut into
    // batches of KR; the next batch is fetched before the current one runs.
    // A long piece is taken in segments of 4 * blockDim runs with the LDS
    // queues drained between segments when half full; every piece ends
    // with a drain.  Segment count, drain decisions and barriers are
    // uniform across the block.  Pieces of one tile on several CUs meet
    // only in the global atomics of the flush.
    const gptr<const int32_t> runs = (gptr<const int32_t>)(I.runs + pbeg);
    auto run_span = [&](int r, int &rs, int &rl) {
        const int e = runs[r];
        rs = min(max(e >> 2, pbeg), pend - 1);
        rl = min((e & 3) + 1, pend - rs);
    };
    if constexpr (KIND == PL_TRACER) {
        // passive tracers deposit nothing: thread k advances the particles of
        // runs r_lo + k, + blockDim, ... on their own
        for (int r = r_lo + (int)threadIdx.x; r < r_hi; r += (int)blockDim.x) {
            int rs = 0, rl = 0;
            run_span(r, rs, rl);
            for (int q = 0; q < rl; ++q) tracer_particle<PREC, SHAPE, DIM>(U, G, S.lds_f, rs + q, err);
        }
    } else {
        const int seg = 4 * (int)blockDim.x;
        for (int s0 = r_lo; s0 < r_hi; s0 += seg) {
            const int s1 = min(r_hi, s0 + seg);
            int r = s0 + (int)threadIdx.x, b = 0, rs = 0, rl = 0;
            bool have = r < s1;
            BatchRaw<PREC, DIM, KR> cur;
            if (have) {
                run_span(r, rs, rl);
                fetch_batch<PREC, DIM, KR>(U, rs, min(KR, rl), cur);
            }
            while (have) {
                int nr = r, nb = b + KR, nrs = rs, nrl = rl;
                if (nb >= rl) {
                    nr = r + blockDim.x;
                    nb = 0;
                    if (nr < s1) run_span(nr, nrs, nrl);
                }
                const bool nhave = nr < s1;
                BatchRaw<PREC, DIM, KR> nxt;
                if (nhave) fetch_batch<PREC, DIM, KR>(U, nrs + nb, min(KR, nrl - nb), nxt);
                run_batch<PREC, SHAPE, DIM, KIND, CHS, KR>(U, G, S, cur, do_sums, err);
                cur = nxt;
                r = nr;
                b = nb;
                rs = nrs;
                rl = nrl;
                have = nhave;
            }
            __syncthreads();
            const int qg = ctl[1], qd = ctl[2];
            __syncthreads();          // all threads hold the same counts before anyone queues again
            if (s1 >= r_hi || 2 * qg > gq_cap(G.hf) || 2 * qd > RunsQ<PREC>::DQ) {
                const int ng = min(qg, gq_cap(G.hf));
                for (int i = threadIdx.x; i < ng; i += blockDim.x)
                    particle_single<PREC, SHAPE, DIM, KIND, CHS>(U, G, S, S.gq[i], do_sums, err);
                const int nd = min(qd, RunsQ<PREC>::DQ);
                for (int i = threadIdx.x; i < nd; i += blockDim.x) record_deposit<PREC, SHAPE, DIM, CHS>(U, G, S, i);
                __syncthreads();
                if (threadIdx.x == 0) {
                    ctl[1] = 0;
                    ctl[2] = 0;
                }
                __syncthreads();
            }
        }

        // flush the deposit tile: one float64 global atomic per touched cell
        // and channel.  The next unit is claimed first, so the claim's
        // round trip overlaps the flush.
        __syncthreads();
        if (threadIdx.x == 0) ctl[0] = (int)atomicAdd(counter + (blockIdx.x + ctl[3]) % kQueues, 1u);
        pre = true;
        if (do_sums && threadIdx.x < 8 && S.sums[threadIdx.x] != 0.0) global_add(I.psum + threadIdx.x, S.sums[threadIdx.x]);
        {
            const int Ly = G.T[1] + 4;
            for (int e = threadIdx.x; e < G.Ld; e += blockDim.x) {
                int lx = e % G.dx;
                int ly = (e / G.dx) % Ly;
                int lz = e / G.dxy;
                int gx = wrap_any(G.lo[0] + lx - 2, U.n[0]);
                int gy = DIM >= 2 ? wrap_any(G.lo[1] + ly - 2, U.n[1]) : 0;
                int gz = DIM >= 3 ? wrap_any(G.lo[2] + lz - 2, U.n[2]) : 0;
                long gc = gx + (long)U.n[0] * (gy + (long)U.n[1] * gz);
#pragma unroll
                for (int ch = 0; ch < kMaxCh; ++ch) {
                    const int so = ch_off<CHS>(U, ch, G.Ld);
                    if (so < 0) continue;
                    double val = S.lds_d[so + e];
                    if (val != 0.0) global_add(U.M[ch] + gc, val * U.inv_dv);
                }
            }
        }
    }
}

// Claim of the run kernels' next work unit.  The launch's unit slots are cut
// into kQueues contiguous chunks (neighbouring tiles share a chunk), each with
// its own counter; block b starts on chunk b % kQueues and moves to the next
// chunk when its own is exhausted (qi chunks passed, mirrored in ctl[3] for
// the claim issued before a flush).  Blocks are dispatched to the XCDs in
// turn, so the blocks of one XCD mostly share a chunk and find its field
// records in their L2; results do not depend on that placement.  The claim
// goes into ctl[0] (or was issued before the last flush, pre): false when
// every chunk is exhausted; otherwise the unit's item, tile and piece, with
// t = -1 for an empty or skipped slot.  Item k of the launch owns slots
// [unit_begin + k * kRunsSplit, + nunits + kRunsSplit); the sort lists an
// item's units largest first as (tile, piece | npieces << 16).
__device__ __forceinline__ int queue_lo(int q, int total) { return (int)((long long)total * q / kQueues); }

__device__ __forceinline__ bool runs_claim(const ItemDesc *__restrict__ items, int nitems, int total_units,
                                           unsigned *counter, int *errflags, int *ctl, bool &pre, int &qi, int &iti,
                                           int &t, int &piece, int &npieces)
{
    __syncthreads();
    if (!pre && threadIdx.x == 0 && qi < kQueues)
        ctl[0] = (int)atomicAdd(counter + (blockIdx.x + qi) % kQueues, 1u);
    __syncthreads();
    pre = false;
    t = -1;
    if (qi >= kQueues) return false;
    const int q = (int)((blockIdx.x + qi) % kQueues);
    const int qlo = queue_lo(q, total_units), qhi = queue_lo(q + 1, total_units);
    const int g = qlo + __builtin_amdgcn_readfirstlane(ctl[0]);
    if (g >= qhi) {
        // this chunk is exhausted: the next one
        ++qi;
        if (threadIdx.x == 0) ctl[3] = qi;
        return true;                                          // uniform
    }
    iti = 0;
    while (iti + 1 < nitems && items[iti + 1].unit_begin + (iti + 1) * kRunsSplit <= g) ++iti;
    const ItemDesc &I = items[iti];
    const int ubeg = I.unit_begin + iti * kRunsSplit;
    const int ucap = I.nunits + kRunsSplit;
    const int local = g - ubeg;
    const int nu = min(max(I.runs[runs_count_at(I.np, I.ntiles)], 0), I.nunits > 0 ? ucap : 0);
    // the sort's tables must cover the item's particles: tile offsets from
    // 0 to np and at least one unit when np > 0; otherwise the item was
    // never sorted (or its count changed since): latch it, leave it alone
    const bool stale = I.tile_start[0] != 0 || I.tile_start[I.ntiles] != I.np || (I.np > 0 && nu == 0);
    if (stale || local >= nu) {
        // the rest of this item's slots in the chunk are empty: move the
        // chunk's counter past them
        if (threadIdx.x == 0) {
            atomicMax(counter + q, (unsigned)(min(ubeg + ucap, qhi) - qlo));
            if (stale) atomicOr(errflags, (int)ERR_UNSORTED);
        }
        return true;                                          // uniform
    }
    const int32_t *unit = I.runs + runs_units_at(I.np, I.ntiles) + 2 * local;
    const int tt = unit[0];
    piece = unit[1] & 0xffff;
    npieces = unit[1] >> 16;
    if ((unsigned)tt >= (unsigned)I.ntiles || npieces < 1 || piece >= npieces) return true;      // uniform
    t = tt;
    return true;
}

// The last block to finish resets the chunk counters for the next launch.
__device__ __forceinline__ void release_queues(unsigned *counter)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        unsigned done = atomicAdd(counter + kQueues, 1u);
        if (done == gridDim.x - 1) {
            for (int q = 0; q < kQueues; ++q) atomicExch(counter + q, 0u);
            atomicExch(counter + kQueues, 0u);
        }
    }
}

__device__ __forceinline__ void runs_latch(int err, int *errflags)
{
    unsigned long long any = __ballot(err != 0);
    if (any) {
        int e = err;
        for (int off = 32; off > 0; off >>= 1) e |= __shfl_xor(e, off, 64);
        if ((threadIdx.x & 63) == 0) atomicOr(errflags, e);
    }
}

// HF: field halo width (1 or 2) fixed at compile time, or 0 to take it from
// the launch flags; TS and HF fixed make every LDS stencil offset an
// immediate.
template <int PREC, int SHAPE, int DIM, int KIND, int HF, int TS, int CHS>
__global__ __launch_bounds__(kRunsThreads) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_runs(const ItemDesc *__restrict__ items, int nitems, int total_units,
                                             unsigned *counter, int *errflags, unsigned flags, int lds_bytes)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    int *ctl = reinterpret_cast<int *>(smem_raw + lds_bytes - 16);
    int err = 0;
    bool pre = false;                      // uniform: ctl[0] already holds the next claim
    int qi = 0;                            // uniform: chunks passed
    if (threadIdx.x == 0) ctl[3] = 0;
    int iti = 0, t = -1, piece = 0, npieces = 1;
    while (runs_claim(items, nitems, total_units, counter, errflags, ctl, pre, qi, iti, t, piece, npieces)) {
        if (t < 0) continue;                                  // uniform
        runs_unit<PREC, SHAPE, DIM, KIND, HF, TS, CHS>(items[iti], t, piece, npieces, flags, lds_bytes, smem_raw,
                                                      counter, pre, err);
    }
    runs_latch(err, errflags);
    release_queues(counter);
}

// One persistent launch over the items of every species kind of a call: each
// claimed unit runs the unit body of its item's kind (uniform per block).
// CHL and CHD fix the channel sets of the charged (rho J F) and dust (rho F)
// items, or are 0 to take them at run time.
template <int PREC, int SHAPE, int DIM, int HF, int TS, int CHL, int CHD>
__global__ __launch_bounds__(kRunsThreads) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_runs_mix(const ItemDesc *__restrict__ items, int nitems, int total_units,
                                             unsigned *counter, int *errflags, unsigned flags, int lds_bytes)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    int *ctl = reinterpret_cast<int *>(smem_raw + lds_bytes - 16);
    int err = 0;
    bool pre = false;
    int qi = 0;
    if (threadIdx.x == 0) ctl[3] = 0;
    int iti = 0, t = -1, piece = 0, npieces = 1;
    while (runs_claim(items, nitems, total_units, counter, errflags, ctl, pre, qi, iti, t, piece, npieces)) {
        if (t < 0) continue;                                  // uniform
        const ItemDesc &I = items[iti];
        const int kind = __builtin_amdgcn_readfirstlane(I.kind);
        if (kind == PL_LORENTZ)
            runs_unit<PREC, SHAPE, DIM, PL_LORENTZ, HF, TS, CHL>(I, t, piece, npieces, flags, lds_bytes, smem_raw,
                                                                 counter, pre, err);
        else if (kind == PL_DUST)
            runs_unit<PREC, SHAPE, DIM, PL_DUST, HF, TS, CHD>(I, t, piece, npieces, flags, lds_bytes, smem_raw,
                                                              counter, pre, err);
        else
            runs_unit<PREC, SHAPE, DIM, PL_TRACER, HF, TS, 0>(I, t, piece, npieces, flags, lds_bytes, smem_raw,
                                                              counter, pre, err);
    }
    runs_latch(err, errflags);
    release_queues(counter);
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

template <int PREC>
static StepKernel pick_runs(int shape, int dim, int kind, int hf, int ts, int chs)
{
#define PL_R(S, D, K, HF_, TS_, CHS_) \
    if (shape == S && dim == D && kind == K && hf == HF_ && ts == TS_ && chs == CHS_) \
        return k_runs<PREC, S, D, K, HF_, TS_, CHS_>;
#define PL_RG(S, D) PL_R(S, D, PL_LORENTZ, 0, 0, 0) PL_R(S, D, PL_DUST, 0, 0, 0)
#define PL_RF(HF_, TS_) PL_R(PL_TSC, 3, PL_LORENTZ, HF_, TS_, 1) PL_R(PL_TSC, 3, PL_DUST, HF_, TS_, 2)
    PL_RG(PL_TSC, 3) PL_RG(PL_TSC, 2) PL_RG(PL_CIC, 3) PL_RG(PL_CIC, 2)
    PL_RF(1, 1) PL_RF(2, 1) PL_RF(1, 2) PL_RF(2, 2)
#undef PL_RF
#undef PL_RG
#undef PL_R
    return nullptr;
}

template <int PREC>
static StepKernel pick_runs_mix(int shape, int dim, int hf, int ts, int chl, int chd)
{
#define PL_M(S, D, HF_, TS_, CL, CD) \
    if (shape == S && dim == D && hf == HF_ && ts == TS_ && chl == CL && chd == CD) \
        return k_runs_mix<PREC, S, D, HF_, TS_, CL, CD>;
    PL_M(PL_TSC, 3, 0, 0, 0, 0) PL_M(PL_TSC, 2, 0, 0, 0, 0) PL_M(PL_CIC, 3, 0, 0, 0, 0) PL_M(PL_CIC, 2, 0, 0, 0, 0)
    PL_M(PL_TSC, 3, 1, 1, 1, 2) PL_M(PL_TSC, 3, 2, 1, 1, 2) PL_M(PL_TSC, 3, 1, 2, 1, 2) PL_M(PL_TSC, 3, 2, 2, 1, 2)
#undef PL_M
    return nullptr;
}

template <int PREC>
static size_t runs_item_lds(const Ctx *c, const ItemDesc &it, int hf)
{
    const int d3 = c->d.ndim >= 3;
    const int Lf = (it.tile[0] + 2 * hf) * (it.tile[1] + 2 * hf) * (d3 ? it.tile[2] + 2 * hf : 1);
    const int Ld = (it.tile[0] + 4) * (it.tile[1] + 4) * (d3 ? it.tile[2] + 4 : 1);
    size_t offs[6];
    if (it.kind == PL_LORENTZ) return runs_lds_bytes<PREC, PL_LORENTZ>(Lf, Ld, it.nslot, hf, offs);
    if (it.kind == PL_DUST) return runs_lds_bytes<PREC, PL_DUST>(Lf, Ld, it.nslot, hf, offs);
    return runs_lds_bytes<PREC, PL_TRACER>(Lf, Ld, 0, hf, offs);
}

// Launch configuration of the run kernel for the items of one launch.
template <int PREC>
bool runs_plan_impl(const Ctx *c, const ItemDesc *host, int nitems, RunsPlan &pl)
{
    pl = RunsPlan{};
    if (nitems < 1) return false;
    bool kinds[3] = {false, false, false};
    for (int i = 0; i < nitems; ++i) kinds[host[i].kind] = true;
    pl.mixed = kinds[PL_TRACER] || (kinds[PL_LORENTZ] && kinds[PL_DUST]);
    // compile-time tile shape (8^3 or 8x8x4) and channel sets when every item
    // allows them: charged rho J F, dust rho F
    if (c->d.shape == PL_TSC && c->d.ndim == 3) {
        bool chall = true;
        for (int i = 0; i < nitems && chall; ++i) {
            const int want = host[i].kind == PL_LORENTZ ? 1 : (host[i].kind == PL_DUST ? 2 : 0);
            for (int ch = 0; ch < kMaxCh && want; ++ch) chall = chall && host[i].slot[ch] == chs_slot(want, ch);
        }
        for (int cand = 1; cand <= 2 && pl.ts == 0 && chall; ++cand) {
            bool all = true;
            for (int i = 0; i < nitems; ++i)
                for (int a = 0; a < 3; ++a) all = all && host[i].tile[a] == ts_dim(cand, a);
            if (all) pl.ts = cand;
        }
    }
    if (pl.ts) {
        pl.chl = 1;
        pl.chd = 2;
    }
    // LDS of the launch: a two-cell field halo when it fits, else one cell
    for (int hf = 2; hf >= 1; --hf) {
        size_t lds = 0;
        for (int i = 0; i < nitems; ++i) lds = std::max(lds, runs_item_lds<PREC>(c, host[i], hf));
        if (lds <= (size_t)c->lds_max) {
            pl.hf = hf;
            pl.lds = lds;
            return true;
        }
    }
    return false;
}

template <int PREC>
hipError_t launch_runs_impl(Ctx *c, const ItemDesc *table, const ItemDesc *host, int nitems, int total_units,
                            unsigned sf, unsigned *counter)
{
    if (total_units <= 0) return hipSuccess;
    RunsPlan pl;
    if (!runs_plan_impl<PREC>(c, host, nitems, pl)) return hipErrorInvalidConfiguration;
    if (pl.hf == 2) sf |= SF_FHALO2;
    StepKernel k;
    int chs = 0;
    if (pl.mixed) {
        // compile-time halo in the fixed-shape kernels, from the flags otherwise
        k = pick_runs_mix<PREC>(c->d.shape, c->d.ndim, pl.ts ? pl.hf : 0, pl.ts, pl.chl, pl.chd);
        chs = pl.chl;
    } else {
        const int kind = host[0].kind;
        chs = pl.ts ? (kind == PL_LORENTZ ? pl.chl : pl.chd) : 0;
        k = pick_runs<PREC>(c->d.shape, c->d.ndim, kind, pl.ts ? pl.hf : 0, pl.ts, chs);
    }
    if (!k) return hipErrorInvalidConfiguration;
    const int rb = kRunsThreads;
    // every item has kRunsSplit units beyond its tiles for the pieces of crowded tiles
    const int units = total_units + nitems * kRunsSplit;
    int grid = std::min(units, resident_blocks(c, k, rb, pl.lds));
    hipLaunchKernelGGL(k, dim3(grid), dim3(rb), pl.lds, c->stream, table, nitems, units, counter, c->errflags, sf,
                       (int)pl.lds);
    c->stats[0]++;
    c->stats[4]++;
    if (pl.ts) c->stats[6]++;
    c->stats[7] = pl.ts | chs << 4 | pl.hf << 8 | (pl.mixed ? 1 << 12 : 0);
    return hipGetLastError();
}

}  // namespace pl
