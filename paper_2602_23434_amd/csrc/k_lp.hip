// Lagrangian-particle extras for gfx950: the spectral update of every
// particle's energy distribution (Sec. 2), and deletion at open boundaries
// with the holes-and-fillers compaction and injection (Sec. 3.2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "pl_device.h"

namespace pl {

// ---------------------------------------------------------------------------
// Spectral update
// ---------------------------------------------------------------------------

constexpr int kSpecThreads = 256;     // particles per block, and threads
constexpr int kSpecUnroll = 4;        // spectral values in flight per thread and array

struct SpecPar {
    double cr, u_rad, ub, inv_c2;
};

// The spectral rows are read and written once per step with non-temporal
// accesses, so they do not displace the fields the sampling reads.

// Cell and float64 offset from the cell centre of particle p, per dimension.
template <int PREC, int DIM>
__device__ __forceinline__ void locate_f64(const ItemDesc &I, int p, int c[3], double d[3], int &err)
{
    if constexpr (PREC == PL_F64) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            c[a] = 0;
            d[a] = 0.0;
            if (a >= DIM) continue;
            double v = static_cast<const double *>(I.x[a])[p];
            const double n = (double)I.n[a];
            if (!(v >= 0.0 && v < n)) {
                if (!isfinite(v)) { err |= ERR_NONFINITE; v = 0.0; }
                v = v - n * floor(v / n);
                if (!(v >= 0.0 && v < n)) v = 0.0;
            }
            const double f = floor(v);
            c[a] = (int)f;
            d[a] = v - f - 0.5;
        }
    } else {
        int ijk[3];
        unpack_cell(I.cell[p], ijk[0], ijk[1], ijk[2]);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            c[a] = 0;
            d[a] = 0.0;
            if (a >= DIM) continue;
            int ci = ijk[a];
            if (ci >= I.n[a]) { err |= ERR_NONFINITE; ci %= I.n[a]; }
            float o = static_cast<const float *>(I.x[a])[p];
            if (!(o >= -0.5f && o < 0.5f)) { err |= ERR_NONFINITE; o = 0.0f; }
            c[a] = ci;
            d[a] = (double)o;
        }
    }
}

// B (3), gas velocity (3) and four-divergence at a particle, float64, with
// the box's CIC/TSC weights (the gather's weights, evaluated in float64).
template <int PREC, int SHAPE, int DIM>
__device__ __forceinline__ void sample_fluid(const ItemDesc &I, int p, double q[7], int &err)
{
    int c[3];
    double d[3];
    locate_f64<PREC, DIM>(I, p, c, d, err);
    double w[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (a < DIM) {
            weights3<SHAPE, double>(d[a], w[a]);
        } else {
            w[a][0] = 0.0;
            w[a][1] = 1.0;
            w[a][2] = 0.0;
        }
    }
    const gptr<const double> f[7] = {(gptr<const double>)I.B[0],  (gptr<const double>)I.B[1],
                                     (gptr<const double>)I.B[2],  (gptr<const double>)I.vg[0],
                                     (gptr<const double>)I.vg[1], (gptr<const double>)I.vg[2],
                                     (gptr<const double>)I.divu};
#pragma unroll
    for (int m = 0; m < 7; ++m) q[m] = 0.0;
    constexpr int SZ = DIM >= 3 ? 3 : 1, SY = DIM >= 2 ? 3 : 1;
    // one stencil row (three x-neighbours, 21 loads) in flight at a time:
    // unrolled further the loads would take the registers the streaming
    // of the spectral rows needs
#pragma unroll 1
    for (int k = 0; k < SZ; ++k) {
        const int gz = DIM >= 3 ? wrap_cell(c[2] + k - 1, I.n[2]) : 0;
#pragma unroll 1
        for (int j = 0; j < SY; ++j) {
            const int gy = DIM >= 2 ? wrap_cell(c[1] + j - 1, I.n[1]) : 0;
            const double wyz = w[2][DIM >= 3 ? k : 1] * w[1][DIM >= 2 ? j : 1];
            const long row = (long)I.n[0] * (gy + (long)I.n[1] * gz);
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const long gc = row + wrap_cell(c[0] + i - 1, I.n[0]);
                const double wt = wyz * w[0][i];
#pragma unroll
                for (int m = 0; m < 7; ++m) q[m] = fma(wt, f[m][gc], q[m]);
            }
        }
    }
}

// W consecutive spectral values of one row (W = 2: one 16-byte access).
template <int W> struct SpecVec;
template <> struct SpecVec<1> {
    typedef double T;
    __device__ static double get(T v, int) { return v; }
    __device__ static void set(T &v, int, double x) { v = x; }
};
template <> struct SpecVec<2> {
    typedef double T __attribute__((ext_vector_type(2)));
    __device__ static double get(T v, int k) { return v[k]; }
    __device__ static void set(T &v, int k, double x) { v[k] = x; }
};

// The block's rows, streamed: access a = pass * 256 + threadIdx.x covers
// values [W a, W a + W) of the rows (all in one row, nb being a multiple of
// W); kSpecUnroll passes are loaded together, and the next group's loads are
// issued before the current group is updated and stored.  The first group
// is loaded by the caller before the fluid sampling, so the block's HBM
// traffic starts at once.
template <int W>
struct SpecStream {
    using V = SpecVec<W>;
    using T = typename V::T;
    typedef __attribute__((address_space(1))) T *P;
    P eng, chi;
    long naccess;                     // accesses of the block: cnt * nb / W
    int nb;
    T ev[kSpecUnroll], cv[kSpecUnroll];
    int rr[kSpecUnroll];
    int row, col;                     // row and first column of this thread's next access

    __device__ void init(gptr<double> e, gptr<double> c, int cnt, int nb_)
    {
        eng = (P)e;
        chi = (P)c;
        nb = nb_;
        naccess = (long)cnt * nb / W;
        const int v = threadIdx.x * W;
        row = v / nb;
        col = v % nb;
    }

    // load the group of passes starting at access a0 (this thread's first)
    __device__ __forceinline__ void load(long a0)
    {
        constexpr int step = kSpecThreads * W;
        const int srow = step / nb, scol = step % nb;
#pragma unroll
        for (int k = 0; k < kSpecUnroll; ++k) {
            const long a = a0 + (long)k * kSpecThreads;
            rr[k] = row;
            if (a < naccess) {
                ev[k] = __builtin_nontemporal_load(eng + a);
                cv[k] = __builtin_nontemporal_load(chi + a);
            }
            row += srow;
            col += scol;
            if (col >= nb) { col -= nb; ++row; }
        }
    }

    __device__ __forceinline__ void update(long a0, const double *sE, const double *siE, const double *sb)
    {
#pragma unroll
        for (int k = 0; k < kSpecUnroll; ++k) {
            const long a = a0 + (long)k * kSpecThreads;
            if (a < naccess) {
                const double E = sE[rr[k]], iE = siE[rr[k]], b = sb[rr[k]];
                T eo, co;
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    const double e0 = V::get(ev[k], w);
                    const double den = 1.0 + b * e0;
                    V::set(eo, w, e0 * E / den);
                    V::set(co, w, V::get(cv[k], w) * den * den * iE);
                }
                __builtin_nontemporal_store(eo, eng + a);
                __builtin_nontemporal_store(co, chi + a);
            }
        }
    }
};

template <int W>
__device__ __forceinline__ void spectra_rows(SpecStream<W> &S, const double *sE, const double *siE,
                                             const double *sb)
{
    constexpr long group = (long)kSpecThreads * kSpecUnroll;
    for (long a0 = threadIdx.x; a0 < S.naccess; a0 += group) {
        // the next group's loads go out before this group's update
        SpecStream<W> nxt = S;
        const bool more = a0 + group < S.naccess;
        if (more) nxt.load(a0 + group);
        S.update(a0, sE, siE, sb);
        if (more) {
            S = nxt;
        }
    }
}

// Coefficients of one particle's step: E = exp(-a d tau), 1/E and
// c_r phi; the identity (1, 1, 0) when the gas moves at c or faster.
template <int PREC, int SHAPE, int DIM>
__device__ __forceinline__ void spectra_coef(const ItemDesc &I, int p, const SpecPar &sp, double &E, double &iE,
                                             double &bphi, int &err)
{
    double q[7];
    sample_fluid<PREC, SHAPE, DIM>(I, p, q, err);
    const double v2 = fma(q[3], q[3], fma(q[4], q[4], q[5] * q[5])) * sp.inv_c2;
    const double b2 = fma(q[0], q[0], fma(q[1], q[1], q[2] * q[2]));
    E = 1.0;
    iE = 1.0;
    bphi = 0.0;
    if (!(v2 < 1.0)) {
        err |= ERR_NONFINITE;
        return;
    }
    const double dtau = I.dt * sqrt(1.0 - v2);      // d tau = dt / gamma_g
    const double a = q[6] / 3.0;
    const double b = sp.cr * fma(sp.ub, b2, sp.u_rad);
    E = exp(-a * dtau);
    iE = 1.0 / E;
    const double phi = a != 0.0 ? -expm1(-a * dtau) / a : dtau;
    bphi = b * phi;
}

// One block per 256 particles of one item: each thread samples the fluid at
// its particle and leaves the step's coefficients in LDS; the block then
// streams its 256 contiguous spectral rows (particle-major).
template <int PREC, int SHAPE, int DIM, int W>
__device__ __forceinline__ void spectra_block(const ItemDesc &I, int p0, int cnt, const SpecPar &sp, double *sE,
                                              double *siE, double *sb, int &err)
{
    SpecStream<W> S;
    S.init((gptr<double>)I.eng + (long)p0 * I.nb, (gptr<double>)I.chi + (long)p0 * I.nb, cnt, I.nb);
    S.load(threadIdx.x);
    {
        const int t = threadIdx.x;
        double E = 1.0, iE = 1.0, bphi = 0.0;
        if (t < cnt) spectra_coef<PREC, SHAPE, DIM>(I, p0 + t, sp, E, iE, bphi, err);
        sE[t] = E;
        siE[t] = iE;
        sb[t] = bphi;
    }
    __syncthreads();
    spectra_rows<W>(S, sE, siE, sb);
}

template <int PREC, int SHAPE, int DIM>
__global__ __launch_bounds__(kSpecThreads) void k_spectra(const ItemDesc *__restrict__ items, int nitems, SpecPar sp,
                                                          int *errflags)
{
    __shared__ double s_E[kSpecThreads], s_iE[kSpecThreads], s_b[kSpecThreads];
    const int g = blockIdx.x;
    int iti = 0;
    while (iti + 1 < nitems && items[iti + 1].unit_begin <= g) ++iti;
    const ItemDesc &I = items[iti];
    const int p0 = (g - I.unit_begin) * kSpecThreads;
    if (p0 >= I.np || I.nb <= 0) return;                  // uniform
    const int cnt = min(kSpecThreads, I.np - p0);
    int err = 0;
    if ((I.nb & 1) == 0) spectra_block<PREC, SHAPE, DIM, 2>(I, p0, cnt, sp, s_E, s_iE, s_b, err);
    else spectra_block<PREC, SHAPE, DIM, 1>(I, p0, cnt, sp, s_E, s_iE, s_b, err);
    if (err) atomicOr(errflags, err);
}

hipError_t launch_spectra(Ctx *c, const ItemDesc *table, const std::vector<ItemDesc> &host, double cr,
                          double u_rad, double ub)
{
    int units = 0;
    for (const ItemDesc &it : host) units = std::max(units, it.unit_begin + it.nunits);
    if (units == 0) return hipSuccess;
    SpecPar sp{cr, u_rad, ub, c->d.c > 0.0 ? 1.0 / (c->d.c * c->d.c) : 0.0};
    using K = void (*)(const ItemDesc *, int, SpecPar, int *);
    K k = nullptr;
    const bool f64 = c->d.prec == PL_F64, tsc = c->d.shape == PL_TSC, d3 = c->d.ndim == 3;
#define PL_SK(P, S, D) \
    if ((P == PL_F64) == f64 && (S == PL_TSC) == tsc && (D == 3) == d3) k = k_spectra<P, S, D>;
    PL_SK(PL_F64, PL_TSC, 3) PL_SK(PL_F64, PL_TSC, 2) PL_SK(PL_F64, PL_CIC, 3) PL_SK(PL_F64, PL_CIC, 2)
    PL_SK(PL_F32_OFFSET, PL_TSC, 3) PL_SK(PL_F32_OFFSET, PL_TSC, 2) PL_SK(PL_F32_OFFSET, PL_CIC, 3)
    PL_SK(PL_F32_OFFSET, PL_CIC, 2)
#undef PL_SK
    if (!k) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k, dim3(units), dim3(kSpecThreads), 0, c->stream, table, (int)host.size(), sp, c->errflags);
    c->stats[0]++;
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Deletion at open boundaries and compaction (holes and fillers)
// ---------------------------------------------------------------------------

constexpr int kBndThreads = 256;
constexpr int kBndPer = 8;                          // consecutive particles per thread
constexpr int kBndBlock = kBndThreads * kBndPer;    // particles per block

struct BndArgs {
    int np, nblk;
    int open[3], ghost, n[3];
    int prec, ndim;
    const uint32_t *cell;
    const void *x[3];
};

// Arrays moved together by the compaction (element sizes 4 or 8).
struct MoveArrays {
    static constexpr int kMax = 10;
    void *a[kMax];
    int wide;                       // bit k: array k has 8-byte elements
    int n;
};

__device__ __forceinline__ bool outside_cell(const BndArgs &A, int p)
{
    int c[3] = {0, 0, 0};
    if (A.prec == PL_F32_OFFSET) {
        unpack_cell(A.cell[p], c[0], c[1], c[2]);
    } else {
        for (int d = 0; d < A.ndim; ++d) {
            const double v = static_cast<const double *>(A.x[d])[p];
            c[d] = isfinite(v) ? (int)floor(v) : -1;
        }
    }
    bool out = false;
    for (int d = 0; d < A.ndim; ++d)
        if (A.open[d]) out = out || c[d] < A.ghost || c[d] >= A.n[d] - A.ghost;
    return out;
}

// 1. flags, one word per particle, and the flagged count of every block
__global__ __launch_bounds__(kBndThreads) void k_bnd_flag(BndArgs A, uint32_t *flags, uint32_t *blkcnt)
{
    __shared__ uint32_t s_cnt;
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    const int b0 = blockIdx.x * kBndBlock;
    uint32_t mine = 0;
    for (int k = 0; k < kBndPer; ++k) {
        const int p = b0 + k * kBndThreads + threadIdx.x;
        if (p < A.np) {
            const uint32_t f = outside_cell(A, p) ? 1u : 0u;
            flags[p] = f;
            mine += f;
        }
    }
    mine = wave_sum(mine);
    if ((threadIdx.x & 63) == 0 && mine) atomicAdd(&s_cnt, mine);
    __syncthreads();
    if (threadIdx.x == 0) blkcnt[blockIdx.x] = s_cnt;
}

// 2. exclusive scan of the block counts (one block): offs[0..nblk], and the
// totals tot[0] = ndel, tot[1] = keep = np - ndel
__global__ __launch_bounds__(1024) void k_bnd_scan(const uint32_t *blkcnt, int nblk, int np, uint32_t *offs,
                                                   int64_t *tot)
{
    __shared__ uint32_t s_w[16];
    __shared__ uint32_t s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int c0 = 0; c0 < nblk; c0 += 1024) {
        const int i = c0 + threadIdx.x;
        const uint32_t v = i < nblk ? blkcnt[i] : 0u;
        uint32_t x = v;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        if (lane == 63) s_w[wv] = x;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t run = 0;
            for (int k = 0; k < 16; ++k) {
                const uint32_t t = s_w[k];
                s_w[k] = run;
                run += t;
            }
        }
        __syncthreads();
        const uint32_t carry = s_carry;
        if (i < nblk) offs[i] = carry + s_w[wv] + x - v;
        __syncthreads();
        if (threadIdx.x == 1023) s_carry = carry + s_w[wv] + x;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        offs[nblk] = s_carry;
        tot[0] = (int64_t)s_carry;
        tot[1] = (int64_t)np - (int64_t)s_carry;
    }
}

// 3. holes below keep: tot[2] = number of flagged particles in [0, keep)
__global__ __launch_bounds__(kBndThreads) void k_bnd_holes(const uint32_t *flags, const uint32_t *offs, int64_t *tot)
{
    __shared__ uint32_t s_cnt;
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    const int keep = (int)tot[1];
    const int b = keep / kBndBlock;
    uint32_t mine = 0;
    for (int p = b * kBndBlock + threadIdx.x; p < keep; p += kBndThreads) mine += flags[p];
    mine = wave_sum(mine);
    if ((threadIdx.x & 63) == 0 && mine) atomicAdd(&s_cnt, mine);
    __syncthreads();
    if (threadIdx.x == 0) tot[2] = (int64_t)offs[b] + s_cnt;
}

// 4. hole and filler lists in index order.  With F(p) the flagged count in
// [0, p): a flagged particle below keep is hole F(p); a survivor at or above
// keep is filler (p - keep) - (F(p) - nholes).
__global__ __launch_bounds__(kBndThreads) void k_bnd_lists(const uint32_t *flags, const uint32_t *offs, int np,
                                                           const int64_t *tot, uint32_t *holes, uint32_t *fillers)
{
    __shared__ uint32_t s_w[kBndThreads / 64 + 1];
    const int keep = (int)tot[1];
    const int nholes = (int)tot[2];
    const int p0 = blockIdx.x * kBndBlock + threadIdx.x * kBndPer;
    uint32_t f[kBndPer];
    uint32_t mine = 0;
#pragma unroll
    for (int k = 0; k < kBndPer; ++k) {
        f[k] = (p0 + k < np) ? flags[p0 + k] : 0u;
        mine += f[k];
    }
    // exclusive prefix of `mine` over the block's threads
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t x = mine;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) s_w[wv] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int k = 0; k < kBndThreads / 64; ++k) {
            const uint32_t t = s_w[k];
            s_w[k] = run;
            run += t;
        }
    }
    __syncthreads();
    uint32_t F = offs[blockIdx.x] + s_w[wv] + x - mine;
#pragma unroll
    for (int k = 0; k < kBndPer; ++k) {
        const int p = p0 + k;
        if (p < np) {
            if (f[k] && p < keep) holes[F] = (uint32_t)p;
            else if (!f[k] && p >= keep) fillers[(p - keep) - ((int)F - nholes)] = (uint32_t)p;
        }
        F += f[k];
    }
}

// 5. move every array of filler k into hole k
__global__ void k_bnd_move(MoveArrays M, const uint32_t *holes, const uint32_t *fillers, const int64_t *tot)
{
    const int nh = (int)tot[2];
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nh; k += gridDim.x * blockDim.x) {
        const uint32_t h = holes[k], s = fillers[k];
        for (int a = 0; a < M.n; ++a) {
            if (M.wide & (1 << a)) {
                uint64_t *v = static_cast<uint64_t *>(M.a[a]);
                v[h] = v[s];
            } else {
                uint32_t *v = static_cast<uint32_t *>(M.a[a]);
                v[h] = v[s];
            }
        }
    }
}

// spectral rows: one wave per moved particle
__global__ __launch_bounds__(256) void k_bnd_move_rows(double *eng, double *chi, int nb, const uint32_t *holes,
                                                       const uint32_t *fillers, const int64_t *tot)
{
    const int nh = (int)tot[2];
    const int lane = threadIdx.x & 63;
    for (int k = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; k < nh; k += (gridDim.x * blockDim.x) >> 6) {
        const long h = (long)holes[k] * nb, s = (long)fillers[k] * nb;
        for (int i = lane; i < nb; i += 64) {
            eng[h + i] = eng[s + i];
            chi[h + i] = chi[s + i];
        }
    }
}

// 6. an item that lost particles must be sorted again
__global__ void k_bnd_mark(int32_t *tile_start, const int64_t *tot)
{
    if (threadIdx.x == 0 && tot[0] > 0) tile_start[0] = -1;
}

hipError_t launch_boundary(Ctx *c, const ItemDesc &it, const pl_boundary_desc &bc, int ndim, int64_t *keep,
                           int64_t *removed)
{
    *keep = it.np;
    *removed = 0;
    if (it.np == 0) return hipSuccess;
    hipStream_t s = c->stream;
    BndArgs A;
    A.np = it.np;
    A.nblk = (it.np + kBndBlock - 1) / kBndBlock;
    A.ghost = bc.ghost;
    A.prec = c->d.prec;
    A.ndim = ndim;
    A.cell = it.cell;
    for (int d = 0; d < 3; ++d) {
        A.open[d] = d < ndim ? bc.open[d] != 0 : 0;
        A.n[d] = it.n[d];
        A.x[d] = it.x[d];
    }
    // scratch: flags in keys[0], holes in idx[0], fillers in idx[1], block
    // counts in hist, their scan and the totals in hist_scan
    if ((int64_t)A.nblk + 1 + 16 > c->hist_cap) return hipErrorInvalidValue;
    uint32_t *flags = c->keys[0];
    uint32_t *blk = c->hist;
    uint32_t *offs = c->hist_scan;
    int64_t *tot = reinterpret_cast<int64_t *>(c->hist_scan + ((c->hist_cap - 8) & ~(int64_t)1));
    hipLaunchKernelGGL(k_bnd_flag, dim3(A.nblk), dim3(kBndThreads), 0, s, A, flags, blk);
    hipLaunchKernelGGL(k_bnd_scan, dim3(1), dim3(1024), 0, s, blk, A.nblk, A.np, offs, tot);
    hipLaunchKernelGGL(k_bnd_holes, dim3(1), dim3(kBndThreads), 0, s, flags, offs, tot);
    hipLaunchKernelGGL(k_bnd_lists, dim3(A.nblk), dim3(kBndThreads), 0, s, flags, offs, A.np, tot, c->idx[0],
                       c->idx[1]);
    MoveArrays M;
    M.n = 0;
    M.wide = 0;
    const bool f64 = c->d.prec == PL_F64;
    auto add = [&](void *p, bool wide) {
        if (!p) return;
        if (wide) M.wide |= 1 << M.n;
        M.a[M.n++] = p;
    };
    if (!f64) add(it.cell, false);
    for (int d = 0; d < ndim; ++d) add(it.x[d], f64);
    for (int d = 0; d < 3; ++d) add(it.u[d], f64);
    add(it.w, f64);
    add(it.id, true);
    const int grid = std::min((it.np + 255) / 256, 16 * c->num_cu);
    hipLaunchKernelGGL(k_bnd_move, dim3(grid), dim3(256), 0, s, M, c->idx[0], c->idx[1], tot);
    if (it.nb > 0 && it.eng && it.chi)
        hipLaunchKernelGGL(k_bnd_move_rows, dim3(std::max(1, std::min(it.np / 4 + 1, 64 * c->num_cu))), dim3(256), 0,
                           s, it.eng, it.chi, it.nb, c->idx[0], c->idx[1], tot);
    if (it.tile_start) hipLaunchKernelGGL(k_bnd_mark, dim3(1), dim3(64), 0, s, it.tile_start, tot);
    c->stats[0] += 6 + (it.nb > 0) + (it.tile_start != nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int64_t h[2] = {0, 0};
    e = hipMemcpyAsync(h, tot, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    *removed = h[0];
    *keep = h[1];
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// Injection: weights, ids and spectral rows of appended particles
// ---------------------------------------------------------------------------

template <typename R>
__global__ void k_inj_w(R *dst, const double *src, double wdef, int64_t k)
{
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < k; j += (int64_t)gridDim.x * blockDim.x)
        dst[j] = (R)(src ? src[j] : wdef);
}

__global__ void k_inj_id(uint64_t *dst, const uint64_t *src, int64_t first, int64_t k)
{
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < k; j += (int64_t)gridDim.x * blockDim.x)
        dst[j] = src ? src[j] : (uint64_t)(first + j);
}

__global__ void k_inj_rows(double *dst, const double *src, int64_t m)
{
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < m; j += (int64_t)gridDim.x * blockDim.x)
        dst[j] = src[j];
}

__global__ void k_inj_mark(int32_t *tile_start)
{
    if (threadIdx.x == 0) tile_start[0] = -1;
}

hipError_t launch_inject_rest(Ctx *c, const ItemDesc &it, int64_t k, const double *w, bool has_w, double wdef,
                              const uint64_t *id, uint64_t *id_dst, const double *eng, const double *chi)
{
    if (k <= 0) return hipSuccess;
    hipStream_t s = c->stream;
    const int grid = (int)std::min<int64_t>((k + 255) / 256, 16 * c->num_cu);
    const int64_t n = it.np;
    if (has_w) {
        if (c->d.prec == PL_F64)
            hipLaunchKernelGGL(k_inj_w<double>, dim3(grid), dim3(256), 0, s, static_cast<double *>(it.w) + n, w,
                               wdef, k);
        else
            hipLaunchKernelGGL(k_inj_w<float>, dim3(grid), dim3(256), 0, s, static_cast<float *>(it.w) + n, w, wdef,
                               k);
        c->stats[0]++;
    }
    if (id_dst) {
        hipLaunchKernelGGL(k_inj_id, dim3(grid), dim3(256), 0, s, id_dst + n, id, n, k);
        c->stats[0]++;
    }
    if (it.nb > 0 && it.eng && it.chi) {
        const int64_t m = k * it.nb;
        const int g2 = (int)std::min<int64_t>((m + 255) / 256, 64 * c->num_cu);
        hipLaunchKernelGGL(k_inj_rows, dim3(g2), dim3(256), 0, s, it.eng + n * it.nb, eng, m);
        hipLaunchKernelGGL(k_inj_rows, dim3(g2), dim3(256), 0, s, it.chi + n * it.nb, chi, m);
        c->stats[0] += 2;
    }
    if (it.tile_start) {
        hipLaunchKernelGGL(k_inj_mark, dim3(1), dim3(64), 0, s, it.tile_start);
        c->stats[0]++;
    }
    return hipGetLastError();
}

}  // namespace pl
