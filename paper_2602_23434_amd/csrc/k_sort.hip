// Stable cell-tile sort for gfx950.
//
// key(p) = tile of the particle's cell, or tile * cells_per_tile + cell in
// tile, or (rank-interleaved) tile, rank of the particle among the particles
// of its cell, cell in tile.  The permutation is the stable one (ties keep their order), built by
// least-significant-digit radix sort on (key, source index) pairs with 8-bit
// digits: per pass a digit histogram per block, an exclusive scan in
// digit-major order, and a scatter in which every wave ranks its 64 elements
// by digit with ballots (so equal digits keep their order) and the block's
// waves take consecutive sub-ranges.  The final index list moves every SoA
// array into the alternate buffer set, and a boundary pass writes the
// first-particle offset of every tile.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "pl_device.h"

namespace pl {

constexpr int kSortWaves = 8;
constexpr int kSortThreads = kSortWaves * 64;
constexpr int kPerWave = 1024;                       // elements per wave per block
constexpr int kPerBlock = kSortWaves * kPerWave;     // elements per block
constexpr int kScanBlocks = 512;

// Digit counts of the 64 keys from e0 (those below end) added to cnt: the
// first lane of every run of equal digits adds the run's length.  All lanes
// of the wave take part.
__device__ __forceinline__ void count_runs(const uint32_t *keys, int e0, int end, int shift, uint32_t mask,
                                           uint32_t *cnt)
{
    const int lane = threadIdx.x & 63;
    const int e = e0 + lane;
    const bool v = e < end;
    const uint32_t d = v ? (keys[e] >> shift) & mask : ~0u;
    const uint32_t prev = __shfl_up(d, 1, 64);
    const bool head = v && (lane == 0 || prev != d);
    const uint64_t hm = __ballot(head);
    if (head) {
        const uint64_t later = hm & ~((2ull << lane) - 1ull);     // heads after this lane
        const int stop = later ? __builtin_ctzll(later) : min(64, end - e0);
        atomicAdd(&cnt[d], (uint32_t)(stop - lane));
    }
}

__global__ void k_keys(SortArgs a, uint32_t *keys)
{
    const int tx = a.tile[0], ty = a.tile[1], tz = a.tile[2];
    const int ntx = a.n[0] / tx, nty = a.n[1] / ty;
    const int per_tile = tx * ty * tz;
    const bool p2 = ((tx & (tx - 1)) | (ty & (ty - 1)) | (tz & (tz - 1))) == 0;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < a.np; p += gridDim.x * blockDim.x) {
        int c[3] = {0, 0, 0};
        if (a.prec == PL_F32_OFFSET) {
            unpack_cell(a.cell[p], c[0], c[1], c[2]);
            for (int d = 0; d < 3; ++d)
                if (c[d] >= a.n[d]) c[d] %= a.n[d];
        } else {
            for (int d = 0; d < a.ndim; ++d) {
                double v = a.x[d][p];
                double nn = (double)a.n[d];
                if (!(v >= 0.0 && v < nn)) {
                    if (!isfinite(v)) v = 0.0;
                    v = v - nn * floor(v / nn);
                    if (v >= nn || v < 0.0) v = 0.0;
                }
                c[d] = (int)floor(v);
            }
        }
        // power-of-two tile sides (the usual case) divide by shifts
        int q[3], r[3];
        const int td[3] = {tx, ty, tz};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            if (p2) {
                const int lg = __builtin_ctz((unsigned)td[d]);
                q[d] = c[d] >> lg;
                r[d] = c[d] & (td[d] - 1);
            } else {
                q[d] = c[d] / td[d];
                r[d] = c[d] % td[d];
            }
        }
        int t = q[0] + ntx * (q[1] + nty * q[2]);
        uint32_t key = (uint32_t)t;
        if (a.key_mode == PL_KEY_TILE_CELL || a.key_mode == PL_KEY_TILE_RUN) {
            int yy = r[1];
            // run order: rows taken as 0, 2, 4, 6, 1, 3, 5, 7 within every group
            // of eight (0, 2, 1, 3 within groups of four), so that the lanes
            // served together by one LDS access hold rows of one parity and
            // their records and deposit cells fall on distinct banks
            if (a.key_mode == PL_KEY_TILE_RUN && (ty & 7) == 0)
                yy = (yy & ~7) | ((yy & 1) << 2) | ((yy >> 1) & 3);
            else if (a.key_mode == PL_KEY_TILE_RUN && (ty & 3) == 0)
                yy = (yy & ~3) | ((yy & 1) << 1) | ((yy >> 1) & 1);
            int loc = r[0] + tx * (yy + ty * r[2]);
            key = (uint32_t)t * (uint32_t)per_tile + (uint32_t)loc;
        }
        keys[p] = key;
    }
}

// Per-block digit histogram of dbits-bit digits, stored digit-major:
// hist[d * nblocks + b].  Equal digits in consecutive lanes (the keys are
// mostly in order after the first sort) count with one LDS atomic per run.
__global__ __launch_bounds__(kSortThreads) void k_hist(const uint32_t *keys, int np, int shift, int dbits,
                                                       int nblocks, uint32_t *hist)
{
    __shared__ uint32_t h[1 << kMaxDigitBits];
    const int nd = 1 << dbits;
    const uint32_t mask = (uint32_t)nd - 1u;
    for (int d = threadIdx.x; d < nd; d += blockDim.x) h[d] = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int beg = blockIdx.x * kPerBlock;
    const int end = min(np, beg + kPerBlock);
    for (int e0 = beg + (int)threadIdx.x - lane; e0 < end; e0 += blockDim.x)       // uniform per wave
        count_runs(keys, e0, end, shift, mask, h);
    __syncthreads();
    for (int d = threadIdx.x; d < nd; d += blockDim.x) hist[(size_t)d * nblocks + blockIdx.x] = h[d];
}

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *sh, uint32_t &total)
{
    // sh: blockDim.x/64 entries
    int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t x = v;
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) sh[wv] = x;
    __syncthreads();
    int nw = blockDim.x >> 6;
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int k = 0; k < nw; ++k) {
            uint32_t t = sh[k];
            sh[k] = run;
            run += t;
        }
        sh[nw] = run;
    }
    __syncthreads();
    uint32_t r = x - v + sh[wv];
    total = sh[nw];
    __syncthreads();
    return r;
}

// Three-kernel exclusive scan of hist[0..m): segment sums, scan of the sums,
// segment scan with offsets.
__global__ __launch_bounds__(256) void k_scan_reduce(const uint32_t *in, long m, long seg, uint32_t *part)
{
    long beg = blockIdx.x * seg, end = min(m, beg + seg);
    uint32_t s = 0;
    for (long i = beg + threadIdx.x; i < end; i += blockDim.x) s += in[i];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    __shared__ uint32_t w[4];
    if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = w[0] + w[1] + w[2] + w[3];
}

__global__ __launch_bounds__(kScanBlocks) void k_scan_parts(uint32_t *part, int nparts)
{
    __shared__ uint32_t sh[kScanBlocks / 64 + 1];
    uint32_t v = threadIdx.x < nparts ? part[threadIdx.x] : 0u;
    uint32_t total;
    uint32_t r = block_exclusive_scan(v, sh, total);
    if (threadIdx.x < nparts) part[threadIdx.x] = r;
}

__global__ __launch_bounds__(256) void k_scan_apply(const uint32_t *in, long m, long seg, const uint32_t *part,
                                                    uint32_t *out)
{
    __shared__ uint32_t sh[256 / 64 + 1];
    long beg = blockIdx.x * seg, end = min(m, beg + seg);
    uint32_t run = part[blockIdx.x];
    for (long base = beg; base < end; base += blockDim.x) {
        long i = base + threadIdx.x;
        uint32_t v = i < end ? in[i] : 0u;
        uint32_t total;
        uint32_t r = block_exclusive_scan(v, sh, total);
        if (i < end) out[i] = run + r;
        run += total;
    }
}

// Stable scatter of one radix pass of dbits-bit digits (per-wave digit
// cursors in dynamic LDS: kSortWaves << dbits words).  idx_in == nullptr
// means identity (first pass).
__global__ __launch_bounds__(kSortThreads) void k_scatter(const uint32_t *keys_in, const uint32_t *idx_in,
                                                          uint32_t *keys_out, uint32_t *idx_out, int np,
                                                          int shift, int dbits, int nblocks, const uint32_t *offs)
{
    extern __shared__ uint32_t wcs[];
    const int nd = 1 << dbits;
    const uint32_t mask = (uint32_t)nd - 1u;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t *wc = wcs + wv * nd;                     // this wave's cursors
    for (int e = threadIdx.x; e < kSortWaves * nd; e += blockDim.x) wcs[e] = 0;
    __syncthreads();
    const int bbeg = blockIdx.x * kPerBlock;
    const int wbeg = bbeg + wv * kPerWave;
    const int wend = min(np, wbeg + kPerWave);
    for (int e0 = wbeg; e0 < wend; e0 += 64) count_runs(keys_in, e0, wend, shift, mask, wc);
    __syncthreads();
    for (int d = threadIdx.x; d < nd; d += blockDim.x) {
        uint32_t run = offs[(size_t)d * nblocks + blockIdx.x];
        for (int w = 0; w < kSortWaves; ++w) {
            uint32_t t = wcs[w * nd + d];
            wcs[w * nd + d] = run;
            run += t;
        }
    }
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int base = wbeg; base < wend; base += 64) {
        int e = base + lane;
        bool valid = e < wend;
        uint32_t k = valid ? keys_in[e] : 0u;
        uint32_t id = valid ? (idx_in ? idx_in[e] : (uint32_t)e) : 0u;
        uint32_t d = (k >> shift) & mask;
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < dbits; ++b) {
            uint64_t m = __ballot(valid && ((d >> b) & 1u));
            peers &= ((d >> b) & 1u) ? m : ~m;
        }
        if (valid) {
            uint32_t rank = (uint32_t)__popcll(peers & lt);
            uint32_t dst = wc[d] + rank;
            keys_out[dst] = k;
            idx_out[dst] = id;
        }
        // make every lane's read of wc[d] happen before the update
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        if (valid) {
            // highest lane of each peer group advances its digit's cursor
            uint64_t higher = peers & ~(lt | (1ull << lane));
            if (higher == 0) wc[d] += (uint32_t)__popcll(peers);
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// Every SoA array of an item moved by one permutation in one pass: the
// permutation is read once, and all of a position's loads are in flight
// before its stores.  With perm2 the source of position r is
// perm2[perm[r]] (run order: new position -> sorted position -> source).
struct PermArrays {
    const void *src[SortArgs::kMaxArrays];
    void *dst[SortArgs::kMaxArrays];
    int wide;                // bit k: array k has 8-byte elements
    int n;
};

__global__ void k_permute_all(const uint32_t *__restrict__ perm, const uint32_t *__restrict__ perm2, int np,
                              PermArrays pa)
{
    // two positions per iteration, every load of both issued before any store
    const int stride = gridDim.x * blockDim.x;
    for (int r0 = blockIdx.x * blockDim.x + threadIdx.x; r0 < np; r0 += 2 * stride) {
        const int r1 = r0 + stride;
        const bool two = r1 < np;
        uint32_t q0 = perm[r0], q1 = two ? perm[r1] : q0;
        if (perm2) {
            q0 = perm2[q0];
            q1 = perm2[q1];
        }
        unsigned long long v0[SortArgs::kMaxArrays], v1[SortArgs::kMaxArrays];
#pragma unroll
        for (int k = 0; k < SortArgs::kMaxArrays; ++k) {
            if (k < pa.n) {
                if ((pa.wide >> k) & 1) {
                    v0[k] = ((const unsigned long long *)pa.src[k])[q0];
                    v1[k] = ((const unsigned long long *)pa.src[k])[q1];
                } else {
                    v0[k] = ((const uint32_t *)pa.src[k])[q0];
                    v1[k] = ((const uint32_t *)pa.src[k])[q1];
                }
            }
        }
#pragma unroll
        for (int k = 0; k < SortArgs::kMaxArrays; ++k) {
            if (k < pa.n) {
                if ((pa.wide >> k) & 1) {
                    ((unsigned long long *)pa.dst[k])[r0] = v0[k];
                    if (two) ((unsigned long long *)pa.dst[k])[r1] = v1[k];
                } else {
                    ((uint32_t *)pa.dst[k])[r0] = (uint32_t)v0[k];
                    if (two) ((uint32_t *)pa.dst[k])[r1] = (uint32_t)v1[k];
                }
            }
        }
    }
}

// Spectral rows (nb float64 per particle, particle-major): destination row r
// takes source row perm[r] (perm2[perm[r]] with perm2); one wave per row.
__global__ __launch_bounds__(256) void k_permute_rows(const uint32_t *perm, const uint32_t *perm2, int np, int nb,
                                                      const double *src0, double *dst0, const double *src1,
                                                      double *dst1)
{
    const int lane = threadIdx.x & 63;
    for (int r = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; r < np; r += (gridDim.x * blockDim.x) >> 6) {
        const uint32_t q = perm2 ? perm2[perm[r]] : perm[r];
        const long s = (long)q * nb, d = (long)r * nb;
        for (int i = lane; i < nb; i += 64) {
            dst0[d + i] = src0[s + i];
            dst1[d + i] = src1[s + i];
        }
    }
}

static void permute_arrays(Ctx *c, const SortArgs &a, const uint32_t *perm, const uint32_t *perm2, int grid)
{
    if (a.nb > 0) {
        const int g = std::max(1, std::min((a.np + 3) / 4, 64 * c->num_cu));
        hipLaunchKernelGGL(k_permute_rows, dim3(g), dim3(256), 0, c->stream, perm, perm2, a.np, a.nb, a.rsrc[0],
                           a.rdst[0], a.rsrc[1], a.rdst[1]);
        c->stats[0]++;
    }
    PermArrays pa;
    memset(&pa, 0, sizeof(pa));
    pa.n = a.narrays;
    for (int k = 0; k < a.narrays; ++k) {
        pa.src[k] = a.src[k];
        pa.dst[k] = a.dst[k];
        if (a.esize[k] == 8) pa.wide |= 1 << k;
    }
    hipLaunchKernelGGL(k_permute_all, dim3(grid), dim3(256), 0, c->stream, perm, perm2, a.np, pa);
    c->stats[0]++;
}

__global__ void k_tile_start(const uint32_t *keys, int np, int shift, int per_tile, int ntiles, int32_t *ts)
{
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < np; r += gridDim.x * blockDim.x) {
        int t = (int)((keys[r] >> shift) / (uint32_t)per_tile);
        int prev = r > 0 ? (int)((keys[r - 1] >> shift) / (uint32_t)per_tile) : -1;
        for (int q = prev + 1; q <= t; ++q) ts[q] = r;
        if (r == np - 1)
            for (int q = t + 1; q <= ntiles; ++q) ts[q] = np;
    }
}

// First sorted position of every cell (keys sorted by tile * cells_per_tile +
// cell in tile); cells without particles are never read.
__global__ void k_cell_start(const uint32_t *keys, int np, int32_t *cs)
{
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < np; r += gridDim.x * blockDim.x)
        if (r == 0 || keys[r] != keys[r - 1]) cs[keys[r]] = r;
}

// Rank-interleaved key of sorted position r: its rank among the particles of
// its cell (positions are in stable order, so this is the number of earlier
// particles of the same cell), capped at 2^rank_bits - 1, between tile and cell.
// The input key is tile * per_tile + cell in tile; per_tile <= 2^cell_bits.
__global__ void k_rank_keys(uint32_t *keys, int np, const int32_t *cs, int per_tile, int cell_bits, int rank_bits)
{
    const uint32_t rmax = (1u << rank_bits) - 1u, pt = (uint32_t)per_tile;
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < np; r += gridDim.x * blockDim.x) {
        uint32_t k = keys[r];
        uint32_t rank = min((uint32_t)(r - cs[k]), rmax);
        uint32_t tile = k / pt, local = k - tile * pt;
        keys[r] = (tile << (rank_bits + cell_bits)) | (rank << cell_bits) | local;
    }
}

// Run table of one tile per block (keys sorted by tile * cells_per_tile + cell
// in tile): the particles of every cell are cut into runs of up to kRunLen
// consecutive positions, and the runs are listed by (index of the run inside
// its cell, cell), so consecutive runs belong to distinct cells.  Entry:
// (first position << 2) | (length - 1), stored from runs[tile_start[t]];
// the tile's run count goes to runs[np + t].  With perm_out (run order) the
// runs are laid out one after another in table order from tile_start[t]: the
// entries hold those positions, and perm_out[new position] = sorted position
// (the permute pass composes it with the sort's permutation).  The first
// kRunsDense rounds (run index inside the cell) take one block scan each; the
// cells with more runs (crowded cells of clumped particles, up to hundreds of
// rounds) are then listed in cell order and the block's waves take the
// remaining rounds in turn, each dropping a cell from its own list after the
// cell's last run in that wave's rounds.
constexpr int kRunsBuildThreads = 256;
constexpr int kRunsDense = 8;
static_assert(kRunLen == 4, "the crowded rounds' ballot prefix sums take run shortfalls of two bits");
__global__ __launch_bounds__(kRunsBuildThreads) void k_runs_build(const uint32_t *keys, int np, int per_tile,
                                                                  int ntiles, const int32_t *ts, int32_t *runs,
                                                                  uint32_t *perm_out)
{
    __shared__ int cnt[kRunsMaxTileCells];
    __shared__ int first[kRunsMaxTileCells];
    __shared__ int4 crowd[kRunsMaxTileCells];
    __shared__ int wl[(kRunsBuildThreads / 64) * kRunsMaxTileCells];
    __shared__ uint32_t sh[kRunsBuildThreads / 64 + 1];
    __shared__ int s_max;
    const int cpt = (per_tile + kRunsBuildThreads - 1) / kRunsBuildThreads;   // cells per thread
    const int c0 = threadIdx.x * cpt, c1 = min(per_tile, c0 + cpt);
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int beg = ts[t], end = ts[t + 1];
        for (int c = threadIdx.x; c < per_tile; c += blockDim.x) cnt[c] = 0;
        if (threadIdx.x == 0) s_max = 0;
        __syncthreads();
        // first sorted position and end of every cell from the key boundaries
        // (the keys are sorted: no atomics, crowded cells included).  Each
        // thread takes four consecutive keys per 16-byte load and issues the
        // loads of KB such groups before using any.
        const uint32_t kb = (uint32_t)t * (uint32_t)per_tile;
        {
            typedef uint32_t U4 __attribute__((ext_vector_type(4), aligned(4)));
            constexpr int KB = 8;
            const int bd = (int)blockDim.x;
            for (int p0 = beg + 4 * (int)threadIdx.x; p0 < end; p0 += 4 * KB * bd) {
                uint32_t kc[KB][4], kp[KB], kn[KB];
#pragma unroll
                for (int i = 0; i < KB; ++i) {
                    const int p = p0 + 4 * i * bd;
                    if (p + 4 <= end) {
                        const U4 v = *reinterpret_cast<const U4 *>(keys + p);
                        kc[i][0] = v[0];
                        kc[i][1] = v[1];
                        kc[i][2] = v[2];
                        kc[i][3] = v[3];
                    } else {
#pragma unroll
                        for (int q = 0; q < 4; ++q) kc[i][q] = p + q < end ? keys[p + q] : ~0u;
                    }
                    kp[i] = p < end && p > beg ? keys[p - 1] : ~0u;
                    kn[i] = p + 4 < end ? keys[p + 4] : ~0u;
                }
#pragma unroll
                for (int i = 0; i < KB; ++i) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int p = p0 + 4 * i * bd + q;
                        const uint32_t k = kc[i][q];
                        const uint32_t before = q == 0 ? kp[i] : kc[i][q - 1];
                        const uint32_t after = q == 3 ? kn[i] : kc[i][q + 1];
                        const uint32_t loc = k - kb;
                        if (p < end && loc < (uint32_t)per_tile) {
                            if (before != k) first[loc] = p;
                            if (after != k) cnt[loc] = p + 1;        // one past the cell's last
                        }
                    }
                }
            }
        }
        __syncthreads();
        // counts, the largest run count and the tile's run count
        int mx = 0;
        uint32_t mruns = 0;
        for (int c = c0; c < c1; ++c) {
            if (cnt[c] > 0) cnt[c] -= first[c];
            mx = max(mx, (cnt[c] + kRunLen - 1) / kRunLen);
            mruns += (uint32_t)((cnt[c] + kRunLen - 1) / kRunLen);
        }
        uint32_t total, truns;
        block_exclusive_scan(mruns, sh, truns);
        atomicMax(&s_max, mx);
        __syncthreads();
        const int nb = s_max;
        const int nb0 = min(nb, kRunsDense);
        int base = 0, lbase = 0;
        for (int b = 0; b < nb0; ++b) {
            // runs (high half) and particles (low half) of this round before my
            // cells: at most 1024 runs and 4096 particles, so the halves never carry
            uint32_t here = 0;
            for (int c = c0; c < c1; ++c) {
                const int left = cnt[c] - b * kRunLen;
                if (left > 0) here += (1u << 16) | (uint32_t)min(kRunLen, left);
            }
            uint32_t pk = block_exclusive_scan(here, sh, total);
            int pos = (int)(pk >> 16), lpos = (int)(pk & 0xffffu);
            for (int c = c0; c < c1; ++c) {
                const int left = cnt[c] - b * kRunLen;
                if (left > 0) {
                    const int len = min(kRunLen, left);
                    const int src = first[c] + b * kRunLen;
                    const int dst = perm_out ? beg + lbase + lpos : src;
                    runs[beg + base + pos] = (dst << 2) | (len - 1);
                    if (perm_out)
                        for (int i = 0; i < len; ++i) perm_out[dst + i] = (uint32_t)(src + i);
                    ++pos;
                    lpos += len;
                }
            }
            base += (int)(total >> 16);
            lbase += (int)(total & 0xffffu);
        }
        if (nb > nb0) {
            // cells with more than nb0 runs, in cell order: (cell, first
            // sorted position, particle count)
            uint32_t mine_c = 0;
            for (int c = c0; c < c1; ++c) mine_c += cnt[c] > nb0 * kRunLen ? 1u : 0u;
            uint32_t k = block_exclusive_scan(mine_c, sh, total);
            for (int c = c0; c < c1; ++c)
                if (cnt[c] > nb0 * kRunLen) crowd[k++] = make_int4(c, first[c], cnt[c], 0);
            __syncthreads();
            // wave w takes rounds nb0 + w, + NW, ... with its own list of the
            // cells that still have a run in its next round (in cell order).
            // Its first base follows from the rounds before it; after each
            // round it adds the runs and particles of that round and of the
            // NW - 1 rounds the other waves take, all counted on its list.
            constexpr int NW = kRunsBuildThreads / 64;
            const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
            const uint64_t lt = (1ull << lane) - 1ull;
            const int K = (int)total;
            int *mylist = wl + w * kRunsMaxTileCells;
            // runs and particles of one round b on a chunk of cells with counts n
            auto round_counts = [&](bool in, int n, int b, int &r, int &q) {
                const bool a = in && n > b * kRunLen;
                const int d = a ? kRunLen - min(kRunLen, n - b * kRunLen) : 0;
                const uint64_t am = __ballot(a), d0 = __ballot(d & 1), d1 = __ballot(d & 2);
                r += __popcll(am);
                q += kRunLen * __popcll(am) - __popcll(d0) - 2 * __popcll(d1);
            };
            int wb = base, wl0 = lbase, Kw = 0;
            for (int j0 = 0; j0 < K; j0 += 64) {
                const int j = j0 + lane;
                const bool in = j < K;
                const int n = in ? crowd[j].z : 0;
                for (int k = 0; k < w; ++k) round_counts(in, n, nb0 + k, wb, wl0);
                const bool keep = in && n > (nb0 + w) * kRunLen;
                const uint64_t km = __ballot(keep);
                if (keep) mylist[Kw + __popcll(km & lt)] = j;
                Kw += __popcll(km);
            }
            for (int b = nb0 + w; Kw > 0; b += NW) {
                int kept = 0, rpos = 0, ppos = 0, radd = 0, padd = 0;
                for (int j0 = 0; j0 < Kw; j0 += 64) {
                    const int j = j0 + lane;
                    const bool in = j < Kw;
                    const int idx = in ? mylist[j] : 0;
                    const int4 e = in ? crowd[idx] : make_int4(0, 0, 0, 0);
                    const int left = e.z - b * kRunLen;
                    const int len = in ? min(kRunLen, left) : 0;
                    // prefix sums of the run lengths from ballots: kRunLen per
                    // active lane minus the shortfall (0..3) of last runs
                    const int d = in ? kRunLen - len : 0;
                    const uint64_t am = __ballot(in);
                    const uint64_t d0 = __ballot(d & 1), d1 = __ballot(d & 2);
                    const int lpre = kRunLen * __popcll(am & lt) - __popcll(d0 & lt) - 2 * __popcll(d1 & lt);
                    if (in) {
                        const int pos = rpos + __popcll(am & lt);
                        const int src = e.y + b * kRunLen;
                        const int dst = perm_out ? beg + wl0 + ppos + lpre : src;
                        runs[beg + wb + pos] = (dst << 2) | (len - 1);
                        if (perm_out)
                            for (int i = 0; i < len; ++i) perm_out[dst + i] = (uint32_t)(src + i);
                    }
                    rpos += __popcll(am);
                    ppos += kRunLen * __popcll(am) - __popcll(d0) - 2 * __popcll(d1);
                    for (int k = 1; k < NW; ++k) round_counts(in, e.z, b + k, radd, padd);
                    // the list is read ahead of every write (kept <= j0)
                    const bool keep = in && e.z > (b + NW) * kRunLen;
                    const uint64_t km = __ballot(keep);
                    if (keep) mylist[kept + __popcll(km & lt)] = idx;
                    kept += __popcll(km);
                }
                wb += rpos + radd;
                wl0 += ppos + padd;
                Kw = kept;
            }
            base = (int)truns;
        }
        if (threadIdx.x == 0) runs[np + t] = base;
        __syncthreads();
    }
}

// Work units of the run-based kernel (one block).  With P = max(ceil(total
// runs / kRunsSplit), kRunsMinPiece), a tile of c runs becomes ceil(c / P)
// pieces (an empty tile none), so at most ntiles + kRunsSplit units exist.
// Tiles cut into pieces or holding more than twice the mean run count go
// first, by decreasing runs per piece (ties by tile index), each followed by
// its pieces in order; then every other non-empty tile in index order.  The
// first kRankMax such tiles (in index order) are ranked; later ones keep index
// order.  Largest-first claiming keeps a crowded tile from finishing last on
// its CU, and splitting keeps one tile from outweighing a CU's share of the
// step.  Every loop that contains a block scan has the same trip count in all
// threads.
constexpr int kOrderThreads = 1024;
constexpr int kRankMax = 1024;
__global__ __launch_bounds__(kOrderThreads) void k_unit_list(int32_t *runs, int np, int ntiles)
{
    __shared__ uint32_t sh[kOrderThreads / 64 + 1];
    __shared__ int rk_tile[kRankMax];
    __shared__ int rk_cnt[kRankMax];
    __shared__ int rk_k[kRankMax];
    __shared__ int by_rank[kRankMax];
    __shared__ unsigned long long s_total;
    const int32_t *cnt = runs + np;
    int32_t *units = runs + runs_units_at(np, ntiles);
    const long long cap = (long long)ntiles + kRunsSplit;
    if (threadIdx.x == 0) s_total = 0ull;
    __syncthreads();
    unsigned long long mine = 0;
    for (int t = threadIdx.x; t < ntiles; t += blockDim.x) mine += (unsigned long long)max(cnt[t], 0);
    atomicAdd(&s_total, mine);
    __syncthreads();
    const long long total = (long long)s_total;
    const long long pz = max((total + kRunsSplit - 1) / kRunsSplit, (long long)kRunsMinPiece);
    const long long thr = 2 * (total / max(ntiles, 1)) + 1;
    auto pieces = [&](int t) -> int {
        const long long c = max(cnt[t], 0);
        return (int)((c + pz - 1) / pz);
    };
    auto emit = [&](long long at, int t, int k) {
        for (int p = 0; p < k; ++p)
            if (at + p < cap) {
                units[2 * (at + p)] = t;
                units[2 * (at + p) + 1] = p | (k << 16);
            }
    };
    // ranked tiles: the first kRankMax split or heavy tiles in index order
    uint32_t hbase = 0;
    for (int t0 = 0; t0 < ntiles; t0 += blockDim.x) {
        const int t = t0 + threadIdx.x;
        const int k = t < ntiles ? pieces(t) : 0;
        const bool h = t < ntiles && (k >= 2 || (long long)cnt[t] > thr);
        uint32_t tot;
        const uint32_t hp = hbase + block_exclusive_scan(h ? 1u : 0u, sh, tot);
        if (h && hp < (uint32_t)kRankMax) {
            rk_tile[hp] = t;
            rk_cnt[hp] = cnt[t];
            rk_k[hp] = k;
        }
        hbase += tot;
    }
    const int nh = (int)min(hbase, (uint32_t)kRankMax);
    __syncthreads();
    // rank by decreasing runs per piece (cnt / k, compared exactly), ties by tile
    for (int i = threadIdx.x; i < nh; i += blockDim.x) {
        const long long ci = rk_cnt[i], ki = rk_k[i];
        int rank = 0;
        for (int j = 0; j < nh; ++j) {
            const long long a = (long long)rk_cnt[j] * ki, b = ci * (long long)rk_k[j];
            rank += a > b || (a == b && rk_tile[j] < rk_tile[i]);
        }
        by_rank[rank] = i;
    }
    __syncthreads();
    uint32_t nranked;
    {
        const int i = threadIdx.x < nh ? by_rank[threadIdx.x] : 0;
        const uint32_t k = threadIdx.x < nh ? (uint32_t)rk_k[i] : 0u;
        const uint32_t at = block_exclusive_scan(k, sh, nranked);
        if (threadIdx.x < nh) emit(at, rk_tile[i], (int)k);
    }
    // every other non-empty tile in index order
    uint32_t hb = 0;
    long long lb = nranked;
    for (int t0 = 0; t0 < ntiles; t0 += blockDim.x) {
        const int t = t0 + threadIdx.x;
        const int k = t < ntiles ? pieces(t) : 0;
        const bool h = t < ntiles && (k >= 2 || (long long)cnt[t] > thr);
        uint32_t toth, totl;
        const uint32_t hp = hb + block_exclusive_scan(h ? 1u : 0u, sh, toth);
        const bool ranked = h && hp < (uint32_t)kRankMax;
        const uint32_t kl = (t < ntiles && !ranked) ? (uint32_t)k : 0u;
        const uint32_t lp = block_exclusive_scan(kl, sh, totl);
        if (kl) emit(lb + lp, t, (int)kl);
        hb += toth;
        lb += totl;
    }
    if (threadIdx.x == 0) runs[runs_count_at(np, ntiles)] = (int32_t)min(lb, cap);
}

__global__ void k_fill_i32(int32_t *p, int n, int v)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

static int bits_for(uint64_t count)
{
    int b = 0;
    while (b < 32 && ((uint64_t)1 << b) < count) ++b;
    return b;
}

// LSD radix passes over the low `bits` bits of keys[src] with indices idx[src]
// (identity when `identity`); returns the buffer index holding the result.
// Digits of kMaxDigitBits bits, the last pass taking only the bits left.
// (Wider digits, 11 bits in two passes for 21-bit keys, were slower: the
// per-block digit tables cost more than the pass they save.)
static int radix_passes(Ctx *c, int np, int src, bool identity, int bits)
{
    hipStream_t s = c->stream;
    const int nblocks = (np + kPerBlock - 1) / kPerBlock;
    bits = std::max(bits, 1);
    const int width = kMaxDigitBits;
    const int npass = (bits + width - 1) / width;
    for (int pass = 0; pass < npass; ++pass) {
        const int shift = width * pass;
        const int dbits = std::min(width, bits - shift);
        const long m = (long)nblocks << dbits;
        const long seg = (m + kScanBlocks - 1) / kScanBlocks;
        const int nparts = (int)((m + seg - 1) / seg);
        uint32_t *part = c->hist_scan + m;
        hipLaunchKernelGGL(k_hist, dim3(nblocks), dim3(kSortThreads), 0, s, c->keys[src], np, shift, dbits, nblocks,
                           c->hist);
        hipLaunchKernelGGL(k_scan_reduce, dim3(nparts), dim3(256), 0, s, c->hist, m, seg, part);
        hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(kScanBlocks), 0, s, part, nparts);
        hipLaunchKernelGGL(k_scan_apply, dim3(nparts), dim3(256), 0, s, c->hist, m, seg, part, c->hist_scan);
        hipLaunchKernelGGL(k_scatter, dim3(nblocks), dim3(kSortThreads), (size_t)(kSortWaves << dbits) * 4, s,
                           c->keys[src], (identity && pass == 0) ? (const uint32_t *)nullptr : c->idx[src],
                           c->keys[1 - src], c->idx[1 - src], np, shift, dbits, nblocks, c->hist_scan);
        c->stats[0] += 5;
        src = 1 - src;
    }
    return src;
}

hipError_t launch_sort(Ctx *c, const SortArgs &a)
{
    hipStream_t s = c->stream;
    if (a.np == 0) {
        hipLaunchKernelGGL(k_fill_i32, dim3(std::max(1, (a.ntiles + 256) / 256)), dim3(256), 0, s, a.tile_start,
                           a.ntiles + 1, 0);
        c->stats[0]++;
        if (a.runs) {
            hipLaunchKernelGGL(k_fill_i32, dim3(std::max(1, (a.ntiles + 256) / 256)), dim3(256), 0, s, a.runs,
                               a.ntiles, 0);
            hipLaunchKernelGGL(k_unit_list, dim3(1), dim3(kOrderThreads), 0, s, a.runs, 0, a.ntiles);
            c->stats[0] += 2;
        }
        return hipGetLastError();
    }
    const int per_tile_cells = a.tile[0] * a.tile[1] * a.tile[2];
    const int grid_e = std::min((a.np + 255) / 256, 16 * c->num_cu);
    int src, shift = 0, div = 1;
    if (a.key_mode == PL_KEY_TILE_RANK) {
        // phase 1: stable sort by (tile, cell); phase 2: stable sort by
        // (tile, rank in cell, cell) on top of it
        SortArgs b = a;
        b.key_mode = PL_KEY_TILE_CELL;
        hipLaunchKernelGGL(k_keys, dim3(grid_e), dim3(256), 0, s, b, c->keys[0]);
        src = radix_passes(c, a.np, 0, true, bits_for((uint64_t)a.ntiles * per_tile_cells));
        const int cb = bits_for((uint64_t)per_tile_cells), tb = bits_for((uint64_t)a.ntiles);
        const int rb = std::min(10, 32 - tb - cb);
        hipLaunchKernelGGL(k_cell_start, dim3(grid_e), dim3(256), 0, s, c->keys[src], a.np, c->cell_start);
        hipLaunchKernelGGL(k_rank_keys, dim3(grid_e), dim3(256), 0, s, c->keys[src], a.np, c->cell_start,
                           per_tile_cells, cb, rb);
        src = radix_passes(c, a.np, src, false, tb + rb + cb);
        shift = rb + cb;
        c->stats[0] += 3;
    } else {
        hipLaunchKernelGGL(k_keys, dim3(grid_e), dim3(256), 0, s, a, c->keys[0]);
        div = a.key_mode == PL_KEY_TILE ? 1 : per_tile_cells;
        src = radix_passes(c, a.np, 0, true, bits_for((uint64_t)a.ntiles * div));
        c->stats[0]++;
    }
    if (a.key_mode == PL_KEY_TILE_RUN) {
        // run order: tile offsets and the run table from the tile+cell order,
        // then every array moved straight into run order
        if (!a.runs) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_tile_start, dim3(grid_e), dim3(256), 0, s, c->keys[src], a.np, 0, div, a.ntiles,
                           a.tile_start);
        // one block per tile: a crowded tile's rounds do not hold up others
        hipLaunchKernelGGL(k_runs_build, dim3(std::max(a.ntiles, 1)), dim3(kRunsBuildThreads), 0, s,
                           c->keys[src], a.np, per_tile_cells, a.ntiles, a.tile_start, a.runs, c->idx[1 - src]);
        permute_arrays(c, a, c->idx[1 - src], c->idx[src], grid_e);
        hipLaunchKernelGGL(k_unit_list, dim3(1), dim3(kOrderThreads), 0, s, a.runs, a.np, a.ntiles);
        c->stats[0] += 3;
        return hipGetLastError();
    }
    permute_arrays(c, a, c->idx[src], nullptr, grid_e);
    hipLaunchKernelGGL(k_tile_start, dim3(grid_e), dim3(256), 0, s, c->keys[src], a.np, shift, div, a.ntiles,
                       a.tile_start);
    c->stats[0]++;
    if (a.runs) {
        // keys are tile * cells_per_tile + cell in tile (PL_KEY_TILE_CELL)
        hipLaunchKernelGGL(k_runs_build, dim3(std::max(a.ntiles, 1)), dim3(kRunsBuildThreads), 0, s,
                           c->keys[src], a.np, per_tile_cells, a.ntiles, a.tile_start, a.runs, nullptr);
        hipLaunchKernelGGL(k_unit_list, dim3(1), dim3(kOrderThreads), 0, s, a.runs, a.np, a.ntiles);
        c->stats[0] += 2;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fixed scratch of pl_sort_noalloc: keys and indices (two buffers each) for
// PL_NOALLOC_MAX_NP particles and the digit histograms and their scan.  Every
// GPU the library runs on holds one copy until the process ends; all calls on
// a device share it (calls that overlap on one device race).
// ---------------------------------------------------------------------------

constexpr int64_t kNaNp = PL_NOALLOC_MAX_NP;
constexpr int64_t kNaHist = (((kNaNp + kPerBlock - 1) / kPerBlock) << kMaxDigitBits) + 1024;
constexpr size_t kNaBytes = (size_t)(4 * kNaNp + 2 * kNaHist) * sizeof(uint32_t);

static __device__ __align__(256) unsigned char scratch[kNaBytes];

constexpr int kNaDevices = 64;
static std::mutex na_mu;
static void *na_ptr[kNaDevices];       // device address of `scratch` on each device
static int na_cu[kNaDevices];

hipError_t launch_sort_noalloc(Ctx *c, const SortArgs &a)
{
    if (a.np > kNaNp) return hipErrorInvalidValue;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kNaDevices) return hipErrorInvalidDevice;
    void *base = nullptr;
    int cu = 0;
    {
        std::lock_guard<std::mutex> lock(na_mu);
        if (!na_ptr[dev]) {
            // once per device, with that device current: the array's device
            // address (the symbol itself is a host-side stand-in)
            void *p = nullptr;
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess) return e;
            int n = 0;
            e = hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev);
            if (e != hipSuccess) return e;
            na_cu[dev] = n > 0 ? n : 1;
            na_ptr[dev] = p;
        }
        base = na_ptr[dev];
        cu = na_cu[dev];
    }
    uint32_t *w = static_cast<uint32_t *>(base);
    c->num_cu = cu;
    c->keys[0] = w;
    c->keys[1] = w + kNaNp;
    c->idx[0] = w + 2 * kNaNp;
    c->idx[1] = w + 3 * kNaNp;
    c->hist = w + 4 * kNaNp;
    c->hist_scan = w + 4 * kNaNp + kNaHist;
    c->hist_cap = kNaHist;
    c->cell_start = nullptr;           // PL_KEY_TILE_RANK is refused before this point
    return launch_sort(c, a);
}

}  // namespace pl
