// Step dispatch (one persistent launch per species kind), zeroing, sums and
// pack / unpack kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "pl_device.h"

namespace pl {

hipError_t launch_group_f32(Ctx *c, const ItemDesc *table, const ItemDesc *host, int nitems, int total_units,
                            unsigned sf, bool push, bool deposit, unsigned *counter);
hipError_t launch_group_f64(Ctx *c, const ItemDesc *table, const ItemDesc *host, int nitems, int total_units,
                            unsigned sf, bool push, bool deposit, unsigned *counter);
hipError_t launch_runs_f32(Ctx *c, const ItemDesc *table, const ItemDesc *host, int nitems, int total_units,
                           unsigned sf, unsigned *counter);
hipError_t launch_runs_f64(Ctx *c, const ItemDesc *table, const ItemDesc *host, int nitems, int total_units,
                           unsigned sf, unsigned *counter);

// The host table is ordered by species kind, then by particle count.  A fused
// run-based step is one launch over every item; otherwise every run of one
// kind is one launch with its own work counter.
hipError_t launch_step(Ctx *c, const ItemDesc *table, const std::vector<ItemDesc> &host, int nitems,
                       int total_units, unsigned flags, bool deposit, bool push)
{
    (void)total_units;
    unsigned sf = (push ? SF_PUSH : 0u) | (deposit ? SF_DEPOSIT : 0u) | ((flags & PL_SUMS) ? SF_SUMS : 0u) |
                  (c->runs ? SF_RUNS : 0u);
    // a fused run-based step with every kind in one launch (the item table
    // numbers units across all items then: see build_table)
    RunsPlan pl;
    if (c->one_launch && c->d.algo == PL_ALGO_RUNS && push && deposit && runs_plan(c, host.data(), nitems, pl)) {
        int units = 0;
        for (int i = 0; i < nitems; ++i) units += host[i].nunits;
        return c->d.prec == PL_F64 ? launch_runs_f64(c, table, host.data(), nitems, units, sf, c->counters)
                                   : launch_runs_f32(c, table, host.data(), nitems, units, sf, c->counters);
    }
    int i0 = 0, group = 0;
    while (i0 < nitems) {
        int i1 = i0;
        int units = 0;
        while (i1 < nitems && host[i1].kind == host[i0].kind) units += host[i1++].nunits;
        // the run-based kernel takes fused steps of charged and dust species;
        // everything else (and a tile too large for its LDS) takes the tiled one
        hipError_t e = hipErrorInvalidConfiguration;
        if (c->d.algo == PL_ALGO_RUNS && push && deposit && host[i0].kind != PL_TRACER)
            e = c->d.prec == PL_F64 ? launch_runs_f64(c, table + i0, host.data() + i0, i1 - i0, units, sf,
                                                      c->counters + kCounterStride * group)
                                    : launch_runs_f32(c, table + i0, host.data() + i0, i1 - i0, units, sf,
                                                      c->counters + kCounterStride * group);
        if (e == hipErrorInvalidConfiguration && c->d.algo == PL_ALGO_RUNS && push && deposit &&
            host[i0].kind != PL_TRACER)
            c->stats[5]++;
        if (e == hipErrorInvalidConfiguration)
            e = c->d.prec == PL_F64
                    ? launch_group_f64(c, table + i0, host.data() + i0, i1 - i0, units, sf, push, deposit,
                                       c->counters + kCounterStride * group)
                    : launch_group_f32(c, table + i0, host.data() + i0, i1 - i0, units, sf, push, deposit,
                                       c->counters + kCounterStride * group);
        if (e != hipSuccess) return e;
        i0 = i1;
        ++group;
    }
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// Zeroing, sums, pack / unpack
// ---------------------------------------------------------------------------

__global__ void k_zero(double *p, long n)
{
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = 0.0;
}

// Every active moment channel of every item of a call in one launch: block
// row y zeroes channel y % kMaxCh of item y / kMaxCh (items from the device
// table of the call).
__global__ void k_zero_items(const ItemDesc *items)
{
    const ItemDesc &it = items[blockIdx.y / kMaxCh];
    const int ch = blockIdx.y % kMaxCh;
    if (it.kind == PL_TRACER || it.slot[ch] < 0) return;
    double *p = it.M[ch];
    const long n = (long)it.n[0] * it.n[1] * it.n[2];
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = 0.0;
}

hipError_t launch_zero(Ctx *c, const ItemDesc *table, const std::vector<ItemDesc> &host)
{
    long cells = 0;
    for (const ItemDesc &it : host)
        if (it.kind != PL_TRACER) cells = std::max(cells, (long)it.n[0] * it.n[1] * it.n[2]);
    if (cells == 0 || host.empty()) return hipSuccess;
    const int channels = (int)host.size() * kMaxCh;
    const int gx = (int)std::max<long>(1, std::min<long>((cells + 255) / 256, (8L * c->num_cu + channels - 1) / channels * 4));
    hipLaunchKernelGGL(k_zero_items, dim3(gx, channels), dim3(256), 0, c->stream, table);
    c->stats[0]++;
    return hipGetLastError();
}

hipError_t launch_zero_sums(Ctx *c, double *sums, int n)
{
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(256), 0, c->stream, sums, (long)n);
    c->stats[0]++;
    return hipGetLastError();
}

__global__ void k_grid_sum(const double *p, long n, double scale, double *out)
{
    double s = 0.0;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) s += p[i];
    s = wave_sum(s);
    __shared__ double part[16];
    int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) part[wv] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += part[k];
        global_add(out, t * scale);
    }
}

hipError_t launch_grid_sums(Ctx *c, const ItemDesc &it, double *out8)
{
    long cells = (long)it.n[0] * it.n[1] * it.n[2];
    double dv = 1.0 / it.inv_dv;
    int grid = (int)std::min<long>((cells + 255) / 256, 4L * c->num_cu);
    for (int ch = 0; ch < kMaxCh; ++ch) {
        if (!it.M[ch]) continue;
        hipLaunchKernelGGL(k_grid_sum, dim3(grid), dim3(256), 0, c->stream, it.M[ch], cells, dv, out8 + ch);
        c->stats[0]++;
    }
    return hipGetLastError();
}

template <int PREC>
__global__ void k_pack(ItemDesc it, int ndim, const double *x0, const double *x1, const double *x2,
                       const double *u0, const double *u1, const double *u2, int *errflags)
{
    const double *xs[3] = {x0, x1, x2};
    const double *us[3] = {u0, u1, u2};
    int err = 0;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < it.np; p += gridDim.x * blockDim.x) {
        int c[3] = {0, 0, 0};
        double xw[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < 3; ++a)
            if (!isfinite(us[a][p])) err |= ERR_NONFINITE;
        for (int a = 0; a < ndim; ++a) {
            double v = xs[a][p];
            double nn = (double)it.n[a];
            if (!(v >= 0.0 && v < nn)) {
                if (!isfinite(v)) { v = 0.0; err |= ERR_NONFINITE; }
                v = v - nn * floor(v / nn);
                if (v >= nn || v < 0.0) v = 0.0;
            }
            xw[a] = v;
        }
        if (PREC == PL_F64) {
            for (int a = 0; a < ndim; ++a) ((double *)it.x[a])[p] = xw[a];
            for (int a = 0; a < 3; ++a) ((double *)it.u[a])[p] = us[a][p];
        } else {
            for (int a = 0; a < ndim; ++a) {
                double f = floor(xw[a]);
                int ci = (int)f;
                float o = (float)(xw[a] - f - 0.5);
                if (o >= 0.5f) {
                    o = -0.5f;
                    ci = ci + 1 == it.n[a] ? 0 : ci + 1;
                }
                c[a] = ci;
                ((float *)it.x[a])[p] = o;
            }
            it.cell[p] = pack_cell(c[0], c[1], c[2]);
            for (int a = 0; a < 3; ++a) ((float *)it.u[a])[p] = (float)us[a][p];
        }
    }
    if (err) atomicOr(errflags, err);
}

template <int PREC>
__global__ void k_unpack(ItemDesc it, int ndim, double *x0, double *x1, double *x2, double *u0, double *u1,
                         double *u2)
{
    double *xs[3] = {x0, x1, x2};
    double *us[3] = {u0, u1, u2};
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < it.np; p += gridDim.x * blockDim.x) {
        if (PREC == PL_F64) {
            for (int a = 0; a < ndim; ++a) xs[a][p] = ((const double *)it.x[a])[p];
            for (int a = 0; a < 3; ++a) us[a][p] = ((const double *)it.u[a])[p];
        } else {
            int c[3];
            unpack_cell(it.cell[p], c[0], c[1], c[2]);
            for (int a = 0; a < ndim; ++a) xs[a][p] = (double)c[a] + 0.5 + (double)((const float *)it.x[a])[p];
            for (int a = 0; a < 3; ++a) us[a][p] = (double)((const float *)it.u[a])[p];
        }
    }
}

hipError_t launch_pack(Ctx *c, const ItemDesc &it, int prec, int ndim, const double *x[3], const double *u[3])
{
    if (it.np == 0) return hipSuccess;
    int grid = std::min((it.np + 255) / 256, 16 * c->num_cu);
    if (prec == PL_F64)
        hipLaunchKernelGGL(k_pack<PL_F64>, dim3(grid), dim3(256), 0, c->stream, it, ndim, x[0], x[1], x[2], u[0],
                           u[1], u[2], c->errflags);
    else
        hipLaunchKernelGGL(k_pack<PL_F32_OFFSET>, dim3(grid), dim3(256), 0, c->stream, it, ndim, x[0], x[1], x[2],
                           u[0], u[1], u[2], c->errflags);
    c->stats[0]++;
    return hipGetLastError();
}

hipError_t launch_unpack(Ctx *c, const ItemDesc &it, int prec, int ndim, double *x[3], double *u[3])
{
    if (it.np == 0) return hipSuccess;
    int grid = std::min((it.np + 255) / 256, 16 * c->num_cu);
    if (prec == PL_F64)
        hipLaunchKernelGGL(k_unpack<PL_F64>, dim3(grid), dim3(256), 0, c->stream, it, ndim, x[0], x[1], x[2], u[0],
                           u[1], u[2]);
    else
        hipLaunchKernelGGL(k_unpack<PL_F32_OFFSET>, dim3(grid), dim3(256), 0, c->stream, it, ndim, x[0], x[1], x[2],
                           u[0], u[1], u[2]);
    c->stats[0]++;
    return hipGetLastError();
}

}  // namespace pl
