// Device-side building blocks of the particle update: weights, positions in
// both storage forms, pushers.  Header-only, included by the kernel sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pl_internal.h"

namespace pl {

template <int PREC> struct RealOf { using T = double; };

// Pointer into global memory.  Pointers read from the item table are generic
// (flat) pointers; loads and stores through flat pointers also count against
// the LDS wait counter, so every wait for an LDS read would wait for
// outstanding HBM loads as well.  Per-unit pointers are converted to this
// type once, and every particle, field and moment access goes through it.
template <typename T> using gptr = __attribute__((address_space(1))) T *;
template <> struct RealOf<PL_F32_OFFSET> { using T = float; };

// Sum over the 64 lanes of a wave.
template <typename R>
__device__ __forceinline__ R wave_sum(R v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Hardware float64 atomic add on global memory (no compare-and-swap loop).
__device__ __forceinline__ void global_add(double *p, double v)
{
    __hip_atomic_fetch_add((__attribute__((address_space(1))) double *)p, v, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void global_add(gptr<double> p, double v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int wrap_cell(int i, int n)
{
    return i < 0 ? i + n : (i >= n ? i - n : i);
}

// One-dimensional assignment weights on cells i-1, i, i+1 of a particle at
// offset d in [-1/2, 1/2) from the centre of cell i.
//   TSC (quadratic B-spline): (1/2)(1/2 - d)^2, 3/4 - d^2, (1/2)(1/2 + d)^2
//   CIC (linear) written on the same three cells: the particle shares itself
//   between cell i and the neighbour on the side of its offset.
template <int SHAPE, typename R>
__device__ __forceinline__ void weights3(R d, R w[3])
{
    if (SHAPE == PL_TSC) {
        R a = R(0.5) - d, b = R(0.5) + d;
        w[0] = R(0.5) * a * a;
        w[1] = fma(-d, d, R(0.75));
        w[2] = R(0.5) * b * b;
    } else {
        bool up = d >= R(0);
        w[0] = up ? R(0) : -d;
        w[1] = up ? R(1) - d : R(1) + d;
        w[2] = up ? d : R(0);
    }
}

__device__ __forceinline__ uint32_t pack_cell(int i, int j, int k)
{
    return (uint32_t)i | ((uint32_t)j << kCellBits) | ((uint32_t)k << (2 * kCellBits));
}

__device__ __forceinline__ void unpack_cell(uint32_t c, int &i, int &j, int &k)
{
    i = (int)(c & (kMaxN - 1));
    j = (int)((c >> kCellBits) & (kMaxN - 1));
    k = (int)(c >> (2 * kCellBits));
}

// ---------------------------------------------------------------------------
// Particle positions.  Pos<PL_F64> holds absolute float64 grid coordinates;
// Pos<PL_F32_OFFSET> holds an integer cell and a float32 offset from its
// centre.  Both expose the cell c[] and offset d[] (zero beyond DIM) and
// advance by a displacement in cells.
// ---------------------------------------------------------------------------
template <int PREC, int DIM> struct Pos;

template <int DIM> struct Pos<PL_F64, DIM> {
    double x[3];
    int c[3];
    double d[3];

    __device__ __forceinline__ void locate()
    {
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            double f = floor(x[a]);
            c[a] = (int)f;
            d[a] = x[a] - f - 0.5;
        }
    }

    // Bring a coordinate into [0, n); non-finite values are replaced by 0 and
    // reported.
    __device__ __forceinline__ static double wrap(double v, int n, int &err)
    {
        if (!(v >= 0.0 && v < (double)n)) {
            if (!isfinite(v)) { err |= ERR_NONFINITE; return 0.0; }
            double y = v - (double)n * floor(v / (double)n);
            if (y >= (double)n) y = 0.0;
            if (y < 0.0) y = 0.0;
            return y;
        }
        return v;
    }

    // Stored form of one particle's position (fetched ahead of use).
    struct Raw {
        double x[3];
    };

    template <class S>
    __device__ __forceinline__ static void fetch(const S &it, int p, Raw &r)
    {
#pragma unroll
        for (int a = 0; a < 3; ++a) r.x[a] = a < DIM ? (double)it.x[a][p] : 0.0;
    }

    template <class S>
    __device__ __forceinline__ void set(const Raw &r, const S &it, int &err)
    {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            x[a] = a < DIM ? wrap(r.x[a], it.n[a], err) : 0.0;
            c[a] = 0;
            d[a] = 0.0;
        }
        locate();
    }

    template <class S>
    __device__ __forceinline__ void load(const S &it, int p, int &err)
    {
        Raw r;
        fetch(it, p, r);
        set(r, it, err);
    }

    template <class S>
    __device__ __forceinline__ void store(const S &it, int p) const
    {
#pragma unroll
        for (int a = 0; a < DIM; ++a) it.x[a][p] = x[a];
    }

    // Move by disp cells per dimension and wrap periodically.
    template <class S>
    __device__ __forceinline__ void advance(const double disp[3], const S &it, int &err)
    {
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            if (!(fabs(disp[a]) < 1.0)) err |= ERR_CFL;
            x[a] = wrap(x[a] + disp[a], it.n[a], err);
        }
        locate();
    }
};

template <int DIM> struct Pos<PL_F32_OFFSET, DIM> {
    int c[3];
    float d[3];

    __device__ __forceinline__ void locate() {}

    // Stored form of one particle's position (fetched ahead of use).
    struct Raw {
        uint32_t cell;
        float o[3];
    };

    template <class S>
    __device__ __forceinline__ static void fetch(const S &it, int p, Raw &r)
    {
        r.cell = it.cell[p];
#pragma unroll
        for (int a = 0; a < 3; ++a) r.o[a] = a < DIM ? (float)it.x[a][p] : 0.0f;
    }

    template <class S>
    __device__ __forceinline__ void set(const Raw &r, const S &it, int &err)
    {
        int ijk[3];
        unpack_cell(r.cell, ijk[0], ijk[1], ijk[2]);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (a < DIM) {
                c[a] = ijk[a];
                if (c[a] >= it.n[a]) { err |= ERR_NONFINITE; c[a] %= it.n[a]; }
                float o = r.o[a];
                if (!(o >= -0.5f && o < 0.5f)) { err |= ERR_NONFINITE; o = 0.0f; }
                d[a] = o;
            } else {
                c[a] = 0;
                d[a] = 0.0f;
            }
        }
    }

    template <class S>
    __device__ __forceinline__ void load(const S &it, int p, int &err)
    {
        Raw r;
        fetch(it, p, r);
        set(r, it, err);
    }

    template <class S>
    __device__ __forceinline__ void store(const S &it, int p) const
    {
        it.cell[p] = pack_cell(c[0], DIM > 1 ? c[1] : 0, DIM > 2 ? c[2] : 0);
#pragma unroll
        for (int a = 0; a < DIM; ++a) it.x[a][p] = d[a];
    }

    // Offset update in float32; when the particle leaves its cell the new
    // offset and cell shift are computed in float64 (exact sum, one rounding)
    // so crossing a face loses no resolution.  An offset that rounds up to
    // +1/2 belongs to the next cell at -1/2.
    template <class S>
    __device__ __forceinline__ void advance(const float disp[3], const S &it, int &err)
    {
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            if (!(fabsf(disp[a]) < 1.0f)) {
                err |= ERR_CFL;
                if (!isfinite(disp[a])) { err |= ERR_NONFINITE; continue; }
            }
            float t = d[a] + disp[a];
            if (t >= -0.5f && t < 0.5f) {
                d[a] = t;
                continue;
            }
            double s = (double)d[a] + (double)disp[a];
            double sh = floor(s + 0.5);
            float o = (float)(s - sh);
            int shift = (int)sh;
            if (o >= 0.5f) { o = -0.5f; shift += 1; }
            // periodic wrap: one correction covers every step within the
            // CFL limit (|shift| <= 2); the remainder only after a violation
            const int nn = it.n[a];
            int ci = c[a] + shift;
            if (ci < 0) ci += nn;
            else if (ci >= nn) ci -= nn;
            if ((unsigned)ci >= (unsigned)nn) {
                ci %= nn;
                if (ci < 0) ci += nn;
            }
            c[a] = ci;
            d[a] = o;
        }
    }
};

// ---------------------------------------------------------------------------
// Pushers.  All return the velocity change du (used for the force channel
// without the cancellation of u_new - u_old) and update u in place.
// ---------------------------------------------------------------------------

// a/sqrt(x) and a/x for x >= 1 (a Lorentz factor squared, 1 + |t|^2).
// Float32: a times the hardware reciprocal square root or reciprocal (1 ulp
// each; the correctly rounded forms take about ten instructions each, a
// tenth of the push).  Float64: the correctly rounded quotient.
__device__ __forceinline__ float div_sqrt_ge1(float a, float x) { return a * __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double div_sqrt_ge1(double a, double x) { return a / sqrt(x); }
__device__ __forceinline__ float div_ge1(float a, float x) { return a * __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double div_ge1(double a, double x) { return a / x; }

// Relativistic Boris push (Boris 1970) for du/dt = (q/m)(E + u/gamma x B):
// half electric kick, rotation about B by 2 atan(|t|), half electric kick.
// The change is du = 2 h E + (u' x s), with u' = u- + u- x t.
template <typename R>
__device__ __forceinline__ void boris(R u[3], const R E[3], const R B[3], R h, R inv_c2, R du[3])
{
    R hE[3] = {h * E[0], h * E[1], h * E[2]};
    R um[3] = {u[0] + hE[0], u[1] + hE[1], u[2] + hE[2]};
    const R g2 = fma(fma(um[0], um[0], fma(um[1], um[1], um[2] * um[2])), inv_c2, R(1));
    const R hg = div_sqrt_ge1(h, g2);
    R t[3] = {hg * B[0], hg * B[1], hg * B[2]};
    const R f = div_ge1(R(2), R(1) + fma(t[0], t[0], fma(t[1], t[1], t[2] * t[2])));
    R s[3] = {f * t[0], f * t[1], f * t[2]};
    R uc[3] = {um[0] + fma(um[1], t[2], -(um[2] * t[1])),
               um[1] + fma(um[2], t[0], -(um[0] * t[2])),
               um[2] + fma(um[0], t[1], -(um[1] * t[0]))};
    R rot[3] = {fma(uc[1], s[2], -(uc[2] * s[1])),
                fma(uc[2], s[0], -(uc[0] * s[2])),
                fma(uc[0], s[1], -(uc[1] * s[0]))};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        du[a] = fma(R(2), hE[a], rot[a]);
        u[a] = (um[a] + rot[a]) + hE[a];
    }
}

}  // namespace pl
