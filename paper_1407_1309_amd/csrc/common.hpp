// common.hpp -- grid geometry, boundary map and small helpers shared by the
// libmpdata kernels (HIP, gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mp {

enum { BC_PERIODIC = 0, BC_OPEN = 1 };
enum { OPT_FCT = 1u, OPT_IGA = 2u, OPT_TOT = 4u, OPT_ABS = 8u, OPT_DFL = 16u, OPT_KAHAN = 32u };

// Grid extents padded with 1 beyond n_dims; boundary type per dimension.
struct Geom {
    int nd;
    int64_t n[3];
    int bc[3];
};

// Boundary map (Sect. 2.2): periodic wraps, open clamps.  Cells live in
// [0, n), walls of the dimension's own advector component in [0, n]; with
// periodic boundaries wall n is wall 0.
__host__ __device__ inline int64_t map_cell(int64_t q, int64_t n, int bc)
{
    if (bc == BC_PERIODIC) {
        q %= n;
        return q < 0 ? q + n : q;
    }
    return q < 0 ? 0 : (q >= n ? n - 1 : q);
}

__host__ __device__ inline int64_t map_wall(int64_t f, int64_t n, int bc)
{
    if (bc == BC_PERIODIC) {
        f %= n;
        return f < 0 ? f + n : f;
    }
    return f < 0 ? 0 : (f > n ? n : f);
}

// Single-wrap variants for coordinates at most one period outside the range
// (q in (-n, 2n)), which is all the stencils need: 32-bit, no division.
__host__ __device__ inline int wrap_cell(int q, int n, int bc)
{
    if (bc == BC_PERIODIC) return q < 0 ? q + n : (q >= n ? q - n : q);
    return q < 0 ? 0 : (q >= n ? n - 1 : q);
}

__host__ __device__ inline int wrap_wall(int f, int n, int bc)
{
    if (bc == BC_PERIODIC) return f < 0 ? f + n : (f >= n ? f - n : f);
    return f < 0 ? 0 : (f > n ? n : f);
}

// Coordinates of flat index t in a row-major box of extents e (32-bit
// arithmetic when the box has fewer than 2^31 entries).
__device__ inline void unflat3(int64_t t, const int64_t e[3], int v[3])
{
    if (e[0] * e[1] * e[2] < ((int64_t)1 << 31)) {
        unsigned u = (unsigned)t, e2 = (unsigned)e[2], e1 = (unsigned)e[1];
        v[2] = (int)(u % e2);
        u /= e2;
        v[1] = (int)(u % e1);
        v[0] = (int)(u / e1);
    } else {
        v[2] = (int)(t % e[2]);
        t /= e[2];
        v[1] = (int)(t % e[1]);
        v[0] = (int)(t / e[1]);
    }
}

template <typename T> __device__ inline T pos(T u) { return u > T(0) ? u : T(0); }
template <typename T> __device__ inline T neg(T u) { return u < T(0) ? u : T(0); }

// Donor-cell flux of eq. F across a wall with advector u, between the cell
// below the wall (value xl) and the cell above it (xr): [u]+ xl + [u]- xr.
// Formed as a product with u, so that a NaN or infinite advector makes the
// flux, and with it the two cells beside the wall, non-finite: the sum form
// with [u]+ = max(u, 0) and [u]- = min(u, 0) turns a NaN advector into 0
// and hides it from the diagnostics.  For finite values the two forms are
// equal (the dropped product of the sum is a signed zero).  upwind() keeps
// the derivative with respect to u at u = 0 equal to 0 (the kink convention
// of the reverse mode) when T is a dual number; upwind_fp() is the plain
// floating-point form, where at u = 0 either cell gives +-0.
template <typename T> __device__ inline T upwind(T u, T xl, T xr)
{
    return u * (u > T(0) ? xl : (u < T(0) ? xr : T(0)));
}
template <typename T> __device__ __forceinline__ T upwind_fp(T u, T xl, T xr)
{
    return u * (u > T(0) ? xl : xr);
}

// Quotients.
// FP64: the quotients of a stage are formed together.  When every lane's
// divisors are zero or normal and below 2^1000 in magnitude (a wave-uniform
// test), each quotient is n * r with r the hardware reciprocal (about 2^-23
// accurate) refined by one Newton step: within 18 ulp of the rounded
// quotient (measured over 2^20 random operands), four instructions instead
// of the eleven of the IEEE sequence.  Otherwise the whole wave takes the
// IEEE division.  A zero divisor's quotient is discarded by every caller.
// FP32: the hardware reciprocal refined by one Newton step when the divisor
// is normal or zero (a per-lane branch, cheap in FP32), else the IEEE
// division.
template <int K> __device__ __forceinline__ void quotients(const double (&n)[K],
                                                          const double (&d)[K], double (&q)[K])
{
    bool ok = true;
#pragma unroll
    for (int k = 0; k < K; k++)
        ok = ok && __builtin_amdgcn_class(d[k], 0x168) && fabs(d[k]) < 0x1p1000;
    if (__builtin_amdgcn_ballot_w64(!ok) == 0) {
#pragma unroll
        for (int k = 0; k < K; k++) {
            double r = __builtin_amdgcn_rcp(d[k]);
            r = fma(fma(-d[k], r, 1.0), r, r);
            q[k] = n[k] * r;
        }
    } else {
#pragma unroll
        for (int k = 0; k < K; k++) q[k] = n[k] / d[k];
    }
}

__device__ inline float qdiv(float n, float d)
{
    if (__builtin_amdgcn_classf(d, 0x168)) {      // +-normal or +-zero
        float r = __builtin_amdgcn_rcpf(d);
        float q = n * r;
        return fmaf(fmaf(-d, q, n), r, q);
    }
    return n / d;
}

template <int K> __device__ __forceinline__ void quotients(const float (&n)[K],
                                                         const float (&d)[K], float (&q)[K])
{
#pragma unroll
    for (int k = 0; k < K; k++) q[k] = qdiv(n[k], d[k]);
}

// s += t with Kahan's compensated summation (compensation c starts at 0):
// y = t - c, u = s + y, c = (u - s) - y, s = u.  No contraction into FMAs.
template <typename T> __device__ __forceinline__ void kahan_add(T &s, T &c, T t)
{
#pragma clang fp contract(off)
    T y = t - c;
    T u = s + y;
    c = (u - s) - y;
    s = u;
}

// Round-up integer division.
__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace mp
