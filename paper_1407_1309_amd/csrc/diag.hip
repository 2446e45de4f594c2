// diag.hip -- conservation / extrema / non-finite diagnostics and the
// Courant-number check.
//
// Two-level deterministic reduction: a fixed grid of blocks writes one
// partial each (FP64 Neumaier-compensated sum, min, max, non-finite count;
// wavefront butterflies inside a block), one block combines the partials in
// index order.  The result does not depend on scheduling.
#include <math.h>

#include "common.hpp"
#include "kernels.hpp"

namespace mp {
namespace {

constexpr int DB = 256;          // threads per block
constexpr int DMAX_BLOCKS = 1024;

struct Acc {
    double s, c, mn, mx, bad;
};

__device__ inline void two_sum(double a, double b, double &s, double &e)
{
    s = a + b;
    double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

__device__ inline void acc_add(Acc &A, double term)
{
    double t = A.s + term;  // Neumaier
    if (fabs(A.s) >= fabs(term))
        A.c += (A.s - t) + term;
    else
        A.c += (term - t) + A.s;
    A.s = t;
}

__device__ inline void acc_merge(Acc &A, const Acc &B)
{
    double s, e;
    two_sum(A.s, B.s, s, e);
    A.s = s;
    A.c = A.c + B.c + e;
    A.mn = fmin(A.mn, B.mn);
    A.mx = fmax(A.mx, B.mx);
    A.bad += B.bad;
}

// Reduction of one block's accumulators: a butterfly within each wavefront
// (lane-to-lane exchanges, no LDS), then the waves' results merged in wave
// order by the first wave.  The data flow is fixed, so the result does not
// depend on scheduling.
__device__ inline Acc lane_xor(const Acc &A, int m)
{
    return {__shfl_xor(A.s, m), __shfl_xor(A.c, m), __shfl_xor(A.mn, m), __shfl_xor(A.mx, m),
            __shfl_xor(A.bad, m)};
}

__device__ void block_reduce(Acc &A)
{
    constexpr int W = 64, NW = DB / W;
    __shared__ double sh[5][NW];
#pragma unroll
    for (int m = W / 2; m > 0; m >>= 1) {
        const Acc B = lane_xor(A, m);
        acc_merge(A, B);
    }
    const int t = threadIdx.x, w = t / W;
    if ((t % W) == 0) {
        sh[0][w] = A.s;
        sh[1][w] = A.c;
        sh[2][w] = A.mn;
        sh[3][w] = A.mx;
        sh[4][w] = A.bad;
    }
    __syncthreads();
    if (t == 0) {
        A = {sh[0][0], sh[1][0], sh[2][0], sh[3][0], sh[4][0]};
        for (int k = 1; k < NW; k++) {
            const Acc B = {sh[0][k], sh[1][k], sh[2][k], sh[3][k], sh[4][k]};
            acc_merge(A, B);
        }
    }
    __syncthreads();
}

template <typename T>
__global__ void __launch_bounds__(DB) k_diag_part(const T *psi, const T *G, int64_t N,
                                                  double *part)
{
    Acc A = {0.0, 0.0, INFINITY, -INFINITY, 0.0};
    int64_t stride = (int64_t)gridDim.x * DB;
    for (int64_t k = (int64_t)blockIdx.x * DB + threadIdx.x; k < N; k += stride) {
        double v = (double)psi[k];
        if (!isfinite(v)) {
            A.bad += 1.0;
            continue;
        }
        acc_add(A, G ? (double)G[k] * v : v);
        A.mn = fmin(A.mn, v);
        A.mx = fmax(A.mx, v);
    }
    block_reduce(A);
    if (threadIdx.x == 0) {
        double *p = part + 5 * blockIdx.x;
        p[0] = A.s;
        p[1] = A.c;
        p[2] = A.mn;
        p[3] = A.mx;
        p[4] = A.bad;
    }
}

__global__ void __launch_bounds__(DB) k_diag_final(const double *part, int nparts, double *out)
{
    Acc A = {0.0, 0.0, INFINITY, -INFINITY, 0.0};
    // each thread merges a contiguous run of partials, in index order
    int per = (nparts + DB - 1) / DB;
    int b = threadIdx.x * per, e = min(nparts, b + per);
    for (int i = b; i < e; i++) {
        const double *p = part + 5 * i;
        Acc B = {p[0], p[1], p[2], p[3], p[4]};
        acc_merge(A, B);
    }
    block_reduce(A);
    if (threadIdx.x == 0) {
        out[0] = A.s + A.c;
        out[1] = A.mn;
        out[2] = A.mx;
        out[3] = A.bad;
    }
}

template <typename T>
__global__ void __launch_bounds__(DB) k_courant_part(Geom g, const T *c0, const T *c1,
                                                     const T *c2, const T *G, double *part)
{
    int64_t N = g.n[0] * g.n[1] * g.n[2];
    const T *c[3] = {c0, c1, c2};
    double best = 0.0, bad = 0.0;
    int64_t stride = (int64_t)gridDim.x * DB;
    for (int64_t t = (int64_t)blockIdx.x * DB + threadIdx.x; t < N; t += stride) {
        int64_t p[3];
        int64_t r = t;
        p[2] = r % g.n[2];
        r /= g.n[2];
        p[1] = r % g.n[1];
        p[0] = r / g.n[1];
        double s = 0.0;
        bool fin = true;
        for (int d = 0; d < g.nd; d++) {
            int64_t e[3] = {g.n[0], g.n[1], g.n[2]};
            e[d] += 1;
            int64_t q[3] = {p[0], p[1], p[2]};
            int64_t lo = (q[0] * e[1] + q[1]) * e[2] + q[2];
            q[d] = map_wall(p[d] + 1, g.n[d], g.bc[d]);
            int64_t hi = (q[0] * e[1] + q[1]) * e[2] + q[2];
            const double a = fabs((double)c[d][lo]), b = fabs((double)c[d][hi]);
            fin = fin && isfinite(a + b);      // fmax alone would pass over a NaN
            s += fmax(a, b);
        }
        if (G) {
            const double gt = (double)G[t];
            fin = fin && isfinite(gt);
            s /= gt;
        }
        if (!fin || !isfinite(s)) {
            bad += 1.0;
            continue;
        }
        best = fmax(best, s);
    }
    Acc A = {0.0, 0.0, INFINITY, best, bad};
    block_reduce(A);
    if (threadIdx.x == 0) {
        part[5 * blockIdx.x + 3] = A.mx;
        part[5 * blockIdx.x + 4] = A.bad;
    }
}

// out[0] = largest finite Courant sum, out[1] = cells with a non-finite one
__global__ void __launch_bounds__(DB) k_courant_final(const double *part, int nparts, double *out)
{
    double best = 0.0, bad = 0.0;
    for (int i = threadIdx.x; i < nparts; i += DB) {
        best = fmax(best, part[5 * i + 3]);
        bad += part[5 * i + 4];
    }
    Acc A = {0.0, 0.0, INFINITY, best, bad};
    block_reduce(A);
    if (threadIdx.x == 0) {
        out[0] = A.mx;
        out[1] = A.bad;
    }
}

int blocks_for(int64_t N)
{
    int64_t b = cdiv(N, (int64_t)DB * 8);
    if (b < 1) b = 1;
    if (b > DMAX_BLOCKS) b = DMAX_BLOCKS;
    return (int)b;
}

}  // namespace

int diag_max_blocks() { return DMAX_BLOCKS; }

template <typename T>
hipError_t diag_launch(const T *psi, const T *G, int64_t N, double *part, double *out,
                       hipStream_t s)
{
    int nb = blocks_for(N);
    k_diag_part<T><<<nb, DB, 0, s>>>(psi, G, N, part);
    k_diag_final<<<1, DB, 0, s>>>(part, nb, out);
    return hipGetLastError();
}

hipError_t diag_final_launch(const double *part, int nparts, double *out, hipStream_t s)
{
    k_diag_final<<<1, DB, 0, s>>>(part, nparts, out);
    return hipGetLastError();
}

template <typename T>
hipError_t courant_launch(const Geom &g, const T *c0, const T *c1, const T *c2, const T *G,
                          double *part, double *out, hipStream_t s)
{
    int nb = blocks_for(g.n[0] * g.n[1] * g.n[2]);
    k_courant_part<T><<<nb, DB, 0, s>>>(g, c0, c1, c2, G, part);
    k_courant_final<<<1, DB, 0, s>>>(part, nb, out);
    return hipGetLastError();
}

template hipError_t diag_launch<float>(const float *, const float *, int64_t, double *, double *,
                                       hipStream_t);
template hipError_t diag_launch<double>(const double *, const double *, int64_t, double *,
                                        double *, hipStream_t);
template hipError_t courant_launch<float>(const Geom &, const float *, const float *,
                                          const float *, const float *, double *, double *,
                                          hipStream_t);
template hipError_t courant_launch<double>(const Geom &, const double *, const double *,
                                           const double *, const double *, double *, double *,
                                           hipStream_t);

}  // namespace mp
