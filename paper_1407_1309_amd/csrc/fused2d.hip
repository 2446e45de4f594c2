// fused2d.hip -- all passes of a 2-D MPDATA step in one launch.
//
// Design (gfx950, wave64):
//   * one wavefront owns a strip of 64 consecutive columns (the contiguous
//     dimension, so every row load is one coalesced 256/512-byte access) and
//     marches down a chunk of rows;
//   * every stage of every pass (donor-cell fluxes, pseudo-velocities, limiter
//     bounds and coefficients, limited velocities, corrective fluxes) is kept
//     in per-lane register row-queues, one row per iteration, so each input
//     row is read from memory once and nothing intermediate leaves the CU;
//   * column neighbours come from wave-wide DPP lane shifts (no LDS, no
//     barriers); the outer H lanes of the strip are a recomputed halo, with H
//     the horizontal dependency radius of the step;
//   * the row pipeline is skewed: pass k lags its input by two rows, so the
//     last pass emits row t - LAG while row t is being loaded.
// Periodic boundaries are handled by wrapping row and column indices of the
// loads; the halo lanes and warm-up rows recompute wrapped cells, which is
// exact because the step is translation-equivariant.
#include "common.hpp"
#include "kernels.hpp"

namespace mp {
namespace {

constexpr int WAVE = 64;

// ---- wave-wide lane shifts --------------------------------------------
// from_left(v): lane l receives lane l-1's v (the value at column j-1);
// from_right(v): lane l receives lane l+1's v (column j+1).  Lanes with no
// source receive 0 (they are halo lanes).  Default: DPP wave shifts
// (wave_shr:1 / wave_shl:1, VALU only); MP_SHIFT_BPERMUTE selects the
// ds_bpermute crossbar instead.
#ifndef MP_SHIFT_BPERMUTE
__device__ inline int lane_from_left(int v) { return __builtin_amdgcn_mov_dpp(v, 0x138, 0xf, 0xf, true); }
__device__ inline int lane_from_right(int v) { return __builtin_amdgcn_mov_dpp(v, 0x130, 0xf, 0xf, true); }
#else
__device__ inline int lane_from_left(int v)
{
    int l = (int)(threadIdx.x & (WAVE - 1));
    int r = __builtin_amdgcn_ds_bpermute(((l + WAVE - 1) & (WAVE - 1)) << 2, v);
    return l == 0 ? 0 : r;
}
__device__ inline int lane_from_right(int v)
{
    int l = (int)(threadIdx.x & (WAVE - 1));
    int r = __builtin_amdgcn_ds_bpermute(((l + 1) & (WAVE - 1)) << 2, v);
    return l == WAVE - 1 ? 0 : r;
}
#endif
__device__ inline float from_left(float v) { return __int_as_float(lane_from_left(__float_as_int(v))); }
__device__ inline float from_right(float v) { return __int_as_float(lane_from_right(__float_as_int(v))); }
__device__ inline double from_left(double v)
{
    return __hiloint2double(lane_from_left(__double2hiint(v)), lane_from_left(__double2loint(v)));
}
__device__ inline double from_right(double v)
{
    return __hiloint2double(lane_from_right(__double2hiint(v)), lane_from_right(__double2loint(v)));
}

template <typename T> __device__ inline T frac(T num, T den)
{
    return den == T(0) ? T(0) : num / den;
}

// ---- one corrective pass --------------------------------------------------
// Row bookkeeping for a pass whose newest input row is a:
//   x rows a-3..a, x(j-1) rows a-2..a, x(j+1) rows a-1..a,
//   input advector walls a-1, a (dimension 0) and rows a-1, a (dimension 1),
//   raw V0 at walls a-1, a, limiter bounds rows a-2..a,
//   limiter coefficients rows a-2, a-1,
//   output advector walls/rows a-3, a-2, a-1.
// Per iteration it computes V0 at wall a and V1 at row a-1, the limiter at
// row a-1, the limited velocities at wall a-1 / row a-1, and the corrected
// field at row a-2.
template <typename T> struct Pass {
    T xq[4], xl[3], xr[2];
    T c0q[2], c1q[2];
    T v0q[2];
    T mxq[3], mnq[3];
    T buq[2], bdq[2];
    T aq0[3], aq1[3];

    __device__ void init()
    {
#pragma unroll
        for (int k = 0; k < 4; k++) xq[k] = T(0);
#pragma unroll
        for (int k = 0; k < 3; k++) xl[k] = mxq[k] = mnq[k] = aq0[k] = aq1[k] = T(0);
#pragma unroll
        for (int k = 0; k < 2; k++) xr[k] = c0q[k] = c1q[k] = v0q[k] = buq[k] = bdq[k] = T(0);
    }

    // x_new: row a of the previous pass's result; c0_new / c1_new: the
    // previous pass's advector at wall a / row a; pn_a: psi^n at row a.
    template <bool FCT> __device__ T advance(T x_new, T c0_new, T c1_new, T pn_a)
    {
        xq[0] = xq[1];
        xq[1] = xq[2];
        xq[2] = xq[3];
        xq[3] = x_new;
        xl[0] = xl[1];
        xl[1] = xl[2];
        xl[2] = from_left(x_new);
        xr[0] = xr[1];
        xr[1] = from_right(x_new);
        c0q[0] = c0q[1];
        c0q[1] = c0_new;
        c1q[0] = c1q[1];
        c1q[1] = c1_new;

        // V0 at wall a (rows a-1 | a), column j
        T v0;
        {
            T xL = xq[2], xR = xq[3];
            T u = c0q[1];
            T A = frac(xR - xL, xR + xL);
            T s1 = c1q[0] + c1q[1];
            T cb = T(0.25) * (s1 + from_right(s1));
            T a = xr[1], b = xr[0], e = xl[2], f = xl[1];
            T B = frac(a + b - e - f, a + b + e + f);
            v0 = (fabs(u) - u * u) * A;
            v0 -= T(0.5) * u * cb * B;
        }
        // V1 at row a-1, wall j (columns j-1 | j)
        T v1;
        {
            T xL = xl[1], xR = xq[2];
            T u = c1q[0];
            T A = frac(xR - xL, xR + xL);
            T s0 = c0q[0] + c0q[1];
            T cb = T(0.25) * (from_left(s0) + s0);
            T a = xq[3], b = xl[2], e = xq[1], f = xl[0];
            T B = frac(a + b - e - f, a + b + e + f);
            v1 = (fabs(u) - u * u) * A;
            v1 -= T(0.5) * u * cb * B;
        }
        v0q[0] = v0q[1];
        v0q[1] = v0;

        T lim0, lim1;
        if (FCT) {
            // local bounds over {psi^n, x} at the cell and its face neighbours
            mxq[0] = mxq[1];
            mxq[1] = mxq[2];
            mxq[2] = fmax(pn_a, xq[3]);
            mnq[0] = mnq[1];
            mnq[1] = mnq[2];
            mnq[2] = fmin(pn_a, xq[3]);
            T mx = fmax(fmax(mxq[1], fmax(mxq[0], mxq[2])),
                        fmax(from_left(mxq[1]), from_right(mxq[1])));
            T mn = fmin(fmin(mnq[1], fmin(mnq[0], mnq[2])),
                        fmin(from_left(mnq[1]), from_right(mnq[1])));
            // in/out fluxes of cell (a-1, j)
            T xc = xq[2];
            T v0lo = v0q[0], v0hi = v0q[1];
            T v1lo = v1, v1hi = from_right(v1);
            T fin = (pos(v0lo) * xq[1] - neg(v0hi) * xq[3]) +
                    (pos(v1lo) * xl[1] - neg(v1hi) * xr[0]);
            T fout = (pos(v0hi) * xc - neg(v0lo) * xc) + (pos(v1hi) * xc - neg(v1lo) * xc);
            T bu = fin > T(0) ? (mx - xc) / fin : T(1);
            T bd = fout > T(0) ? (xc - mn) / fout : T(1);
            buq[0] = buq[1];
            buq[1] = bu;
            bdq[0] = bdq[1];
            bdq[1] = bd;
            // limited V1 at row a-1, wall j: L = (a-1, j-1), R = (a-1, j)
            {
                T up = fmin(fmin(T(1), from_left(bd)), bu);
                T dn = fmin(fmin(T(1), from_left(bu)), bd);
                lim1 = pos(v1) * up + neg(v1) * dn;
            }
            // limited V0 at wall a-1: L = (a-2, j), R = (a-1, j)
            {
                T v = v0q[0];
                T up = fmin(fmin(T(1), bdq[0]), buq[1]);
                T dn = fmin(fmin(T(1), buq[0]), bdq[1]);
                lim0 = pos(v) * up + neg(v) * dn;
            }
        } else {
            lim0 = v0q[0];
            lim1 = v1;
        }
        aq0[0] = aq0[1];
        aq0[1] = aq0[2];
        aq0[2] = lim0;
        aq1[0] = aq1[1];
        aq1[1] = aq1[2];
        aq1[2] = lim1;

        // corrective donor-cell pass at row a-2
        T x = xq[1];
        T f0lo = pos(aq0[1]) * xq[0] + neg(aq0[1]) * x;
        T f0hi = pos(aq0[2]) * x + neg(aq0[2]) * xq[2];
        T f1lo = pos(aq1[1]) * xl[0] + neg(aq1[1]) * x;
        T f1hi = from_right(f1lo);
        return x - ((f0hi - f0lo) + (f1hi - f1lo));
    }
};

template <int NI, bool FCT> struct Cfg {
    static constexpr int NP = NI - 1;                 // corrective passes
    static constexpr int H = 1 + (FCT ? 2 : 1) * NP;  // horizontal halo (lanes)
    static constexpr int LAG = 1 + 2 * NP;            // output row = t - LAG
    static constexpr int QP = (2 * NI > 3) ? 2 * NI : 3;  // psi^n rows kept
    static constexpr int OW = WAVE - 2 * H;           // output columns per strip
};

// Prefetch distance (rows in flight ahead of the one being consumed).
constexpr int PF = 2;

template <typename T, int NI, bool FCT>
__device__ __forceinline__ void strip_body(int n0, int n1, const T *__restrict__ psi_n,
                                           T *__restrict__ psi_out, const T *__restrict__ c0,
                                           const T *__restrict__ c1, int jstrip0, int i0, int i1)
{
    using C = Cfg<NI, FCT>;
    const int lane = threadIdx.x & (WAVE - 1);
    // global column of this lane (may lie outside [0, n1) in the halo)
    const int col = jstrip0 - C::H + lane;
    int jj = col % n1;
    if (jj < 0) jj += n1;

    T pq[C::QP];
#pragma unroll
    for (int k = 0; k < C::QP; k++) pq[k] = T(0);
    T dc0[2] = {T(0), T(0)}, dc1[2] = {T(0), T(0)};
    Pass<T> ps[C::NP > 0 ? C::NP : 1];
#pragma unroll
    for (int k = 0; k < C::NP; k++) ps[k].init();

    const int t_begin = i0 - C::LAG - 1;
    const int t_end = i1 - 1 + C::LAG;    // inclusive
    // row (mod n0) of the next row to load, and its row pointers
    int rr = t_begin % n0;
    if (rr < 0) rr += n0;
    const int64_t ld1 = (int64_t)n1 + 1;
    const T *prow = psi_n + (int64_t)rr * n1;
    const T *c0row = c0 + (int64_t)rr * n1;
    const T *c1row = c1 + (int64_t)rr * ld1;

    // prefetch queue: rows t .. t+PF-1
    T fp[PF], f0[PF], f1[PF];
#pragma unroll
    for (int k = 0; k < PF; k++) {
        fp[k] = prow[jj];
        f0[k] = c0row[jj];
        f1[k] = c1row[jj];
        if (++rr == n0) {
            rr = 0;
            prow = psi_n;
            c0row = c0;
            c1row = c1;
        } else {
            prow += n1;
            c0row += n1;
            c1row += ld1;
        }
    }

    const bool out_lane = lane >= C::H && lane < WAVE - C::H && col < n1;
    T *orow = psi_out + (int64_t)i0 * n1 + (out_lane ? col : 0);

    for (int t = t_begin; t <= t_end; t++) {
        T p_new = fp[0], c0_new = f0[0], c1_new = f1[0];
#pragma unroll
        for (int k = 0; k < PF - 1; k++) {
            fp[k] = fp[k + 1];
            f0[k] = f0[k + 1];
            f1[k] = f1[k + 1];
        }
        fp[PF - 1] = prow[jj];
        f0[PF - 1] = c0row[jj];
        f1[PF - 1] = c1row[jj];
        if (++rr == n0) {
            rr = 0;
            prow = psi_n;
            c0row = c0;
            c1row = c1;
        } else {
            prow += n1;
            c0row += n1;
            c1row += ld1;
        }

#pragma unroll
        for (int k = 0; k < C::QP - 1; k++) pq[k] = pq[k + 1];
        pq[C::QP - 1] = p_new;
        dc0[0] = dc0[1];
        dc0[1] = c0_new;
        dc1[0] = dc1[1];
        dc1[1] = c1_new;

        // donor-cell pass at row t-1
        T x = pq[C::QP - 2];
        T f0lo = pos(dc0[0]) * pq[C::QP - 3] + neg(dc0[0]) * x;
        T f0hi = pos(dc0[1]) * x + neg(dc0[1]) * pq[C::QP - 1];
        T f1lo = pos(dc1[0]) * from_left(x) + neg(dc1[0]) * x;
        T f1hi = from_right(f1lo);
        T y = x - ((f0hi - f0lo) + (f1hi - f1lo));
        T cn0 = dc0[0], cn1 = dc1[0];

#pragma unroll
        for (int k = 0; k < C::NP; k++) {
            // pass m = k+2 takes input row a = t - 1 - 2k (psi^n row a sits at
            // pq index QP - 2 - 2k).  Its first input row inside the dependency
            // cone of output row i0 is i0 - 2(NI - m + 1), reached at iteration
            // i0 - 2 NI + 4 m - 5; earlier iterations of this pass are skipped
            // (the queues then hold only rows outside the cone).
            if (t < i0 - 2 * NI + 4 * (k + 2) - 5) break;
            T yk = ps[k].template advance<FCT>(y, cn0, cn1, pq[C::QP - 2 - 2 * k]);
            cn0 = ps[k].aq0[1];
            cn1 = ps[k].aq1[1];
            y = yk;
        }

        if (t - C::LAG >= i0) {
            if (out_lane) *orow = y;
            orow += n1;
        }
    }
}

template <typename T, int NI, bool FCT>
__global__ void __launch_bounds__(WAVE) k_fused2d(int n0, int n1, int th, int strips,
                                                  const T *__restrict__ psi_n,
                                                  T *__restrict__ psi_out,
                                                  const T *__restrict__ c0,
                                                  const T *__restrict__ c1)
{
    using C = Cfg<NI, FCT>;
    int b = blockIdx.x;
    int strip = b % strips, chunk = b / strips;
    int i0 = chunk * th;
    int i1 = i0 + th < n0 ? i0 + th : n0;
    strip_body<T, NI, FCT>(n0, n1, psi_n, psi_out, c0, c1, strip * C::OW, i0, i1);
}

template <typename T, int NI, bool FCT>
__global__ void __launch_bounds__(WAVE) k_fused2d_batched(const BatchGrid *__restrict__ grids,
                                                          int n_grids, int th,
                                                          const T *__restrict__ psi_n,
                                                          T *__restrict__ psi_out,
                                                          const T *__restrict__ c0,
                                                          const T *__restrict__ c1)
{
    using C = Cfg<NI, FCT>;
    int b = blockIdx.x;
    // grid owning tile b: last grid with tile_begin <= b
    int lo = 0, hi = n_grids - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (grids[mid].tile_begin <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    const BatchGrid g = grids[lo];
    int local = b - g.tile_begin;
    int strip = local % g.tiles_w, chunk = local / g.tiles_w;
    int n0 = (int)g.n0, n1 = (int)g.n1;
    int i0 = chunk * th;
    int i1 = i0 + th < n0 ? i0 + th : n0;
    strip_body<T, NI, FCT>(n0, n1, psi_n + g.off_psi, psi_out + g.off_psi, c0 + g.off_c0,
                           c1 + g.off_c1, strip * C::OW, i0, i1);
}

// default rows per chunk (when not tuned): about two waves per SIMD, so the
// chip is full while the warm-up rows stay a modest fraction
int64_t rows_per_chunk(int64_t n0, int64_t strips)
{
    int64_t target_waves = 2048;
    int64_t chunks = target_waves / (strips > 0 ? strips : 1);
    if (chunks < 1) chunks = 1;
    int64_t th = cdiv(n0, chunks);
    if (th < 32) th = 32;
    return th;
}

template <typename T, int NI, bool FCT>
hipError_t launch(const Fused2DShape &sh, const T *psi_n, T *psi_out, const T *c0, const T *c1,
                  hipStream_t s)
{
    using C = Cfg<NI, FCT>;
    int64_t strips = cdiv(sh.n1, C::OW);
    int64_t th = sh.tile_rows > 0 ? sh.tile_rows : rows_per_chunk(sh.n0, strips);
    if (th > sh.n0) th = sh.n0;
    int64_t chunks = cdiv(sh.n0, th);
    int64_t blocks = strips * chunks;
    k_fused2d<T, NI, FCT><<<(unsigned)blocks, WAVE, 0, s>>>((int)sh.n0, (int)sh.n1, (int)th,
                                                           (int)strips, psi_n, psi_out, c0, c1);
    return hipGetLastError();
}

template <typename T, int NI, bool FCT>
hipError_t launch_batched(const BatchGrid *g, int n_grids, int n_tiles, const T *psi_n,
                          T *psi_out, const T *c0, const T *c1, hipStream_t s)
{
    k_fused2d_batched<T, NI, FCT><<<(unsigned)n_tiles, WAVE, 0, s>>>(
        g, n_grids, fused2d_tile_rows(), psi_n, psi_out, c0, c1);
    return hipGetLastError();
}

}  // namespace

bool fused2d_supported(int nd, int n_iters, unsigned opts, int has_g, int bc0, int bc1)
{
    if (nd != 2 || has_g || bc0 != BC_PERIODIC || bc1 != BC_PERIODIC) return false;
    if (opts & ~OPT_FCT) return false;          // tot / iga: staged path
    return n_iters >= 1 && n_iters <= 4;
}

int fused2d_tile_rows() { return 64; }

int fused2d_strip_cols(int n_iters, unsigned opts)
{
    int np = n_iters - 1;
    int h = 1 + ((opts & OPT_FCT) ? 2 : 1) * np;
    return WAVE - 2 * h;
}

template <typename T>
hipError_t fused2d_step(const Fused2DShape &sh, int n_iters, unsigned opts, const T *psi_n,
                        T *psi_out, const T *c0, const T *c1, const T *G, hipStream_t s)
{
    if (G || sh.bc0 != BC_PERIODIC || sh.bc1 != BC_PERIODIC) return hipErrorNotSupported;
    bool fct = opts & OPT_FCT;
    switch (n_iters * 2 + (fct ? 1 : 0)) {
    case 2: case 3: return launch<T, 1, false>(sh, psi_n, psi_out, c0, c1, s);
    case 4: return launch<T, 2, false>(sh, psi_n, psi_out, c0, c1, s);
    case 5: return launch<T, 2, true>(sh, psi_n, psi_out, c0, c1, s);
    case 6: return launch<T, 3, false>(sh, psi_n, psi_out, c0, c1, s);
    case 7: return launch<T, 3, true>(sh, psi_n, psi_out, c0, c1, s);
    case 8: return launch<T, 4, false>(sh, psi_n, psi_out, c0, c1, s);
    case 9: return launch<T, 4, true>(sh, psi_n, psi_out, c0, c1, s);
    default: return hipErrorNotSupported;
    }
}

template <typename T>
hipError_t fused2d_batched_step(const BatchGrid *g, int n_grids, int n_tiles, int bc,
                                int n_iters, unsigned opts, const T *psi_n, T *psi_out,
                                const T *c0, const T *c1, hipStream_t s)
{
    if (bc != BC_PERIODIC) return hipErrorNotSupported;
    bool fct = opts & OPT_FCT;
    switch (n_iters * 2 + (fct ? 1 : 0)) {
    case 2: case 3: return launch_batched<T, 1, false>(g, n_grids, n_tiles, psi_n, psi_out, c0, c1, s);
    case 4: return launch_batched<T, 2, false>(g, n_grids, n_tiles, psi_n, psi_out, c0, c1, s);
    case 5: return launch_batched<T, 2, true>(g, n_grids, n_tiles, psi_n, psi_out, c0, c1, s);
    case 6: return launch_batched<T, 3, false>(g, n_grids, n_tiles, psi_n, psi_out, c0, c1, s);
    case 7: return launch_batched<T, 3, true>(g, n_grids, n_tiles, psi_n, psi_out, c0, c1, s);
    case 8: return launch_batched<T, 4, false>(g, n_grids, n_tiles, psi_n, psi_out, c0, c1, s);
    case 9: return launch_batched<T, 4, true>(g, n_grids, n_tiles, psi_n, psi_out, c0, c1, s);
    default: return hipErrorNotSupported;
    }
}

template hipError_t fused2d_step<float>(const Fused2DShape &, int, unsigned, const float *, float *,
                                        const float *, const float *, const float *, hipStream_t);
template hipError_t fused2d_step<double>(const Fused2DShape &, int, unsigned, const double *,
                                         double *, const double *, const double *, const double *,
                                         hipStream_t);
template hipError_t fused2d_batched_step<float>(const BatchGrid *, int, int, int, int, unsigned,
                                                const float *, float *, const float *,
                                                const float *, hipStream_t);
template hipError_t fused2d_batched_step<double>(const BatchGrid *, int, int, int, int, unsigned,
                                                 const double *, double *, const double *,
                                                 const double *, hipStream_t);

}  // namespace mp
