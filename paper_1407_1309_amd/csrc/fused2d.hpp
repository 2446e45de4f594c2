// fused2d.hpp -- all passes of a 2-D MPDATA step in one launch (kernel
// templates; fused2d_f32.hip and fused2d_f64.hip instantiate them, so the two
// element types compile in parallel).
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
#pragma once

#include "common.hpp"
#include "kernels.hpp"

// Multiply-add contraction only within one source expression (decided by the
// front end from the source alone).  The kernel body is instantiated twice
// (fast and safe quotient modes, see qset); with contraction left to the
// back end, the two instantiations could fuse different multiply-add pairs
// and round a value differently, and a chunk's bits would depend on whether
// it was recomputed.
#pragma clang fp contract(on)

namespace mp {
namespace {

constexpr int WAVE = 64;

// ---- wave-wide lane shifts --------------------------------------------
// from_left(v): lane l receives lane l-1's v (the value at column j-1);
// from_right(v): lane l receives lane l+1's v (column j+1).  Lanes with no
// source receive 0 (they are halo lanes).  DPP wave shifts (wave_shr:1 /
// wave_shl:1): VALU only, no LDS traffic.
__device__ inline int lane_from_left(int v) { return __builtin_amdgcn_mov_dpp(v, 0x138, 0xf, 0xf, true); }
__device__ inline int lane_from_right(int v) { return __builtin_amdgcn_mov_dpp(v, 0x130, 0xf, 0xf, true); }
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

// Donor-cell update of one cell from the flux differences of the two
// dimensions (G = 1): straightforward x - (d0 + d1), or Kahan-compensated.
template <bool KAHAN, typename T> __device__ __forceinline__ T donor_update(T x, T d0, T d1)
{
    if constexpr (!KAHAN) return x - (d0 + d1);
    T s = x, c = T(0);
    kahan_add(s, c, -d0);
    kahan_add(s, c, -d1);
    return s;
}

// ---- quotient sets ---------------------------------------------------------
// A wave first runs its whole chunk in fast mode: every quotient is n * r
// with r the hardware reciprocal refined by one Newton step (FP64: within 18
// ulp of the rounded quotient; FP32: the residual-corrected form), for every
// lane and with no branch, so each row stays one long straight-line region
// for the instruction scheduler.  `keep` marks the quotients the caller uses
// (a zero divisor's, or a limiter coefficient's with no in- or out-flux, is
// replaced by a constant).  A kept quotient is in range when
//   FP64: the hardware reciprocal of the divisor is a normal number (so the
//         divisor is neither 2^1022 or more in magnitude, whose reciprocal
//         is subnormal, nor a subnormal the reciprocal cannot invert;
//         one class test of r replaces tests of the divisor's class and
//         magnitude),
//   FP32: the divisor is normal or zero (one class test of the divisor, for
//         kept and discarded quotients alike, which is cheaper there than
//         combining it with the caller's test).
// Fast mode records, wave-uniformly, whether any kept quotient was out of
// range.  A wave with such a record recomputes its chunk in safe mode,
// rewriting every row it stored (the kernel reads only psi^n and the
// advector, so the redo sees the same inputs).  Safe mode decides lane by
// lane with the same test: the fast quotient in range, the IEEE quotient
// elsewhere.  A kept quotient's value therefore depends only on its
// operands, never on which lanes share its wave or where its chunk begins,
// so every tiling (and the batched kernel) gives the same bits.
__device__ __forceinline__ double q_rcp(double d) { return __builtin_amdgcn_rcp(d); }
__device__ __forceinline__ float q_rcp(float d) { return __builtin_amdgcn_rcpf(d); }
__device__ __forceinline__ bool q_in_range(double d, double r)
{
    return __builtin_amdgcn_class(r, 0x108);     // r is +-normal
}
__device__ __forceinline__ bool q_in_range(float d, float)
{
    return __builtin_amdgcn_classf(d, 0x168);    // d is +-normal or +-zero
}
__device__ __forceinline__ double q_fast(double n, double d, double r)
{
    r = fma(fma(-d, r, 1.0), r, r);
    return n * r;
}
__device__ __forceinline__ float q_fast(float n, float d, float r)
{
    const float q0 = n * r;
    return fmaf(fmaf(-d, q0, n), r, q0);
}

template <bool SAFE, int K, typename T>
__device__ __forceinline__ void qset(const T (&n)[K], const T (&d)[K], const bool (&keep)[K],
                                     T (&q)[K], uint64_t &bad)
{
    bool ok = true;
#pragma unroll
    for (int k = 0; k < K; k++) {
        const T r = q_rcp(d[k]);
        const bool in = q_in_range(d[k], r);
        if constexpr (SAFE) {
            q[k] = in ? q_fast(n[k], d[k], r) : n[k] / d[k];
        } else {
            if constexpr (sizeof(T) == 8)
                ok = ok & (in | !keep[k]);     // bitwise: lane masks, no short circuit
            else
                ok = ok && in;
            q[k] = q_fast(n[k], d[k], r);
        }
    }
    if constexpr (!SAFE) bad |= __builtin_amdgcn_ballot_w64(!ok);
}

// ---- register row-queues ------------------------------------------------
// The row loop is unrolled by U iterations and every queue is a ring whose
// depth divides U, so the slot holding "the row pushed `age` iterations ago"
// is a compile-time index for each unrolled iteration (phase P): queues
// advance by renaming registers instead of moving them.
template <int D> __host__ __device__ constexpr int slot(int phase, int age)
{
    return ((phase - age) % D + D) % D;
}

template <typename T, int D> struct Ring {
    T v[D];
    __device__ __forceinline__ void zero()
    {
#pragma unroll
        for (int k = 0; k < D; k++) v[k] = T(0);
    }
};
#define AT(ring, depth, age) (ring).v[slot<depth>(P, (age))]

// ---- one corrective pass --------------------------------------------------
// Row bookkeeping for a pass whose newest input row is a (ages count rows
// back from a):
//   x rows a-3..a, x(j-1) rows a-2..a, x(j+1) rows a-1..a,
//   input advector walls a-1, a (dimension 0) and rows a-1, a (dimension 1),
//   raw V0 at walls a-1, a, limiter bounds rows a-2..a,
//   limiter coefficients rows a-2, a-1,
//   output advector walls/rows a-3, a-2, a-1.
// Per iteration it computes V0 at wall a and V1 at row a-1, the limiter at
// row a-1, the limited velocities at wall a-1 / row a-1, and the corrected
// field at row a-2.
template <typename T> struct Pass {
    Ring<T, 4> xq, xl, mxq, mnq, aq0, aq1;
    Ring<T, 2> xr, c0q, c1q, v0q, buq, bdq;

    __device__ __forceinline__ void init()
    {
        xq.zero(); xl.zero(); mxq.zero(); mnq.zero(); aq0.zero(); aq1.zero();
        xr.zero(); c0q.zero(); c1q.zero(); v0q.zero(); buq.zero(); bdq.zero();
    }

    // x_new: row a of the previous pass's result; c0_new / c1_new: the
    // previous pass's advector at wall a / row a; pn_a: psi^n at row a.
    template <bool FCT, bool ABS, bool KH, bool SAFE, int P>
    __device__ __forceinline__ T advance(T x_new, T c0_new, T c1_new, T pn_a, uint64_t &bad)
    {
        AT(xq, 4, 0) = x_new;
        AT(xl, 4, 0) = from_left(x_new);
        AT(xr, 2, 0) = from_right(x_new);
        AT(c0q, 2, 0) = c0_new;
        AT(c1q, 2, 0) = c1_new;

        // psi-fractions of V0 at wall a (rows a-1 | a), column j, and of V1 at
        // row a-1, wall j (columns j-1 | j): A terms and cross (B) terms
        // (|psi| in every fraction under the abs option)
        auto fa = [](T v) -> T { return ABS ? fabs(v) : v; };
        T num[4], den[4], fr[4];
        {
            T xL = fa(AT(xq, 4, 1)), xR = fa(AT(xq, 4, 0));
            num[0] = xR - xL;
            den[0] = xR + xL;
            T a = fa(AT(xr, 2, 0)), b = fa(AT(xr, 2, 1)), e = fa(AT(xl, 4, 0)), f = fa(AT(xl, 4, 1));
            num[1] = a + b - e - f;
            den[1] = a + b + e + f;
        }
        {
            T xL = fa(AT(xl, 4, 1)), xR = fa(AT(xq, 4, 1));
            num[2] = xR - xL;
            den[2] = xR + xL;
            T a = fa(AT(xq, 4, 0)), b = fa(AT(xl, 4, 0)), e = fa(AT(xq, 4, 2)), f = fa(AT(xl, 4, 2));
            num[3] = a + b - e - f;
            den[3] = a + b + e + f;
        }
        const bool keep[4] = {den[0] != T(0), den[1] != T(0), den[2] != T(0), den[3] != T(0)};
        qset<SAFE, 4>(num, den, keep, fr, bad);
#pragma unroll
        for (int k = 0; k < 4; k++) fr[k] = keep[k] ? fr[k] : T(0);
        T v0;
        {
            T u = AT(c0q, 2, 0);
            T s1 = AT(c1q, 2, 1) + AT(c1q, 2, 0);
            T cb = T(0.25) * (s1 + from_right(s1));
            v0 = (fabs(u) - u * u) * fr[0];
            v0 -= T(0.5) * u * cb * fr[1];
        }
        T v1;
        {
            T u = AT(c1q, 2, 1);
            T s0 = AT(c0q, 2, 1) + AT(c0q, 2, 0);
            T cb = T(0.25) * (from_left(s0) + s0);
            v1 = (fabs(u) - u * u) * fr[2];
            v1 -= T(0.5) * u * cb * fr[3];
        }
        AT(v0q, 2, 0) = v0;

        T lim0, lim1;
        if (FCT) {
            // local bounds over {psi^n, x} at the cell and its face neighbours
            AT(mxq, 4, 0) = fmax(pn_a, AT(xq, 4, 0));
            AT(mnq, 4, 0) = fmin(pn_a, AT(xq, 4, 0));
            T m1 = AT(mxq, 4, 1), n1 = AT(mnq, 4, 1);
            T mx = fmax(fmax(m1, fmax(AT(mxq, 4, 2), AT(mxq, 4, 0))),
                        fmax(from_left(m1), from_right(m1)));
            T mn = fmin(fmin(n1, fmin(AT(mnq, 4, 2), AT(mnq, 4, 0))),
                        fmin(from_left(n1), from_right(n1)));
            // in/out fluxes of cell (a-1, j)
            T xc = AT(xq, 4, 1);
            T v0lo = AT(v0q, 2, 1), v0hi = AT(v0q, 2, 0);
            T v1lo = v1, v1hi = from_right(v1);
            T fin = (pos(v0lo) * AT(xq, 4, 2) - neg(v0hi) * AT(xq, 4, 0)) +
                    (pos(v1lo) * AT(xl, 4, 1) - neg(v1hi) * AT(xr, 2, 1));
            T fout = (pos(v0hi) * xc - neg(v0lo) * xc) + (pos(v1hi) * xc - neg(v1lo) * xc);
            T bn[2] = {mx - xc, xc - mn}, bdv[2] = {fin, fout}, bq[2];
            const bool keep[2] = {fin > T(0), fout > T(0)};
            qset<SAFE, 2>(bn, bdv, keep, bq, bad);
            T bu = keep[0] ? bq[0] : T(1);
            T bd = keep[1] ? bq[1] : T(1);
            AT(buq, 2, 0) = bu;
            AT(bdq, 2, 0) = bd;
            // limited V1 at row a-1, wall j: L = (a-1, j-1), R = (a-1, j)
            {
                T up = fmin(fmin(T(1), from_left(bd)), bu);
                T dn = fmin(fmin(T(1), from_left(bu)), bd);
                lim1 = pos(v1) * up + neg(v1) * dn;
            }
            // limited V0 at wall a-1: L = (a-2, j), R = (a-1, j)
            {
                T v = AT(v0q, 2, 1);
                T up = fmin(fmin(T(1), AT(bdq, 2, 1)), AT(buq, 2, 0));
                T dn = fmin(fmin(T(1), AT(buq, 2, 1)), AT(bdq, 2, 0));
                lim0 = pos(v) * up + neg(v) * dn;
            }
        } else {
            lim0 = AT(v0q, 2, 1);
            lim1 = v1;
        }
        AT(aq0, 4, 0) = lim0;
        AT(aq1, 4, 0) = lim1;

        // corrective donor-cell pass at row a-2
        T x = AT(xq, 4, 2);
        T f0lo = pos(AT(aq0, 4, 1)) * AT(xq, 4, 3) + neg(AT(aq0, 4, 1)) * x;
        T f0hi = pos(AT(aq0, 4, 0)) * x + neg(AT(aq0, 4, 0)) * AT(xq, 4, 1);
        T f1lo = pos(AT(aq1, 4, 1)) * AT(xl, 4, 2) + neg(AT(aq1, 4, 1)) * x;
        T f1hi = from_right(f1lo);
        return donor_update<KH>(x, f0hi - f0lo, f1hi - f1lo);
    }
};

// Row-loop unroll: U = 8 rows per loop trip.  With 4 the register copies
// of the loop-carried prefetch at the back edge made the compiler wait for
// the newest loads (s_waitcnt vmcnt(0)) once per trip, draining the
// two-row prefetch; with 8 the waits stay two rows behind the loads.  The
// rows left over after the last whole trip run in blocks of UT = 4 (every
// ring depth divides 4 when the psi^n ring has depth 4), so a chunk is
// rounded up to a multiple of 4 iterations, not 8.
template <int NI, bool FCT> struct Cfg {
    static constexpr int NP = NI - 1;                 // corrective passes
    static constexpr int H = 1 + (FCT ? 2 : 1) * NP;  // horizontal halo (lanes)
    static constexpr int LAG = 1 + 2 * NP;            // output row = t - LAG
    static constexpr int QP = NI <= 3 ? 4 : 8;        // psi^n ring (ages 0..2NI-3 used)
    static constexpr int U = 8;                       // row-loop unroll
    static constexpr int UT = QP;                     // tail block (divides U)
    static constexpr int OW = WAVE - 2 * H;           // output columns per strip
};

// Prefetch distance (rows in flight ahead of the one being consumed).
constexpr int PF = 2;

// Diagnostics of the cells a lane stores (the conserved sum G psi of Sect. 1
// with G = 1, the extrema, and the non-finite count of the NaN checks of
// Sect. 2.4), accumulated in FP64 with Neumaier's compensation and reduced
// over the wave at the end of a chunk into one partial (sum, compensation,
// min, max, count), the layout of the diagnostics kernels' partials.  A
// non-finite value is recognised from its exponent bits: this file is built
// assuming NaN-free floating-point arithmetic, so no floating-point test is
// trusted to see one.
struct StepDiag {
    double s, c, mn, mx, bad;

    __device__ __forceinline__ void init()
    {
        s = c = bad = 0.0;
        mn = __builtin_huge_val();
        mx = -__builtin_huge_val();
    }
    template <typename T> __device__ __forceinline__ void add(T y, bool on)
    {
        const double v = (double)y;
        // this file is built assuming no NaN arithmetic: the empty asm hides
        // where the bits came from, so the test of them is not folded away
        long long b = __double_as_longlong(v);
        asm volatile("" : "+v"(b));
        const bool nonfin = ((b >> 52) & 0x7ff) == 0x7ff;
        const bool fin = on && !nonfin;
        const double term = fin ? v : 0.0;
        const double t = s + term;
        c += fabs(s) >= fabs(term) ? (s - t) + term : (term - t) + s;
        s = t;
        mn = fin ? fmin(mn, v) : mn;
        mx = fin ? fmax(mx, v) : mx;
        bad += (on && nonfin) ? 1.0 : 0.0;
    }
    // butterfly over the wave (fixed data flow: deterministic); lane 0 writes
    __device__ __forceinline__ void wave_write(double *p)
    {
#pragma unroll
        for (int m = WAVE / 2; m > 0; m >>= 1) {
            const double s2 = __shfl_xor(s, m), c2 = __shfl_xor(c, m), mn2 = __shfl_xor(mn, m),
                         mx2 = __shfl_xor(mx, m), b2 = __shfl_xor(bad, m);
            const double ss = s + s2, bb = ss - s, e = (s - (ss - bb)) + (s2 - bb);
            s = ss;
            c = c + c2 + e;
            mn = fmin(mn, mn2);
            mx = fmax(mx, mx2);
            bad += b2;
        }
        if ((threadIdx.x & (WAVE - 1)) == 0) {
            p[0] = s;
            p[1] = c;
            p[2] = mn;
            p[3] = mx;
            p[4] = bad;
        }
    }
};

// State of one wavefront marching down rows i0..i1-1 of a 64-column strip
// (quotients in fast or safe mode, see qset).
template <typename T, int NI, bool FCT, bool ABS, bool KH, bool DG, bool SAFE> struct Strip {
    using C = Cfg<NI, FCT>;
    int n0, n1, i0, i1, jj, rr;
    int64_t ld1;
    bool out_lane;
    uint64_t bad;      // fast mode: lanes whose divisors left the fast range
    const T *psi_n, *c0, *c1;
    const T *prow, *c0row, *c1row;
    T *orow;
    Ring<T, C::QP> pq;
    Ring<T, 2> dc0, dc1;
    T fp[PF], f0[PF], f1[PF];
    Pass<T> ps[C::NP > 0 ? C::NP : 1];
    StepDiag dg;       // DG: diagnostics of the cells this lane stores

    // advance the load pointers one row, wrapping at n0 (selects, not a
    // branch, so that a row of the unrolled loop stays one basic block)
    __device__ __forceinline__ void next_row()
    {
        const bool wrap = ++rr == n0;
        rr = wrap ? 0 : rr;
        prow = wrap ? psi_n : prow + n1;
        c0row = wrap ? c0 : c0row + n1;
        c1row = wrap ? c1 : c1row + ld1;
    }

    // one row of the pipeline at loop position t (phase P = t - t_begin mod U)
    // NPASS: corrective passes run on this row (fewer on the first warm-up
    // rows, whose later passes would work outside the dependency cone)
    template <int P, int NPASS> __device__ __forceinline__ void iter(int t)
    {
        constexpr int S = P % PF;
        T p_new = fp[S], c0_new = f0[S], c1_new = f1[S];
        fp[S] = prow[jj];
        f0[S] = c0row[jj];
        f1[S] = c1row[jj];
        next_row();

        AT(pq, C::QP, 0) = p_new;
        AT(dc0, 2, 0) = c0_new;
        AT(dc1, 2, 0) = c1_new;

        // donor-cell pass at row t-1
        T x = AT(pq, C::QP, 1);
        T f0lo = upwind_fp(AT(dc0, 2, 1), AT(pq, C::QP, 2), x);
        T f0hi = upwind_fp(AT(dc0, 2, 0), x, AT(pq, C::QP, 0));
        T f1lo = upwind_fp(AT(dc1, 2, 1), from_left(x), x);
        T f1hi = from_right(f1lo);
        T y = donor_update<KH>(x, f0hi - f0lo, f1hi - f1lo);
        T cn0 = AT(dc0, 2, 1), cn1 = AT(dc1, 2, 1);

        // pass m = k+2 takes input row a = t - 1 - 2k (psi^n row a is 1 + 2k
        // rows old)
#pragma unroll
        for (int k = 0; k < NPASS; k++) {
            T yk = ps[k].template advance<FCT, ABS, KH, SAFE, P>(
                y, cn0, cn1, pq.v[slot<C::QP>(P, 1 + 2 * k)], bad);
            cn0 = ps[k].aq0.v[slot<4>(P, 1)];
            cn1 = ps[k].aq1.v[slot<4>(P, 1)];
            y = yk;
        }

        if constexpr (NPASS == C::NP) {     // warm-up rows store nothing
            const bool row_out = t - C::LAG >= i0 && t - C::LAG < i1;
            if (out_lane && row_out) *orow = y;
            if constexpr (DG) dg.add(y, out_lane && row_out);
            orow += row_out ? n1 : 0;
        }
    }
};

// iterations t .. t+N-1 with phases P0 .. P0+N-1, NPASS corrective passes
template <typename T, int NI, bool FCT, bool ABS, bool KH, bool DG, bool SAFE, int N, int P0,
          int NPASS,
          int I = 0>
__device__ __forceinline__ void iter_block(Strip<T, NI, FCT, ABS, KH, DG, SAFE> &st, int t)
{
    if constexpr (I < N) {
        st.template iter<P0 + I, NPASS>(t + I);
        iter_block<T, NI, FCT, ABS, KH, DG, SAFE, N, P0, NPASS, I + 1>(st, t);
    }
}

// Warm-up of a chunk (iterations relative to t_begin).  Pass k's first input
// row inside the dependency cone of the chunk's first output row i0 is
// i0 - 2(NI - k - 1), reached at relative iteration 4k + 3; before that the
// pass would work on rows no output reads.  So relative iterations 0..2 run
// the donor pass only, and each following group of four runs one corrective
// pass more (stage K: iterations 4K-1 .. 4K+2, K passes), all in straight
// code; from relative iteration 4 NP - 1 on every pass runs.
template <typename T, int NI, bool FCT, bool ABS, bool KH, bool DG, bool SAFE, int K = 0>
__device__ __forceinline__ void warm_up(Strip<T, NI, FCT, ABS, KH, DG, SAFE> &st, int t_begin)
{
    constexpr int NP = Cfg<NI, FCT>::NP;
    if constexpr (K < NP) {
        constexpr int start = K == 0 ? 0 : 4 * K - 1, len = K == 0 ? 3 : 4;
        iter_block<T, NI, FCT, ABS, KH, DG, SAFE, len, start, K>(st, t_begin + start);
        warm_up<T, NI, FCT, ABS, KH, DG, SAFE, K + 1>(st, t_begin);
    }
}

// One chunk of one strip; returns true when fast mode met a divisor outside
// its range (the rows stored are then not to be kept).
template <typename T, int NI, bool FCT, bool ABS, bool KH, bool DG, bool SAFE>
__device__ __forceinline__ bool strip_pass(int n0, int n1, const T *__restrict__ psi_n,
                                           T *__restrict__ psi_out, const T *__restrict__ c0,
                                           const T *__restrict__ c1, int jstrip0, int i0, int i1,
                                           StepDiag &dg)
{
    using C = Cfg<NI, FCT>;
    Strip<T, NI, FCT, ABS, KH, DG, SAFE> st;
    st.bad = 0;
    st.dg.init();
    const int lane = threadIdx.x & (WAVE - 1);
    // global column of this lane (may lie outside [0, n1) in the halo)
    const int col = jstrip0 - C::H + lane;
    int jj = col % n1;
    if (jj < 0) jj += n1;
    st.n0 = n0;
    st.n1 = n1;
    st.i0 = i0;
    st.i1 = i1;
    st.jj = jj;
    st.psi_n = psi_n;
    st.c0 = c0;
    st.c1 = c1;
    st.pq.zero();
    st.dc0.zero();
    st.dc1.zero();
#pragma unroll
    for (int k = 0; k < C::NP; k++) st.ps[k].init();

    // iterations t_begin .. t_end; the loop runs whole blocks of U and then
    // of UT, so up to UT-1 extra iterations at the end compute rows that are
    // not stored (their loads wrap like every other row index)
    const int t_begin = i0 - C::LAG - 1;
    const int t_end = i1 - 1 + C::LAG;    // inclusive
    // row (mod n0) of the next row to load, and its row pointers
    int rr = t_begin % n0;
    if (rr < 0) rr += n0;
    st.rr = rr;
    st.ld1 = (int64_t)n1 + 1;
    st.prow = psi_n + (int64_t)rr * n1;
    st.c0row = c0 + (int64_t)rr * n1;
    st.c1row = c1 + (int64_t)rr * st.ld1;

    // prefetch: rows t_begin .. t_begin+PF-1 (slot k holds row t_begin+k)
#pragma unroll
    for (int k = 0; k < PF; k++) {
        st.fp[k] = st.prow[jj];
        st.f0[k] = st.c0row[jj];
        st.f1[k] = st.c1row[jj];
        st.next_row();
    }

    st.out_lane = lane >= C::H && lane < WAVE - C::H && col < n1;
    st.orow = psi_out + (int64_t)i0 * n1 + (st.out_lane ? col : 0);

    // warm-up (W iterations; a chunk has th + 4 NI - 1 > W), then the full
    // rows in blocks of U and UT whose phases continue from W
    constexpr int W = C::NP == 0 ? 0 : 4 * C::NP - 1;
    warm_up<T, NI, FCT, ABS, KH, DG, SAFE>(st, t_begin);
    int t = t_begin + W;
    for (; t + C::U - 1 <= t_end; t += C::U)
        iter_block<T, NI, FCT, ABS, KH, DG, SAFE, C::U, W, C::NP>(st, t);
    if constexpr (C::UT < C::U) {
        for (; t <= t_end; t += C::UT) iter_block<T, NI, FCT, ABS, KH, DG, SAFE, C::UT, W, C::NP>(st, t);
    } else {
        if (t <= t_end) iter_block<T, NI, FCT, ABS, KH, DG, SAFE, C::U, W, C::NP>(st, t);
    }
    dg = st.dg;
    return st.bad != 0;
}

// Fast mode, then (rarely, wave-uniformly) the same chunk again in safe mode.
// DG: the diagnostics of the rows kept, reduced over the wave, are written as
// partial `part_idx` of dpart (sum, compensation, min, max, non-finite count).
template <typename T, int NI, bool FCT, bool ABS, bool KH, bool DG>
__device__ __forceinline__ void strip_body(int n0, int n1, const T *__restrict__ psi_n,
                                           T *__restrict__ psi_out, const T *__restrict__ c0,
                                           const T *__restrict__ c1, int jstrip0, int i0, int i1,
                                           double *__restrict__ dpart, int part_idx)
{
    StepDiag dg;
    if (strip_pass<T, NI, FCT, ABS, KH, DG, false>(n0, n1, psi_n, psi_out, c0, c1, jstrip0, i0,
                                                   i1, dg))
        strip_pass<T, NI, FCT, ABS, KH, DG, true>(n0, n1, psi_n, psi_out, c0, c1, jstrip0, i0, i1,
                                                  dg);
    if constexpr (DG) dg.wave_write(dpart + 5 * (int64_t)part_idx);
}

template <typename T, int NI, bool FCT, bool ABS, bool KH, bool DG>
__global__ void __launch_bounds__(WAVE) k_fused2d(int n0, int n1, int th, int strips,
                                                  const T *__restrict__ psi_n,
                                                  T *__restrict__ psi_out,
                                                  const T *__restrict__ c0,
                                                  const T *__restrict__ c1,
                                                  double *__restrict__ dpart)
{
    using C = Cfg<NI, FCT>;
    int b = blockIdx.x;
    int strip = b % strips, chunk = b / strips;
    int i0 = chunk * th;
    int i1 = i0 + th < n0 ? i0 + th : n0;
    strip_body<T, NI, FCT, ABS, KH, DG>(n0, n1, psi_n, psi_out, c0, c1, strip * C::OW, i0, i1,
                                        dpart, b);
}

template <typename T, int NI, bool FCT, bool ABS, bool KH>
__global__ void __launch_bounds__(WAVE) k_fused2d_batched(const BatchGrid *__restrict__ grids,
                                                          int n_grids, int th, int n_tiles,
                                                          int xcd_order,
                                                          const T *__restrict__ psi_n,
                                                          T *__restrict__ psi_out,
                                                          const T *__restrict__ c0,
                                                          const T *__restrict__ c1)
{
    using C = Cfg<NI, FCT>;
    int b = blockIdx.x;
    if (xcd_order) {
        // the hardware deals workgroup b to XCD b % 8: number the tiles so
        // that consecutive tiles (neighbouring strips of one grid, sharing
        // halo columns) run on the same XCD and its L2
        const int x = b & 7, per = n_tiles >> 3, rem = n_tiles & 7;
        b = x * per + (x < rem ? x : rem) + (b >> 3);
    }
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
    strip_body<T, NI, FCT, ABS, KH, false>(n0, n1, psi_n + g.off_psi, psi_out + g.off_psi,
                                           c0 + g.off_c0, c1 + g.off_c1, strip * C::OW, i0, i1,
                                           nullptr, 0);
}

// default rows per chunk (when not tuned): about two waves per SIMD, so the
// chip is full while the warm-up rows stay a modest fraction
int64_t rows_per_chunk(int64_t n0, int64_t strips)
{
    int64_t target_waves = 2048;
    int64_t chunks = target_waves / (strips > 0 ? strips : 1);
    if (chunks < 1) chunks = 1;
    int64_t th = cdiv(n0, chunks);
    if (th < 16) th = 16;
    return th;
}

template <typename T, int NI, bool FCT, bool ABS, bool KH>
hipError_t launch(const Fused2DShape &sh, const T *psi_n, T *psi_out, const T *c0,
                  const T *c1, double *dpart, int *dparts, hipStream_t s)
{
    using C = Cfg<NI, FCT>;
    int64_t strips = cdiv(sh.n1, C::OW);
    int64_t th = sh.tile_rows > 0 ? sh.tile_rows : rows_per_chunk(sh.n0, strips);
    if (th > sh.n0) th = sh.n0;
    int64_t chunks = cdiv(sh.n0, th);
    int64_t blocks = strips * chunks;
    if (dpart) {
        if (dparts) *dparts = (int)blocks;
        k_fused2d<T, NI, FCT, ABS, KH, true><<<(unsigned)blocks, WAVE, 0, s>>>(
            (int)sh.n0, (int)sh.n1, (int)th, (int)strips, psi_n, psi_out, c0, c1, dpart);
    } else {
        k_fused2d<T, NI, FCT, ABS, KH, false><<<(unsigned)blocks, WAVE, 0, s>>>(
            (int)sh.n0, (int)sh.n1, (int)th, (int)strips, psi_n, psi_out, c0, c1, nullptr);
    }
    return hipGetLastError();
}

template <typename T, int NI, bool FCT, bool ABS, bool KH>
hipError_t launch_batched(const BatchGrid *g, int n_grids, int n_tiles, int th, int xcd,
                          const T *psi_n, T *psi_out, const T *c0, const T *c1,
                          hipStream_t s)
{
    k_fused2d_batched<T, NI, FCT, ABS, KH><<<(unsigned)n_tiles, WAVE, 0, s>>>(
        g, n_grids, th, n_tiles, xcd, psi_n, psi_out, c0, c1);
    return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t fused2d_step(const Fused2DShape &sh, int n_iters, unsigned opts, const T *psi_n,
                        T *psi_out, const T *c0, const T *c1, const T *G, hipStream_t s,
                        double *dpart, int *dparts)
{
    if (G || sh.bc0 != BC_PERIODIC || sh.bc1 != BC_PERIODIC) return hipErrorNotSupported;
    if (psi_n == psi_out) return hipErrorInvalidValue;   // a chunk may be recomputed (qset)
    bool fct = opts & OPT_FCT;
    const bool kahan = opts & OPT_KAHAN;
    const bool absf = (opts & OPT_ABS) && n_iters > 1;
#define MP_L(NI, F, A)                                                                     \
    (kahan ? launch<T, NI, F, A, true>(sh, psi_n, psi_out, c0, c1, dpart, dparts, s)       \
           : launch<T, NI, F, A, false>(sh, psi_n, psi_out, c0, c1, dpart, dparts, s))
    if (absf) {
        switch (n_iters * 2 + (fct ? 1 : 0)) {
        case 4: return MP_L(2, false, true);
        case 5: return MP_L(2, true, true);
        case 6: return MP_L(3, false, true);
        case 7: return MP_L(3, true, true);
        default: return hipErrorNotSupported;
        }
    }
    switch (n_iters * 2 + (fct ? 1 : 0)) {
    case 2: case 3: return MP_L(1, false, false);
    case 4: return MP_L(2, false, false);
    case 5: return MP_L(2, true, false);
    case 6: return MP_L(3, false, false);
    case 7: return MP_L(3, true, false);
    case 8: return MP_L(4, false, false);
    case 9: return MP_L(4, true, false);
    default: return hipErrorNotSupported;
    }
#undef MP_L
}

template <typename T>
hipError_t fused2d_batched_step(const BatchGrid *g, int n_grids, int n_tiles, int bc,
                                int n_iters, unsigned opts, int th, int xcd, const T *psi_n,
                                T *psi_out, const T *c0, const T *c1, hipStream_t s)
{
    if (bc != BC_PERIODIC || th < 1) return hipErrorNotSupported;
    if (psi_n == psi_out) return hipErrorInvalidValue;   // a chunk may be recomputed (qset)
    bool fct = opts & OPT_FCT;
    const bool kahan = opts & OPT_KAHAN;
    const bool absf = (opts & OPT_ABS) && n_iters > 1;
#define MP_B(NI, F, A)                                                                       \
    (kahan ? launch_batched<T, NI, F, A, true>(g, n_grids, n_tiles, th, xcd, psi_n, psi_out, \
                                               c0, c1, s)                                    \
           : launch_batched<T, NI, F, A, false>(g, n_grids, n_tiles, th, xcd, psi_n,         \
                                                psi_out, c0, c1, s))
    if (absf) {
        switch (n_iters * 2 + (fct ? 1 : 0)) {
        case 4: return MP_B(2, false, true);
        case 5: return MP_B(2, true, true);
        case 6: return MP_B(3, false, true);
        case 7: return MP_B(3, true, true);
        default: return hipErrorNotSupported;
        }
    }
    switch (n_iters * 2 + (fct ? 1 : 0)) {
    case 2: case 3: return MP_B(1, false, false);
    case 4: return MP_B(2, false, false);
    case 5: return MP_B(2, true, false);
    case 6: return MP_B(3, false, false);
    case 7: return MP_B(3, true, false);
    case 8: return MP_B(4, false, false);
    case 9: return MP_B(4, true, false);
    default: return hipErrorNotSupported;
    }
#undef MP_B
}

}  // namespace mp
