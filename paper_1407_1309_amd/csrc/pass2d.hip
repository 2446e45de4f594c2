// pass2d.hip -- one corrective MPDATA pass on a 2-D grid in one launch, and
// the 2-D donor-cell pass that precedes it.
//
// For the 2-D configurations the whole-step fused kernel does not take (open
// boundaries, iga, dfl, variable G, third-order terms): the pseudo-velocities
// of both dimensions (eq. adf_vel with its cross terms, the divergent-flow
// term and the third-order terms of Sect. 3.1.2, with the wall means of G),
// the limiter bounds and coefficients, the limited velocities and the
// corrective donor-cell update (divided by G) are computed in one sweep.
//
// Design (gfx950, wave64), the row march of the fused step kernel applied to
// a single pass whose input lives in HBM:
//   * one wavefront owns a strip of 64 columns and marches down a chunk of
//     rows; every stage is kept in per-lane register rings (one row per
//     iteration), column neighbours come from DPP lane shifts;
//   * the halo is 2 lanes on the left and 3 on the right (the divergent-flow
//     term reaches one wall further right), so a strip emits 59 columns
//     (more halo with the donor pass folded in and the third-order terms,
//     see Lanes);
//   * every load goes through the boundary map of its array (cells: wrap or
//     clamp; walls of the dimension's own advector: wrap, or clamp to the
//     edge wall), so the halo lanes and warm-up rows see exactly what the
//     stage-by-stage path reads.  The one quantity a halo cell may not
//     recompute is the limiter coefficient pair: with open boundaries the
//     coefficient of a cell outside the domain is that of the edge cell (the
//     boundary map applied to the coefficient array), so those lanes and rows
//     take it from the edge lane (readlane) or the edge row (ring slot).
#include "common.hpp"
#include "kernels.hpp"

#include <type_traits>

// Multiply-add contraction only within one source expression, decided by the
// front end, as in the fused step kernel (fused2d.hpp): the expressions the
// two kernels share then round alike, so a corrective pass formed here (the
// adjoint's recording launches) gives the bits of the same pass inside the
// fused step.
#pragma clang fp contract(on)

namespace mp {
namespace {

// Quotients of a stage with the fused step kernel's rule: a kept quotient is
// n * r, r the hardware reciprocal refined by one Newton step, where it is in
// range (FP64: r is a normal number; FP32: the divisor is normal or zero),
// else the IEEE quotient -- lane by lane, so its value depends on its
// operands only.  FP64 first tests the wave (no kept quotient out of range:
// the fast forms only, no division issued).  Quotients not kept are
// discarded by the caller.
template <int K>
__device__ __forceinline__ void lane_quotients(const double (&n)[K], const double (&d)[K],
                                               const bool (&keep)[K], double (&q)[K])
{
    double r[K];
    bool in[K];
    bool ok = true;
#pragma unroll
    for (int k = 0; k < K; k++) {
        r[k] = __builtin_amdgcn_rcp(d[k]);
        in[k] = __builtin_amdgcn_class(r[k], 0x108);   // +-normal
        ok = ok & (in[k] | !keep[k]);
    }
#pragma unroll
    for (int k = 0; k < K; k++) {
        const double rr = fma(fma(-d[k], r[k], 1.0), r[k], r[k]);
        q[k] = n[k] * rr;
    }
    if (__builtin_amdgcn_ballot_w64(!ok) != 0) {
#pragma unroll
        for (int k = 0; k < K; k++) q[k] = in[k] ? q[k] : n[k] / d[k];
    }
}
template <int K>
__device__ __forceinline__ void lane_quotients(const float (&n)[K], const float (&d)[K],
                                               const bool (&)[K], float (&q)[K])
{
#pragma unroll
    for (int k = 0; k < K; k++) {
        if (__builtin_amdgcn_classf(d[k], 0x168)) {   // +-normal or +-zero
            const float r = __builtin_amdgcn_rcpf(d[k]);
            const float q0 = n[k] * r;
            q[k] = fmaf(fmaf(-d[k], q0, n[k]), r, q0);
        } else {
            q[k] = n[k] / d[k];
        }
    }
}

constexpr int WAVE = 64;
constexpr int PF = 2;                    // rows in flight ahead of use

// Halo lanes left / right and output columns per strip.  With the donor
// pass computed in the kernel its result is valid one lane less on each
// side, so the strip needs one more halo lane on the left.  The third-order
// term of V1 reads x two columns to the left of its wall and one to the
// right: one more lane on the left, and with the donor pass (whose result
// the last lane cannot form) one more on the right.
template <bool DONOR, bool TOT> struct Lanes {
    static constexpr int HL = (DONOR ? 3 : 2) + (TOT ? 1 : 0);
    static constexpr int HR = 3 + (DONOR && TOT ? 1 : 0);
    static constexpr int OW = WAVE - HL - HR;
};

// ---- wave-wide lane shifts (DPP wave_shr:1 / wave_shl:1) -------------------
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
// value of v in lane l (l wave-uniform)
__device__ inline float lane_value(float v, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ inline double lane_value(double v, int l)
{
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}

template <typename T> __device__ __forceinline__ T donor_update(bool kahan, T x, T d0, T d1)
{
    if (!kahan) return x - (d0 + d1);
    T s = x, c = T(0);
    kahan_add(s, c, -d0);
    kahan_add(s, c, -d1);
    return s;
}

// the same with the flux differences divided by the cell's G (HG), as
// the stage-by-stage path: x - (d0 + d1) / G, or the two terms d_k / G
// compensated
template <bool HG, typename T>
__device__ __forceinline__ T donor_update_g(bool kahan, T x, T d0, T d1, T g)
{
    if constexpr (!HG) {
        return donor_update(kahan, x, d0, d1);
    } else {
        const bool keep[2] = {true, true};
        if (!kahan) {
            T n[1] = {d0 + d1}, d[1] = {g}, q[1];
            const bool k1[1] = {true};
            lane_quotients<1>(n, d, k1, q);
            return x - q[0];
        }
        T n[2] = {d0, d1}, d[2] = {g, g}, q[2];
        lane_quotients<2>(n, d, keep, q);
        return donor_update(true, x, q[0], q[1]);
    }
}

// ---- register rings (slot of the row pushed `age` iterations ago is a
// compile-time index for each unrolled phase P) ------------------------------
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

// Row-loop unroll: every ring depth divides it (8 under the third-order
// terms, whose rings are deeper).
template <bool TOT> constexpr int unroll() { return TOT ? 8 : 4; }

// State of one wavefront.  At iteration a (the newest row) it holds
//   x rows a..a-3 (and their left / right neighbours), psi^n row a,
//   dimension-0 walls a+1..a-1, dimension-1 walls of rows a, a-1,
//   raw V0 at walls a, a-1, bounds rows a..a-2, coefficients rows a-1, a-2,
//   limited V0 at walls a-1, a-2 and limited V1 of rows a-1, a-2;
// it computes V0 at wall a, V1 of row a-1, the coefficients of row a-1, the
// limited velocities at wall a-1 / row a-1 and the corrected row a-2.
// TOT: the third-order term of V0 at wall w reads x rows w-2..w+1, so V0 is
// formed at wall a-1 and every later stage one row later (SH = 1): the
// coefficients and limited velocities of row a-2, the corrected row a-3;
// x is kept back to row a-4, and V1 (still formed at row a-1, its
// third-order term reaching one column further left) for one more row.
//
// DONOR: the pass input x is the donor-cell pass of psi^n, computed here
// (row a from psi^n rows a-1..a+1, which are loaded one row ahead like the
// dimension-0 walls); otherwise x is loaded.  With open boundaries the donor
// result of a cell outside the domain is the edge cell's: edge lanes are
// copied across (readlane), rows past the end repeat the last row, and the
// first chunk starts at row 0 with the rows above filled with row 0.
// HG: G is an array (loaded with the cell rows, row a at age CO); otherwise
// G = 1.
template <typename T, bool FCT, bool IGA, bool ABS, bool DONOR, bool HG, bool TOT> struct March {
    static constexpr int CO = DONOR ? 1 : 0;   // age of row a in the c1 and G rings
    static constexpr int SH = TOT ? 1 : 0;     // row shift of the stages after V0
    static constexpr int XQ = TOT ? 8 : 4;     // x ring depth (ages 0..3+SH used)
    static constexpr int XR = TOT ? 4 : 2;     // right-neighbour ring (ages 0..1+SH)
    static constexpr int GQ = TOT ? 8 : 4;     // G ring (ages 0..CO+2+SH)
    int n0, n1, i0, i1, bc0, rr, rw;   // rr: next cell row to load, rw: next wall row
    int pr, pw;                        // rr, rw wrapped periodically (carried row to row)
    int lane_lo, lane_hi;              // lanes of columns 0 and n1-1 (edge strips)
    bool dfl, kahan, out_lane, w1_lane, fix_lo, fix_hi, prefill;
    int64_t ocol, ccol, wcol;          // per-lane column offsets
    const T *x, *pn, *c0, *c1, *G;
    T *y, *w0, *w1;
    T *v0r, *v1r, *bur, *bdr;          // records: raw velocities, coefficients
    T *xd;                             // record of the donor pass's result (DONOR)
    T fx[PF], fp[PF], f0[PF], f1[PF], fg[PF];
    Ring<T, XQ> xq;
    Ring<T, 4> xl, c0q, c1q, mxq, mnq, pq;
    Ring<T, GQ> gq;
    Ring<T, XR> xr;
    Ring<T, 2> v0q, v1q, buq, bdq, aq0, aq1;

    // x (or psi^n), psi^n, c1 and G of cell row r_cell and the dimension-0
    // wall r_wall
    __device__ __forceinline__ void fetch(int r_cell, int r_wall, T &vx, T &vp, T &v1, T &v0,
                                          T &vg)
    {
        fetch_at(map_cell(r_cell, n0, bc0), map_wall(r_wall, n0, bc0), vx, vp, v1, v0, vg);
    }
    // the same at mapped rows r (cell) and w (wall)
    __device__ __forceinline__ void fetch_at(int64_t r, int64_t w, T &vx, T &vp, T &v1, T &v0,
                                             T &vg)
    {
        vx = x[r * n1 + ccol];
        if (FCT && !DONOR) vp = pn[r * n1 + ccol];
        v1 = c1[r * (n1 + 1) + wcol];
        v0 = c0[w * n1 + ccol];
        if (HG) vg = G[r * n1 + ccol];
    }

    // rows rr / rw: open, clamped; periodic, the carried wrapped indices (a
    // wrap test per row instead of a division)
    __device__ __forceinline__ void load(int k)
    {
        const bool open = bc0 == BC_OPEN;
        const int r = open ? min(max(rr, 0), n0 - 1) : pr;
        const int w = open ? min(max(rw, 0), n0) : pw;
        fetch_at(r, w, fx[k], fp[k], f1[k], f0[k], fg[k]);
        rr++;
        rw++;
        pr = pr + 1 == n0 ? 0 : pr + 1;
        pw = pw + 1 == n0 ? 0 : pw + 1;
    }

    // G of cell row a - k (1 without HG)
    template <int P> __device__ __forceinline__ T g_row(int k) const
    {
        if constexpr (HG) return gq.v[slot<GQ>(P, CO + k)];
        else return T(1);
    }

    // donor result at a lane outside an open domain: the edge lane's
    __device__ __forceinline__ T edge_cols(T v)
    {
        if (fix_lo) {
            T e = lane_value(v, lane_lo);
            if (lane < lane_lo) v = e;
        }
        if (fix_hi) {
            T e = lane_value(v, lane_hi);
            if (lane > lane_hi) v = e;
        }
        return v;
    }

    template <int P> __device__ __forceinline__ void iter(int a)
    {
        constexpr int S = P % PF;
        T x_a, pn_a;
        if (HG) AT(gq, GQ, 0) = fg[S];   // row a + CO
        if (DONOR) {
            // psi^n, c1 of row a+1 and wall a+1 arrive; donor pass of row a
            AT(pq, 4, 0) = fx[S];
            AT(c1q, 4, 0) = f1[S];
            AT(c0q, 4, 0) = f0[S];
            load(S);
            const T pc = AT(pq, 4, 1), pm = AT(pq, 4, 2), pp = AT(pq, 4, 0);
            const T u0lo = AT(c0q, 4, 1), u0hi = AT(c0q, 4, 0), u1 = AT(c1q, 4, 1);
            const T f0lo = upwind_fp(u0lo, pm, pc);
            const T f0hi = upwind_fp(u0hi, pc, pp);
            const T f1lo = upwind_fp(u1, from_left(pc), pc);
            const T f1hi = from_right(f1lo);
            x_a = edge_cols(donor_update_g<HG>(kahan, pc, f0hi - f0lo, f1hi - f1lo,
                                               g_row<P>(0)));
            if (bc0 == BC_OPEN && a >= n0) x_a = AT(xq, XQ, 1);   // rows past the end
            pn_a = pc;
            // the donor result of the chunk's own rows and columns
            if (xd && a >= i0 && a < i1 && out_lane) xd[(int64_t)a * n1 + ocol] = x_a;
        } else {
            x_a = fx[S];
            pn_a = fp[S];
            AT(c1q, 4, 0) = f1[S];   // row a
            AT(c0q, 4, 0) = f0[S];   // wall a+1
            load(S);
        }
        AT(xq, XQ, 0) = x_a;
        AT(xl, 4, 0) = from_left(x_a);
        AT(xr, XR, 0) = from_right(x_a);
        if (DONOR && prefill) {
            // first row of an open domain: the rows above are copies of it
            prefill = false;
#pragma unroll
            for (int k = 1; k <= 3 + SH; k++) AT(xq, XQ, k) = x_a;
#pragma unroll
            for (int k = 1; k <= 2 + SH; k++) AT(xl, 4, k) = AT(xl, 4, 0);
#pragma unroll
            for (int k = 1; k <= 1 + SH; k++) AT(xr, XR, k) = AT(xr, XR, 0);
            if (FCT) {
#pragma unroll
                for (int k = 1; k <= 2 + SH; k++) {
                    AT(mxq, 4, k) = fmax(pn_a, x_a);
                    AT(mnq, 4, k) = fmin(pn_a, x_a);
                }
            }
        }

        // psi-fractions: V0 at wall w = a - SH (rows w-1 | w), V1 of row a-1
        // at wall j (columns j-1 | j): A terms and cross (B) terms, with TOT
        // the third-order D and E terms; with HG the reciprocal wall means
        // of G at both walls (the last two quotients)
        auto fa = [](T v) -> T { return ABS ? fabs(v) : v; };
        constexpr int NF = TOT ? 8 : 4;          // psi-fractions
        constexpr int NQ = NF + (HG ? 2 : 0);
        T num[NQ], den[NQ], fr[NQ];
        {
            const T xL = fa(AT(xq, XQ, SH + 1)), xR = fa(AT(xq, XQ, SH));
            num[0] = xR - xL;
            den[0] = xR + xL;
            const T p = fa(AT(xr, XR, SH)), q = fa(AT(xr, XR, SH + 1));
            const T e = fa(AT(xl, 4, SH)), f = fa(AT(xl, 4, SH + 1));
            num[1] = p + q - e - f;
            den[1] = p + q + e + f;
            if constexpr (TOT) {
                const T xR2 = fa(AT(xq, XQ, 0)), xL2 = fa(AT(xq, XQ, 3));
                num[4] = xR2 - xR - xL + xL2;
                den[4] = xR2 + xR + xL + xL2;
                num[5] = p - q - e + f;
                den[5] = den[1];
            }
        }
        {
            const T xL = fa(AT(xl, 4, 1)), xR = fa(AT(xq, XQ, 1));
            num[2] = xR - xL;
            den[2] = xR + xL;
            const T p = fa(AT(xq, XQ, 0)), q = fa(AT(xl, 4, 0));
            const T e = fa(AT(xq, XQ, 2)), f = fa(AT(xl, 4, 2));
            num[3] = p + q - e - f;
            den[3] = p + q + e + f;
            if constexpr (TOT) {
                const T xR2 = fa(AT(xr, XR, 1)), xL2 = fa(from_left(AT(xl, 4, 1)));
                num[6] = xR2 - xR - xL + xL2;
                den[6] = xR2 + xR + xL + xL2;
                num[7] = p - q - e + f;
                den[7] = den[3];
            }
        }
        T ig0 = T(1), ig1 = T(1);    // 1 / wall mean of G: wall a-SH | row a-1, wall j
        if constexpr (HG) {
            const T gw = g_row<P>(SH), gwm = g_row<P>(SH + 1), gm = g_row<P>(1);
            num[NF] = T(1);
            den[NF] = T(0.5) * (gwm + gw);
            num[NF + 1] = T(1);
            den[NF + 1] = T(0.5) * (from_left(gm) + gm);
        }
        if (IGA) {
            fr[0] = num[0] / T(2);
            fr[1] = num[1] / T(4);
            fr[2] = num[2] / T(2);
            fr[3] = num[3] / T(4);
#pragma unroll
            for (int k = 4; k < NF; k++) fr[k] = num[k] / T(4);
            if constexpr (HG) {
                T n2[2] = {num[NF], num[NF + 1]}, d2[2] = {den[NF], den[NF + 1]}, q2[2];
                const bool k2[2] = {true, true};
                lane_quotients<2>(n2, d2, k2, q2);
                ig0 = q2[0];
                ig1 = q2[1];
            }
        } else {
            bool keep[NQ];
#pragma unroll
            for (int k = 0; k < NQ; k++) keep[k] = k >= NF || den[k] != T(0);
            lane_quotients<NQ>(num, den, keep, fr);
#pragma unroll
            for (int k = 0; k < NF; k++) fr[k] = den[k] == T(0) ? T(0) : fr[k];
            if constexpr (HG) {
                ig0 = fr[NF];
                ig1 = fr[NF + 1];
            }
        }
        T v0, v1;
        {
            const T u = AT(c0q, 4, 1 + SH);                  // wall a-SH
            const T s1 = AT(c1q, 4, CO + SH + 1) + AT(c1q, 4, CO + SH);
            const T cb = T(0.25) * (s1 + from_right(s1));
            if constexpr (HG) {
                v0 = (fabs(u) - u * u * ig0) * fr[0];
                v0 -= T(0.5) * u * cb * ig0 * fr[1];
            } else {
                v0 = (fabs(u) - u * u) * fr[0];
                v0 -= T(0.5) * u * cb * fr[1];
            }
            if (dfl) {
                // mean of the divergences of the wall's two cells
                const T c1a = AT(c1q, 4, CO + SH), c1b = AT(c1q, 4, CO + SH + 1);
                T dv = (AT(c0q, 4, 1 + SH) - AT(c0q, 4, 2 + SH)) +
                       (AT(c0q, 4, SH) - AT(c0q, 4, 1 + SH));
                dv += (from_right(c1b) - c1b) + (from_right(c1a) - c1a);
                if (IGA) dv *= T(0.5) * (AT(xq, XQ, SH + 1) + AT(xq, XQ, SH));
                v0 -= T(0.25) * u * ig0 * dv;
            }
            if constexpr (TOT) {
                v0 += (T(3) * u * fabs(u) * ig0 - T(2) * u * u * u * (ig0 * ig0) - u) *
                      (T(1) / T(3)) * fr[4];
                v0 += (fabs(u) * cb * ig0 - T(2) * u * u * cb * (ig0 * ig0)) * fr[5];
            }
        }
        {
            const T u = AT(c1q, 4, CO + 1);                  // row a-1, wall j
            const T s0 = AT(c0q, 4, 2) + AT(c0q, 4, 1);
            const T cb = T(0.25) * (from_left(s0) + s0);
            if constexpr (HG) {
                v1 = (fabs(u) - u * u * ig1) * fr[2];
                v1 -= T(0.5) * u * cb * ig1 * fr[3];
            } else {
                v1 = (fabs(u) - u * u) * fr[2];
                v1 -= T(0.5) * u * cb * fr[3];
            }
            if (dfl) {
                // mean of the divergences of cells (a-1, j-1) and (a-1, j)
                const T d0 = AT(c0q, 4, 1) - AT(c0q, 4, 2);
                T dv = from_left(d0) + d0;
                const T c = AT(c1q, 4, CO + 1);
                dv += (c - from_left(c)) + (from_right(c) - c);
                if (IGA) dv *= T(0.5) * (AT(xl, 4, 1) + AT(xq, XQ, 1));
                v1 -= T(0.25) * u * ig1 * dv;
            }
            if constexpr (TOT) {
                v1 += (T(3) * u * fabs(u) * ig1 - T(2) * u * u * u * (ig1 * ig1) - u) *
                      (T(1) / T(3)) * fr[6];
                v1 += (fabs(u) * cb * ig1 - T(2) * u * u * cb * (ig1 * ig1)) * fr[7];
            }
        }
        AT(v0q, 2, 0) = v0;
        if constexpr (TOT) AT(v1q, 2, 0) = v1;
        // V1 of the limiter's row rl = a-1-SH
        const T v1l = TOT ? AT(v1q, 2, 1) : v1;
        const int rl = a - 1 - SH;

        T lim0, lim1;
        if (FCT) {
            // bounds over {psi^n, x} at the cell and its face neighbours
            AT(mxq, 4, 0) = fmax(pn_a, x_a);
            AT(mnq, 4, 0) = fmin(pn_a, x_a);
            const T m1 = AT(mxq, 4, SH + 1), n1v = AT(mnq, 4, SH + 1);
            const T mx = fmax(fmax(m1, fmax(AT(mxq, 4, SH + 2), AT(mxq, 4, SH))),
                              fmax(from_left(m1), from_right(m1)));
            const T mn = fmin(fmin(n1v, fmin(AT(mnq, 4, SH + 2), AT(mnq, 4, SH))),
                              fmin(from_left(n1v), from_right(n1v)));
            // in / out fluxes of cell (rl, j); unit field under iga
            const T xc = AT(xq, XQ, SH + 1);
            const T v0lo = AT(v0q, 2, 1), v0hi = v0;
            const T v1lo = v1l, v1hi = from_right(v1l);
            T fin, fout;
            if (IGA) {
                fin = (pos(v0lo) - neg(v0hi)) + (pos(v1lo) - neg(v1hi));
                fout = (pos(v0hi) - neg(v0lo)) + (pos(v1hi) - neg(v1lo));
            } else {
                fin = (pos(v0lo) * AT(xq, XQ, SH + 2) - neg(v0hi) * AT(xq, XQ, SH)) +
                      (pos(v1lo) * AT(xl, 4, SH + 1) - neg(v1hi) * AT(xr, XR, SH + 1));
                fout = (pos(v0hi) * xc - neg(v0lo) * xc) + (pos(v1hi) * xc - neg(v1lo) * xc);
            }
            const T gc = g_row<P>(1 + SH);
            T bn[2] = {HG ? gc * (mx - xc) : mx - xc, HG ? gc * (xc - mn) : xc - mn};
            T bdv[2] = {fin, fout}, bq[2];
            const bool bkeep[2] = {fin > T(0), fout > T(0)};
            lane_quotients<2>(bn, bdv, bkeep, bq);
            T bu = fin > T(0) ? bq[0] : T(1);
            T bd = fout > T(0) ? bq[1] : T(1);
            // open columns: a cell left of column 0 / right of column n1-1
            // has the edge cell's coefficients
            if (fix_lo) {
                T eu = lane_value(bu, lane_lo), ed = lane_value(bd, lane_lo);
                if (lane < lane_lo) {
                    bu = eu;
                    bd = ed;
                }
            }
            if (fix_hi) {
                T eu = lane_value(bu, lane_hi), ed = lane_value(bd, lane_hi);
                if (lane > lane_hi) {
                    bu = eu;
                    bd = ed;
                }
            }
            AT(buq, 2, 0) = bu;
            AT(bdq, 2, 0) = bd;
            // limited V1 of row rl at wall j: L = (rl, j-1), R = (rl, j)
            {
                T up = fmin(fmin(T(1), from_left(bd)), bu);
                T dn = fmin(fmin(T(1), from_left(bu)), bd);
                lim1 = pos(v1l) * up + neg(v1l) * dn;
            }
            // limited V0 at wall rl: L = row rl-1, R = row rl; with open rows
            // the row outside the domain takes the edge row's coefficients
            {
                T bu_l = AT(buq, 2, 1), bd_l = AT(bdq, 2, 1);
                T bu_r = AT(buq, 2, 0), bd_r = AT(bdq, 2, 0);
                if (bc0 == BC_OPEN) {
                    if (rl == 0) {
                        bu_l = bu_r;
                        bd_l = bd_r;
                    } else if (rl == n0) {
                        bu_r = bu_l;
                        bd_r = bd_l;
                    }
                }
                T v = AT(v0q, 2, 1);
                T up = fmin(fmin(T(1), bd_l), bu_r);
                T dn = fmin(fmin(T(1), bu_l), bd_r);
                lim0 = pos(v) * up + neg(v) * dn;
            }
        } else {
            lim0 = AT(v0q, 2, 1);
            lim1 = v1l;
        }
        AT(aq0, 2, 0) = lim0;
        AT(aq1, 2, 0) = lim1;

        // limited velocities for a following pass (and, when asked, the raw
        // velocities and the coefficients): wall rl and row rl
        if (w0) {
            const int w = rl;
            if (w >= i0 && (w < i1 || (w == n0 && i1 == n0 && bc0 == BC_OPEN))) {
                const int64_t k0 = (int64_t)w * n1 + ocol, k1 = (int64_t)w * (n1 + 1) + ocol;
                if (out_lane) {
                    w0[k0] = lim0;
                    if (v0r) v0r[k0] = AT(v0q, 2, 1);
                }
                if (w < i1 && w1_lane) {
                    w1[k1] = lim1;
                    if (v1r) v1r[k1] = v1l;
                }
                if (FCT && bur && w < i1 && out_lane) {
                    bur[k0] = AT(buq, 2, 0);
                    bdr[k0] = AT(bdq, 2, 0);
                }
            }
        }

        // corrective donor-cell pass at row rl-1 (flux = limited velocity
        // under iga)
        const T xc = AT(xq, XQ, SH + 2);
        T f0lo, f0hi, f1lo;
        if (IGA) {
            f0lo = AT(aq0, 2, 1);
            f0hi = AT(aq0, 2, 0);
            f1lo = AT(aq1, 2, 1);
        } else {
            f0lo = pos(AT(aq0, 2, 1)) * AT(xq, XQ, SH + 3) + neg(AT(aq0, 2, 1)) * xc;
            f0hi = pos(AT(aq0, 2, 0)) * xc + neg(AT(aq0, 2, 0)) * AT(xq, XQ, SH + 1);
            f1lo = pos(AT(aq1, 2, 1)) * AT(xl, 4, SH + 2) + neg(AT(aq1, 2, 1)) * xc;
        }
        const T f1hi = from_right(f1lo);
        const T res = donor_update_g<HG>(kahan, xc, f0hi - f0lo, f1hi - f1lo, g_row<P>(2 + SH));
        const int r = rl - 1;
        if (y && r >= i0 && r < i1 && out_lane) y[(int64_t)r * n1 + ocol] = res;
    }
    int lane;
};

template <typename T, bool FCT, bool IGA, bool ABS, bool DONOR, bool HG, bool TOT, int P = 0>
__device__ __forceinline__ void iter_block(March<T, FCT, IGA, ABS, DONOR, HG, TOT> &m, int a)
{
    if constexpr (P < unroll<TOT>()) {
        m.template iter<P>(a + P);
        iter_block<T, FCT, IGA, ABS, DONOR, HG, TOT, P + 1>(m, a);
    }
}

// DONOR: x is psi^n (the donor pass is done here); otherwise x is the
// previous pass's result and psi_n is psi^n.
template <typename T, bool FCT, bool IGA, bool ABS, bool DONOR, bool HG, bool TOT>
__global__ void __launch_bounds__(WAVE)
    k_pass2d(int n0, int n1, int bc0, int bc1, int th, int strips, int dfl, int kahan,
             const T *__restrict__ x, const T *__restrict__ c0, const T *__restrict__ c1,
             const T *__restrict__ psi_n, const T *__restrict__ G, T *__restrict__ y,
             T *__restrict__ w0,
             T *__restrict__ w1, T *__restrict__ v0r, T *__restrict__ v1r,
             T *__restrict__ bur, T *__restrict__ bdr, T *__restrict__ xd)
{
    constexpr int HL = Lanes<DONOR, TOT>::HL, HR = Lanes<DONOR, TOT>::HR;
    constexpr int OW = Lanes<DONOR, TOT>::OW;
    const int b = blockIdx.x;
    const int strip = b % strips, chunk = b / strips;
    const int i0 = chunk * th;
    const int i1 = i0 + th < n0 ? i0 + th : n0;
    const int jstrip0 = strip * OW;
    const int lane = threadIdx.x & (WAVE - 1);
    const int col = jstrip0 - HL + lane;

    using M = March<T, FCT, IGA, ABS, DONOR, HG, TOT>;
    M m;
    m.n0 = n0;
    m.n1 = n1;
    m.i0 = i0;
    m.i1 = i1;
    m.bc0 = bc0;
    m.lane = lane;
    m.dfl = dfl != 0;
    m.kahan = kahan != 0;
    m.x = x;
    m.pn = psi_n;
    m.c0 = c0;
    m.c1 = c1;
    m.G = G;
    m.y = y;
    m.w0 = w0;
    m.w1 = w1;
    m.v0r = v0r;
    m.v1r = v1r;
    m.bur = bur;
    m.bdr = bdr;
    m.xd = DONOR ? xd : nullptr;
    m.ccol = map_cell(col, n1, bc1);
    m.wcol = map_wall(col, n1, bc1);
    m.ocol = col;
    m.out_lane = lane >= HL && lane < WAVE - HR && col >= 0 && col < n1;
    // walls of dimension 1 written for a following pass: the strip's output
    // columns, plus the edge wall n1 (open) by the last strip
    m.w1_lane = (lane >= HL && lane < WAVE - HR && col >= 0 && col < n1) ||
                (bc1 == BC_OPEN && col == n1 && strip == strips - 1);
    m.lane_lo = HL - jstrip0;
    m.lane_hi = n1 - 1 - jstrip0 + HL;
    m.fix_lo = bc1 == BC_OPEN && jstrip0 - HL < 0;
    m.fix_hi = bc1 == BC_OPEN && jstrip0 - HL + WAVE > n1;
    m.xq.zero();
    m.xl.zero();
    m.c0q.zero();
    m.pq.zero();
#pragma unroll
    for (int k = 0; k < M::GQ; k++) m.gq.v[k] = T(1);
    m.mxq.zero();
    m.mnq.zero();
    m.xr.zero();
    m.c1q.zero();
    m.v0q.zero();
    m.v1q.zero();
    m.buq.zero();
    m.bdq.zero();
    m.aq0.zero();
    m.aq1.zero();
#pragma unroll
    for (int k = 0; k < PF; k++) m.fp[k] = T(0);

    // iterations a = i0-3 .. i1+1+SH (whole blocks of the unroll; extra
    // rows are not stored).  The first output row i0 needs the limiter coefficients of
    // row i0-1, hence V0 at wall i0-1, whose divergent-flow term reads wall
    // i0-2: loaded as the newest wall at iteration i0-3.  Without the donor
    // pass, cell rows are loaded from a and dimension-0 walls one row
    // ahead; with it, psi^n, c1 and the walls all one row ahead, and the
    // rings start with rows a-1 and a.  The first chunk of an open domain
    // starts at row 0 (the rows above are copies of row 0).
    m.prefill = DONOR && bc0 == BC_OPEN && i0 == 0;
    const int a_begin = m.prefill ? 0 : i0 - 3;
    const int a_end = i1 + 1 + M::SH;
    if (DONOR) {
        T vp;
        m.fetch(a_begin - 1, a_begin - 1, m.pq.v[slot<4>(0, 2)], vp, m.c1q.v[slot<4>(0, 2)],
                m.c0q.v[slot<4>(0, 2)], m.gq.v[slot<M::GQ>(0, 2)]);
        m.fetch(a_begin, a_begin, m.pq.v[slot<4>(0, 1)], vp, m.c1q.v[slot<4>(0, 1)],
                m.c0q.v[slot<4>(0, 1)], m.gq.v[slot<M::GQ>(0, 1)]);
        m.rr = a_begin + 1;
        m.rw = a_begin + 1;
    } else {
        m.rr = a_begin;
        m.rw = a_begin + 1;
    }
    m.pr = (int)map_cell(m.rr, n0, BC_PERIODIC);
    m.pw = (int)map_cell(m.rw, n0, BC_PERIODIC);
#pragma unroll
    for (int k = 0; k < PF; k++) m.load(k);
    for (int a = a_begin; a <= a_end; a += unroll<TOT>())
        iter_block<T, FCT, IGA, ABS, DONOR, HG, TOT>(m, a);
}

// Donor-cell pass of a 2-D grid (eqs. upstream, F; G = 1): one thread per
// cell, a block of 256 threads per row segment (the row is wave-uniform, so
// no division per thread).  With `copy`, psi^n is also written there (for
// an in-place step whose corrective passes still need psi^n).
constexpr int DB = 256;

template <typename T>
__global__ void __launch_bounds__(DB)
    k_donor2d(int n0, int n1, int bc0, int bc1, int bpr, int kahan, const T *__restrict__ x,
              const T *__restrict__ c0, const T *__restrict__ c1, T *__restrict__ out,
              T *__restrict__ copy)
{
    const int row = blockIdx.x / bpr;
    const int j = (blockIdx.x - row * bpr) * DB + threadIdx.x;
    if (j >= n1) return;
    const int64_t r = (int64_t)row * n1;
    const int64_t rm = (int64_t)wrap_cell(row - 1, n0, bc0) * n1;
    const int64_t rp = (int64_t)wrap_cell(row + 1, n0, bc0) * n1;
    const int jm = wrap_cell(j - 1, n1, bc1), jp = wrap_cell(j + 1, n1, bc1);
    const T xc = x[r + j];
    const T u0lo = c0[r + j];
    const T u0hi = c0[(int64_t)wrap_wall(row + 1, n0, bc0) * n1 + j];
    const int64_t r1 = (int64_t)row * (n1 + 1);
    const T u1lo = c1[r1 + j];
    const T u1hi = c1[r1 + wrap_wall(j + 1, n1, bc1)];
    const T f0lo = upwind_fp(u0lo, x[rm + j], xc);
    const T f0hi = upwind_fp(u0hi, xc, x[rp + j]);
    const T f1lo = upwind_fp(u1lo, x[r + jm], xc);
    const T f1hi = upwind_fp(u1hi, xc, x[r + jp]);
    out[r + j] = donor_update(kahan != 0, xc, f0hi - f0lo, f1hi - f1lo);
    if (copy) copy[r + j] = xc;
}

// Default rows per chunk: about four waves per SIMD (the FP64 kernels hold
// 4-5 waves per SIMD), at least 11 rows, and a chunk length whose iteration
// count (rows + 5 + sh) is a whole number of unrolled blocks of u rows.
int64_t chunk_rows(int64_t n0, int64_t strips, int tile_rows, int u, int sh)
{
    int64_t th = tile_rows;
    if (th <= 0) {
        int64_t chunks = 4096 / (strips > 0 ? strips : 1);
        if (chunks < 1) chunks = 1;
        th = cdiv(n0, chunks);
        if (th < 11) th = 11;
        th = cdiv(th + 5 + sh, u) * u - 5 - sh;
    }
    return th > n0 ? n0 : th;
}

template <typename T, bool FCT, bool IGA, bool ABS, bool DONOR, bool HG, bool TOT>
hipError_t launch(const Geom &g, unsigned opts, const T *x, const T *c0, const T *c1,
                  const T *psi_n, const T *G, T *y, T *w0, T *w1, const PassRecord<T> &rec,
                  int tile_rows, hipStream_t s)
{
    const int64_t n0 = g.n[0], n1 = g.n[1];
    const int64_t strips = cdiv(n1, Lanes<DONOR, TOT>::OW);
    const int64_t th = chunk_rows(n0, strips, tile_rows, unroll<TOT>(), TOT ? 1 : 0);
    const int64_t blocks = strips * cdiv(n0, th);
    k_pass2d<T, FCT, IGA, ABS, DONOR, HG, TOT><<<(unsigned)blocks, WAVE, 0, s>>>(
        (int)n0, (int)n1, g.bc[0], g.bc[1], (int)th, (int)strips, (opts & OPT_DFL) ? 1 : 0,
        (opts & OPT_KAHAN) ? 1 : 0, x, c0, c1, psi_n, G, y, w0, w1, rec.v0, rec.v1, rec.bu,
        rec.bd, rec.xd);
    return hipGetLastError();
}

}  // namespace

bool pass2d_supported(int nd, int n_iters, unsigned opts, int has_g, const int64_t n[3])
{
    (void)has_g;   // G = 1 and variable G alike
    if (nd != 2 || n_iters < 2) return false;
    if ((opts & OPT_ABS) && (opts & OPT_IGA)) return false;
    // 32-bit row / column arithmetic
    return n[0] < (1 << 30) && n[1] < (1 << 30) && n[0] * (n[1] + 1) < ((int64_t)1 << 31);
}

template <typename T>
hipError_t pass2d_launch(const Geom &g, unsigned opts, const T *x, const T *c0, const T *c1,
                         const T *psi_n, const T *G, T *y, T *w0, T *w1, hipStream_t s,
                         const PassRecord<T> &rec, int tile_rows)
{
    const bool fct = opts & OPT_FCT, iga = opts & OPT_IGA, absf = opts & OPT_ABS;
    // psi_n NULL: the first corrective pass with the donor pass folded in
    // (x = psi^n)
    const bool donor = psi_n == nullptr;
    const T *pn = donor ? x : psi_n;
    const bool tot = opts & OPT_TOT;
    auto go = [&](auto F, auto I, auto A, auto D, auto H, auto O) {
        return launch<T, decltype(F)::value, decltype(I)::value, decltype(A)::value,
                      decltype(D)::value, decltype(H)::value, decltype(O)::value>(
            g, opts, x, c0, c1, pn, G, y, w0, w1, rec, tile_rows, s);
    };
    using TT = std::true_type;
    using FF = std::false_type;
    auto by_t = [&](auto F, auto I, auto A, auto D, auto H) {
        return tot ? go(F, I, A, D, H, TT{}) : go(F, I, A, D, H, FF{});
    };
    auto by_g = [&](auto F, auto I, auto A, auto D) {
        return G ? by_t(F, I, A, D, TT{}) : by_t(F, I, A, D, FF{});
    };
    auto by_d = [&](auto F, auto I, auto A) {
        return donor ? by_g(F, I, A, TT{}) : by_g(F, I, A, FF{});
    };
    auto by_f = [&](auto I, auto A) { return fct ? by_d(TT{}, I, A) : by_d(FF{}, I, A); };
    if (iga) return by_f(TT{}, FF{});
    if (absf) return by_f(FF{}, TT{});
    return by_f(FF{}, FF{});
}

template <typename T>
hipError_t donor2d_launch(const Geom &g, unsigned opts, const T *x, const T *c0, const T *c1,
                          T *out, T *copy, hipStream_t s)
{
    const int bpr = (int)cdiv(g.n[1], DB);
    k_donor2d<T><<<(unsigned)(bpr * g.n[0]), DB, 0, s>>>((int)g.n[0], (int)g.n[1], g.bc[0],
                                                         g.bc[1], bpr,
                                                         (opts & OPT_KAHAN) ? 1 : 0, x, c0, c1,
                                                         out, copy);
    return hipGetLastError();
}

template hipError_t donor2d_launch<float>(const Geom &, unsigned, const float *, const float *,
                                          const float *, float *, float *, hipStream_t);
template hipError_t donor2d_launch<double>(const Geom &, unsigned, const double *,
                                           const double *, const double *, double *, double *,
                                           hipStream_t);
template hipError_t pass2d_launch<float>(const Geom &, unsigned, const float *, const float *,
                                         const float *, const float *, const float *, float *,
                                         float *, float *, hipStream_t, const PassRecord<float> &,
                                         int);
template hipError_t pass2d_launch<double>(const Geom &, unsigned, const double *, const double *,
                                          const double *, const double *, const double *,
                                          double *, double *, double *, hipStream_t,
                                          const PassRecord<double> &, int);

}  // namespace mp
