// step3d.hip -- a whole 3-D MPDATA step with two passes and no limiter in
// one launch (donor-cell pass, pseudo-velocity with its cross and
// third-order terms, corrective pass; infinite gauge, |psi| fractions, the
// divergent-flow term, variable G, both boundary types), and the passes of
// longer steps or steps with the limiter (modes below).
//
// A workgroup of SJ x SK threads owns a tile of SJ x SK (j, k) output
// columns and marches along i over a chunk of planes.  In the iteration
// that brings plane t on chip it
//   1. stores the planes its global loads fetched during the previous
//      iteration into LDS rings: psi^n (plane t+1, the tile with a ring of 3
//      cells), the dimension-0 advector (wall t+1), the dimension-1 and
//      dimension-2 advectors and G (plane t), each on the tile with a ring
//      of 2 cells; then issues the loads of the next iteration;
//   2. forms the donor-cell result y1 of plane t on the tile and its ring of
//      2 cells from LDS, so y1 never goes through HBM;
//   3. forms the pseudo-velocities (eq. adf_vel with the multi-dimensional
//      cross terms and the third-order terms): V0 at the wall between planes
//      t-2 and t-1 of its own column, V1 and V2 at plane t-2 on the low walls
//      of its own cell (the tile's far edge walls by the first threads);
//   4. applies the corrective pass to plane t-2 of its own column.
// Two barriers per plane.  Every thread computes one output cell (the
// ring's y1 cells are shared out as a second cell to the first threads), so
// no thread only recomputes a halo.
//
// Modes for steps with the limiter or more passes (Step3dOut): in output
// mode step 4 is replaced by writing the donor result and the raw V0, V1, V2
// of each plane (each wall by its owner), and with BETA also the limiter
// coefficients of plane t-2 (Sect. 3.1.4: the bounds over the cell and its
// face neighbours of psi^n and the pass input, the in- and out-fluxes, and
// their quotients), which needs psi^n of planes t-3..t-1 (a six-plane
// ring); in pass mode (XIN) step 2 is replaced by reading the pass input.
//
// Boundaries: every global read goes through the boundary map (periodic
// wrap / open clamp), so ring positions hold mapped values.  The y1 of a
// cell outside an open domain must be the edge cell's (what the stage-by-
// stage path reads there): in j and k it is computed at the clamped
// position, in i it is read from the edge plane's ring slot.
//
// The donor-cell arithmetic is that of k_donor3d (fused3d.hip), term by
// term in the same order, so the two give the same bits.
#include "common.hpp"
#include "kernels.hpp"

#include <type_traits>

namespace mp {
namespace {

constexpr int SJ = 16, SK = 32, NT = SJ * SK;   // output tile and threads
constexpr int BJ = SJ + 4, BK = SK + 4;         // y1 box: tile + ring of 2
constexpr int PJ = SJ + 6, PK = SK + 6;         // psi^n box: tile + ring of 3
constexpr int NY = BJ * BK;                     // cells of a y1 box plane
constexpr int NP = PJ * PK;                     // cells of a psi^n box plane
constexpr int N1 = (BJ + 1) * BK;               // dimension-1 walls of the box
constexpr int N2 = BJ * (BK + 1);               // dimension-2 walls of the box
static_assert(NY <= 2 * NT && NP <= 2 * NT && N1 <= 2 * NT && N2 <= 2 * NT,
              "each thread loads at most two entries of every box plane");
static_assert(NT <= NY && NT <= NP && NT <= N1 && NT <= N2, "entry 0 of every box plane is in it");
static_assert(SK <= NT && SK + SJ <= NT, "far-edge walls need that many threads");
constexpr int WAVE64 = 64;
static_assert(NT % WAVE64 == 0, "whole waves");
static_assert(NY - NT == 4 * BK + 4 * SJ && NY - NT <= NT, "ring cells: one per thread at most");

struct G3s {
    int n0, n1, n2;
    int bc0, bc1, bc2;
};

template <typename T, bool IGA> __device__ __forceinline__ T fr3(T num, T den, T m)
{
    if (IGA) return num * (T(1) / m);
    return den == T(0) ? T(0) : num / den;
}

// ring slot of a virtual plane index t >= -12
__device__ __forceinline__ int slot3(int t) { return (t + 12) % 3; }
__device__ __forceinline__ int slot4(int t) { return (t + 12) & 3; }
// psi^n ring slot: planes t-1..t+1 (three slots), or t-4..t+1 (six) when
// the kernel also forms the limiter coefficients of plane t-2 (read after
// the second barrier, while the next iteration may already store plane t+2)
template <bool BETA> __device__ __forceinline__ int slotp(int t)
{
    return BETA ? (t + 18) % 6 : (t + 12) % 3;
}

// Reciprocals 1 / d[k] as one FP64 quotient set (the range test and the
// refined hardware reciprocal of the quotient sets in common.hpp, numerator
// 1), and whether the set took the refined form: then n * q[k] has the bits
// of that set's quotient n / d[k] for any n, so a later quotient by the same
// divisor can reuse q[k]; else q[k] is the IEEE quotient and such a later
// quotient must divide.
template <int K> __device__ __forceinline__ bool rcp_set(const double (&d)[K], double (&q)[K])
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
            q[k] = 1.0 * r;
        }
        return true;
    }
#pragma unroll
    for (int k = 0; k < K; k++) q[k] = 1.0 / d[k];
    return false;
}

// in-plane offset of box entry e of a box with `w` entries per row, the
// box's origin at (jb, kb) in global cell (or wall) coordinates; `wall_j` /
// `wall_k` mark the dimension whose coordinate is a wall index.  -1 when e
// is past the box.
__device__ __forceinline__ int64_t box_offset(int e, int n_e, int w, int jb, int kb, bool wall_j,
                                              bool wall_k, const G3s &g, int64_t row_len)
{
    if (e >= n_e) return -1;
    const int bj = e / w, bk = e % w;
    const int64_t j = wall_j ? map_wall(jb + bj, g.n1, g.bc1) : map_cell(jb + bj, g.n1, g.bc1);
    const int64_t k = wall_k ? map_wall(kb + bk, g.n2, g.bc2) : map_cell(kb + bk, g.n2, g.bc2);
    return j * row_len + k;
}

template <typename T, bool HAS_G, bool IGA, bool ABS, bool DFL, bool TOT, bool XIN, bool BETA>
__global__ void __launch_bounds__(NT) k_step3d(G3s g, int th, int tiles_k, int tiles_j, int nblk,
                                               int kahan, const T *__restrict__ x,
                                               const T *__restrict__ c0,
                                               const T *__restrict__ c1,
                                               const T *__restrict__ c2,
                                               const T *__restrict__ G, T *__restrict__ out,
                                               Step3dOut<T> vo)
{
    __shared__ T Ps[BETA ? 6 : 3][NP];                   // psi^n, planes t-1..t+1 (BETA: t-4..)
    __shared__ T Ys[4][NY];                              // y1, planes t-3..t
    __shared__ T C0s[4][NY];                             // c0, walls t-2..t+1
    __shared__ T C1s[3][N1];                             // c1, planes t-2..t
    __shared__ T C2s[3][N2];                             // c2, planes t-2..t
    __shared__ T Gs[HAS_G ? 3 : 1][HAS_G ? NY : 1];      // G, planes t-2..t
    __shared__ T V1s[(SJ + 1) * SK];                     // V1 at plane t-2
    __shared__ T V2s[SJ * (SK + 1)];                     // V2 at plane t-2

    const int tid = threadIdx.x;
    const int r = tid / SK, l = tid % SK;
    // The hardware deals workgroup b to XCD b % 8; tiles are numbered so that
    // consecutive tiles (which share ring cells) run on one XCD and its L2.
    int b;
    {
        const int xq = blockIdx.x & 7, per = nblk >> 3, rem = nblk & 7;
        b = xq * per + (xq < rem ? xq : rem) + (blockIdx.x >> 3);
    }
    const int tk = b % tiles_k;
    b /= tiles_k;
    const int tj = b % tiles_j;
    const int ch = b / tiles_j;
    const int j0 = tj * SJ, k0 = tk * SK;
    const int i0 = ch * th, i1 = min(i0 + th, g.n0);
    const int64_t pl = (int64_t)g.n1 * g.n2, pl1 = (int64_t)(g.n1 + 1) * g.n2,
                  pl2 = (int64_t)g.n1 * (g.n2 + 1);

    // in-plane offsets of the box entries this thread loads (two per array)
    // and their places in the LDS planes.  Entry 0 (e = tid) is in every
    // box.  Entry 1 (e = tid + NT) exists for the first lanes only: whole
    // waves past a box skip it by a branch on the wave index, which is
    // uniform; a lane past the box in the one wave that straddles its end
    // loads and stores its entry 0 again (same address, same value), so no
    // load or store needs a per-lane branch.
    const int wv = __builtin_amdgcn_readfirstlane(tid / WAVE64);
    // (one flag for the psi^n box, one shared by the y1-sized boxes: a wave
    // that reaches into any of them runs the entry-1 work of all of them,
    // the boxes it is past by duplicates)
    constexpr int NW = (NY > N1 ? (NY > N2 ? NY : N2) : (N1 > N2 ? N1 : N2));
    const bool hasP = wv * WAVE64 < NP - NT, hasW = wv * WAVE64 < NW - NT;
    int64_t oP[2], oY[2], o1[2], o2[2];
    int eP[2], eY[2], eW1[2], eW2[2];
    for (int m = 0; m < 2; m++) {
        const int e = tid + m * NT;
        oP[m] = box_offset(e, NP, PK, j0 - 3, k0 - 3, false, false, g, g.n2);
        oY[m] = box_offset(e, NY, BK, j0 - 2, k0 - 2, false, false, g, g.n2);
        o1[m] = box_offset(e, N1, BK, j0 - 2, k0 - 2, true, false, g, g.n2);
        o2[m] = box_offset(e, N2, BK + 1, j0 - 2, k0 - 2, false, true, g, g.n2 + 1);
        eP[m] = eY[m] = eW1[m] = eW2[m] = e;
    }
    if (oP[1] < 0) oP[1] = oP[0], eP[1] = tid;
    if (oY[1] < 0) oY[1] = oY[0], eY[1] = tid;
    if (o1[1] < 0) o1[1] = o1[0], eW1[1] = tid;
    if (o2[1] < 0) o2[1] = o2[0], eW2[1] = tid;
    // y1 cells this thread forms, each at its effective position (the
    // clamped cell outside an open domain): first its own column's cell,
    // then, for the first NRING threads, one cell of the ring of 2 around
    // the tile (rows 0-1, rows SJ+2..SJ+3, then lanes 0-1 and SK+2..SK+3 of
    // the rows between).  Waves past the ring skip the second cell (uniform
    // branch); the lanes past it in the wave that straddles its end form
    // their own cell again and store the same value to the same place.
    constexpr int NRING = NY - NT;
    const bool hasR = wv * WAVE64 < NRING;
    int ye[2], yp[2];
    for (int m = 0; m < 2; m++) {
        int bj, bk;
        if (m == 0 || tid >= NRING) {
            bj = r + 2;
            bk = l + 2;
        } else if (tid < 2 * BK) {
            bj = tid / BK;
            bk = tid % BK;
        } else if (tid < 4 * BK) {
            bj = SJ + 2 + (tid - 2 * BK) / BK;
            bk = (tid - 2 * BK) % BK;
        } else {
            const int q = tid - 4 * BK;
            bj = 2 + q / 4;
            bk = (q & 3) < 2 ? (q & 3) : SK + (q & 3);
        }
        int ej = bj, ek = bk;
        if (g.bc1 == BC_OPEN) ej = min(max(j0 - 2 + bj, 0), g.n1 - 1) - (j0 - 2);
        if (g.bc2 == BC_OPEN) ek = min(max(k0 - 2 + bk, 0), g.n2 - 1) - (k0 - 2);
        ye[m] = ej * BK + ek;      // effective entry in the y1 box
        yp[m] = bj * BK + bk;      // where the result goes
    }

    // pass mode: the pass input is read (plane t into the y1 ring, on the
    // box, at boundary-mapped positions -- what the donor pass forms at the
    // clamped positions) instead of formed by the donor pass
    const T *xin = XIN ? vo.xin : nullptr;
    const bool open0 = g.bc0 == BC_OPEN;
    // prefetched plane values (stored to LDS at the start of the next
    // iteration): psi^n (donor pass) or the pass input, c0 (two entries
    // each), c1, c2, G
    T fP[2], fC0[2], fC1[2], fC2[2], fG[2];
    T fQ0 = T(0), fQ1 = T(0);   // pass mode with the coefficients: psi^n entries
    // The boundary map along i and the ring slots are carried from plane to
    // plane (a wrap test each) instead of formed by a division per use: wt /
    // wt1 are planes t / t+1 wrapped periodically, r3 / r6 the slots
    // slot3(t) / slotp<true>(t) of the plane being brought on chip.
    const int t_first = i0 - 2, t_last = i1 + 1;
    int r3 = slot3(t_first), r6 = slotp<true>(t_first);
    auto sl3 = [&](int k) {     // slot3(t + k), |k| <= 3
        const int v = r3 + k;
        return v < 0 ? v + 3 : (v >= 3 ? v - 3 : v);
    };
    auto slp = [&](int k) {     // slotp<BETA>(t + k), -5 <= k <= 2
        if (!BETA) return sl3(k);
        const int v = r6 + k;
        return v < 0 ? v + 6 : (v >= 6 ? v - 6 : v);
    };
    auto fetch = [&](int t, int wt, int wt1) {
        // psi^n plane t+1, c0 wall t+1, plane t (open: clamped)
        const int64_t ip = (int64_t)(open0 ? min(max(t + 1, 0), g.n0 - 1) : wt1) * pl;
        const int64_t iw = (int64_t)(open0 ? min(max(t + 1, 0), g.n0) : wt1) * pl;
        const int64_t ic = open0 ? min(max(t, 0), g.n0 - 1) : wt;
        #pragma unroll
        for (int m = 0; m < 2; m++) {
            if (m == 0 || hasP) {
                if (!XIN) {
                    fP[m] = x[ip + oP[m]];
                } else if (BETA) {
                    const T v = x[ip + oP[m]];
                    if (m) fQ1 = v;
                    else fQ0 = v;
                }
            }
            if (m == 0 || hasW) {
                if (XIN) fP[m] = xin[ic * pl + oY[m]];
                fC0[m] = c0[iw + oY[m]];
                fC1[m] = c1[ic * pl1 + o1[m]];
                fC2[m] = c2[ic * pl2 + o2[m]];
                if (HAS_G) fG[m] = G[ic * pl + oY[m]];
            }
        }
    };
    auto store = [&](int t) {   // t: the plane of r3 / r6
        const int sp = slp(1), sw = slot4(t + 1), sc = sl3(0);
        // (pass mode, open: planes outside the domain are not stored, so
        // the edge plane's slot stays what those planes read)
        const bool xplane = XIN && (!open0 || (t >= 0 && t < g.n0));
        #pragma unroll
        for (int m = 0; m < 2; m++) {
            if (m == 0 || hasP) {
                if (!XIN) Ps[sp][eP[m]] = fP[m];
                else if (BETA) Ps[sp][eP[m]] = m ? fQ1 : fQ0;
            }
            if (m == 0 || hasW) {
                if (XIN && xplane) Ys[slot4(t)][eY[m]] = fP[m];
                C0s[sw][eY[m]] = fC0[m];
                C1s[sc][eW1[m]] = fC1[m];
                C2s[sc][eW2[m]] = fC2[m];
                if (HAS_G) Gs[sc][eY[m]] = fG[m];
            }
        }
    };

    // prologue: psi^n planes t_first-1 and t_first, c0 wall t_first
    {
        const int64_t ipm = map_cell(t_first - 1, g.n0, g.bc0) * pl;
        const int64_t ip0 = map_cell(t_first, g.n0, g.bc0) * pl;
        const int64_t iw0 = map_wall(t_first, g.n0, g.bc0) * pl;
        #pragma unroll
        for (int m = 0; m < 2; m++) {
            if ((!XIN || BETA) && (m == 0 || hasP)) {
                Ps[slotp<BETA>(t_first - 1)][eP[m]] = x[ipm + oP[m]];
                Ps[slotp<BETA>(t_first)][eP[m]] = x[ip0 + oP[m]];
            }
            if (m == 0 || hasW) C0s[slot4(t_first)][eY[m]] = c0[iw0 + oY[m]];
        }
    }
    int w1 = (int)map_cell(t_first + 1, g.n0, BC_PERIODIC);
    int w2 = w1 + 1 == g.n0 ? 0 : w1 + 1;
    fetch(t_first, (int)map_cell(t_first, g.n0, BC_PERIODIC), w1);

    // y1 ring slot of virtual plane q (open: planes outside the domain read
    // the edge plane)
    auto yslot = [&](int q) { return slot4(open0 ? min(max(q, 0), g.n0 - 1) : q); };
    // own cell in the boxes
    const int bj = r + 2, bk = l + 2;
    const int cy = bj * BK + bk;
    const bool own_out = j0 + r < g.n1 && k0 + l < g.n2;
    T v0_lo = T(0);      // V0 at the low wall of the plane being corrected
    T y_own = T(0);      // y1 of plane t of the thread's own column

    for (int t = t_first; t <= t_last; t++, r3 = r3 == 2 ? 0 : r3 + 1, r6 = r6 == 5 ? 0 : r6 + 1,
                                         w1 = w2, w2 = w2 + 1 == g.n0 ? 0 : w2 + 1) {
        store(t);
        if (t < t_last) fetch(t + 1, w1, w2);
        __syncthreads();   // (B1) plane t's inputs are in LDS

        // ---- donor-cell pass: y1 of plane t on the box ----
        if (XIN) {
            if (!open0 || (t >= 0 && t < g.n0)) y_own = Ys[slot4(t)][cy];
        } else if (!open0 || (t >= 0 && t < g.n0)) {
            const int pm = slp(-1), p0 = slp(0), pp = slp(1);
            const int wl = slot4(t), wh = slot4(t + 1), sc = sl3(0), sy = slot4(t);
            for (int m = 0; m < 2; m++) {
                if (m == 1 && !hasR) continue;
                const int ee = ye[m];
                const int ej = ee / BK, ek = ee % BK;
                const int q = (ej + 1) * PK + (ek + 1);        // psi^n box entry
                const T xc = Ps[p0][q];
                T dv[3];
                {
                    T flo = upwind_fp(C0s[wl][ee], Ps[pm][q], xc);
                    T fhi = upwind_fp(C0s[wh][ee], xc, Ps[pp][q]);
                    dv[0] = fhi - flo;
                }
                {
                    T flo = upwind_fp(C1s[sc][ej * BK + ek], Ps[p0][q - PK], xc);
                    T fhi = upwind_fp(C1s[sc][(ej + 1) * BK + ek], xc, Ps[p0][q + PK]);
                    dv[1] = fhi - flo;
                }
                {
                    T flo = upwind_fp(C2s[sc][ej * (BK + 1) + ek], Ps[p0][q - 1], xc);
                    T fhi = upwind_fp(C2s[sc][ej * (BK + 1) + ek + 1], xc, Ps[p0][q + 1]);
                    dv[2] = fhi - flo;
                }
                T y;
                if (kahan) {
                    T ks = xc, kc = T(0);
#pragma unroll
                    for (int d = 0; d < 3; d++)
                        kahan_add(ks, kc, -(HAS_G ? dv[d] / Gs[sc][ee] : dv[d]));
                    y = ks;
                } else {
                    T acc = T(0);
                    acc += dv[0];
                    acc += dv[1];
                    acc += dv[2];
                    y = xc - (HAS_G ? acc / Gs[sc][ee] : acc);
                }
                Ys[sy][yp[m]] = y;
                if (m == 0) y_own = y;
            }
        }
        // No barrier here: the pseudo-velocities of plane t-2 read y1 of
        // planes t-3..t-1 only (written before the barrier above), except
        // the third-order term of V0, which takes plane t of the thread's
        // own column from y_own (or, past an open domain's last plane, the
        // edge plane's slot).  The ring cells of plane t are read from the
        // next iteration on, after its barrier.

        // ---- pseudo-velocities ----
        const int p = t - 2;
        const int sA = yslot(p - 1), sB = yslot(p), sC = yslot(p + 1), sD = yslot(p + 2);
        const int cs = sl3(-2), cs1 = sl3(-1);            // c1, c2, G planes p, p+1
        const int ws = slot4(p), ws1 = slot4(p + 1);      // c0 walls p, p+1
        const T *YA = Ys[sA], *YB = Ys[sB], *YC = Ys[sC];

        // V0 at wall p+1 (planes p | p+1) of column (bj, bk)
        // psi value entering a psi-fraction: |psi| under the abs option
        auto ya = [](T v) -> T { return ABS ? fabs(v) : v; };
        // 1 / mean G at the own cell's three low walls, formed as one set
        // (one range test for the quotients; the far-edge walls form their
        // own); in FP64 without the coefficients the set also holds 1 / G of
        // the own cell for the corrective pass's quotient (gfast: the set
        // took the refined form)
        T igo[4] = {T(1), T(1), T(1), T(1)};
        bool gfast = false;
        if (HAS_G) {
            T gb[4] = {T(0.5) * (Gs[cs][cy] + Gs[cs1][cy]), T(0.5) * (Gs[cs][cy - BK] + Gs[cs][cy]),
                       T(0.5) * (Gs[cs][cy - 1] + Gs[cs][cy]), Gs[cs][cy]};
            if constexpr (std::is_same<T, double>::value && !BETA) {
                gfast = rcp_set<4>(gb, igo);
            } else {
                // (with the coefficients the launch is in output mode: no
                // corrective pass; gfast stays false)
                T one[3] = {T(1), T(1), T(1)}, g3[3] = {gb[0], gb[1], gb[2]}, q3[3];
                quotients<3>(one, g3, q3);
                igo[0] = q3[0];
                igo[1] = q3[1];
                igo[2] = q3[2];
            }
        }
        auto vel0 = [&]() -> T {
            const int c = cy;
            const T ig = igo[0];
            const T xL = ya(YB[c]), xR = ya(YC[c]);
            const T u = C0s[ws1][c];
            T A = fr3<T, IGA>(xR - xL, xR + xL, T(2));
            T v = (fabs(u) - u * u * ig) * A;
            const int w1 = bj * BK + bk, w1p = (bj + 1) * BK + bk;
            const T s1a = C1s[cs][w1] + C1s[cs1][w1], s1b = C1s[cs][w1p] + C1s[cs1][w1p];
            const int w2 = bj * (BK + 1) + bk;
            const T s2a = C2s[cs][w2] + C2s[cs1][w2], s2b = C2s[cs][w2 + 1] + C2s[cs1][w2 + 1];
            const T cb1 = T(0.25) * (s1a + s1b);
            const T cb2 = T(0.25) * (s2a + s2b);
            // o = 1 (j)
            T a1 = ya(YC[c + BK]), b1 = ya(YB[c + BK]), e1 = ya(YC[c - BK]), f1 = ya(YB[c - BK]);
            v -= T(0.5) * u * cb1 * ig * fr3<T, IGA>(a1 + b1 - e1 - f1, a1 + b1 + e1 + f1, T(4));
            // o = 2 (k)
            T a2 = ya(YC[c + 1]), b2 = ya(YB[c + 1]), e2 = ya(YC[c - 1]), f2 = ya(YB[c - 1]);
            v -= T(0.5) * u * cb2 * ig * fr3<T, IGA>(a2 + b2 - e2 - f2, a2 + b2 + e2 + f2, T(4));
            if (DFL) {
                // divergent-flow term: the mean of the two cells' advector
                // divergences (planes p and p+1 of the column), times
                // -c / (2 Gb); under iga times the wall mean of psi
                const int ws2 = slot4(p + 2);
                T dv = (C0s[ws1][c] - C0s[ws][c]) + (C0s[ws2][c] - C0s[ws1][c]);
                dv += (C1s[cs][w1p] - C1s[cs][w1]) + (C1s[cs1][w1p] - C1s[cs1][w1]);
                dv += (C2s[cs][w2 + 1] - C2s[cs][w2]) + (C2s[cs1][w2 + 1] - C2s[cs1][w2]);
                if (IGA) dv *= T(0.5) * (xL + xR);
                v -= T(0.25) * u * ig * dv;
            }
            if (TOT) {
                const T xR2 = (open0 && t >= g.n0) ? ya(Ys[sD][c]) : ya(y_own), xL2 = ya(YA[c]);
                v += (T(3) * u * fabs(u) * ig - T(2) * u * u * u * (ig * ig) - u) * (T(1) / T(3)) *
                     fr3<T, IGA>(xR2 - xR - xL + xL2, xR2 + xR + xL + xL2, T(4));
                v += (fabs(u) * cb1 * ig - T(2) * u * u * cb1 * (ig * ig)) *
                     fr3<T, IGA>(a1 - b1 - e1 + f1, a1 + b1 + e1 + f1, T(4));
                v += (fabs(u) * cb2 * ig - T(2) * u * u * cb2 * (ig * ig)) *
                     fr3<T, IGA>(a2 - b2 - e2 + f2, a2 + b2 + e2 + f2, T(4));
                T num = T(0), den = T(0);
                for (int sd = 0; sd < 2; sd++) {
                    const T *Yp = sd ? YC : YB;
                    T pp_ = ya(Yp[c + BK + 1]), mp_ = ya(Yp[c - BK + 1]), pm_ = ya(Yp[c + BK - 1]),
                      mm_ = ya(Yp[c - BK - 1]);
                    num += pp_ - mp_ - pm_ + mm_;
                    den += pp_ + mp_ + pm_ + mm_;
                }
                v += -(T(2) / T(3)) * u * cb1 * cb2 * (ig * ig) * fr3<T, IGA>(num, den, T(8));
            }
            return v;
        };
        // V1 at plane p, wall between box rows wj-1 | wj, lane wk
        // (own: the own cell's wall, whose 1 / mean G is in igo)
        auto vel1 = [&](int wj, int wk, bool own) -> T {
            const int c = wj * BK + wk;
            T ig = igo[1];
            if (HAS_G && !own) {
                T one[1] = {T(1)}, gb[1] = {T(0.5) * (Gs[cs][c - BK] + Gs[cs][c])}, q[1];
                quotients<1>(one, gb, q);
                ig = q[0];
            }
            const T xL = ya(YB[c - BK]), xR = ya(YB[c]);
            const T u = C1s[cs][c];
            T A = fr3<T, IGA>(xR - xL, xR + xL, T(2));
            T v = (fabs(u) - u * u * ig) * A;
            const T cb0 = T(0.25) * ((C0s[ws][c - BK] + C0s[ws1][c - BK]) + (C0s[ws][c] + C0s[ws1][c]));
            const int w2 = wj * (BK + 1) + wk, w2m = (wj - 1) * (BK + 1) + wk;
            const T cb2 = T(0.25) * ((C2s[cs][w2m] + C2s[cs][w2m + 1]) + (C2s[cs][w2] + C2s[cs][w2 + 1]));
            // o = 0 (i)
            T a0 = ya(YC[c]), b0 = ya(YC[c - BK]), e0 = ya(YA[c]), f0 = ya(YA[c - BK]);
            v -= T(0.5) * u * cb0 * ig * fr3<T, IGA>(a0 + b0 - e0 - f0, a0 + b0 + e0 + f0, T(4));
            // o = 2 (k)
            T a2 = ya(YB[c + 1]), b2 = ya(YB[c - BK + 1]), e2 = ya(YB[c - 1]), f2 = ya(YB[c - BK - 1]);
            v -= T(0.5) * u * cb2 * ig * fr3<T, IGA>(a2 + b2 - e2 - f2, a2 + b2 + e2 + f2, T(4));
            if (DFL) {
                // cells (p, wj-1) and (p, wj)
                T dv = (C0s[ws1][c - BK] - C0s[ws][c - BK]) + (C0s[ws1][c] - C0s[ws][c]);
                dv += (C1s[cs][c] - C1s[cs][c - BK]) + (C1s[cs][c + BK] - C1s[cs][c]);
                dv += (C2s[cs][w2m + 1] - C2s[cs][w2m]) + (C2s[cs][w2 + 1] - C2s[cs][w2]);
                if (IGA) dv *= T(0.5) * (xL + xR);
                v -= T(0.25) * u * ig * dv;
            }
            if (TOT) {
                const T xR2 = ya(YB[c + BK]), xL2 = ya(YB[c - 2 * BK]);
                v += (T(3) * u * fabs(u) * ig - T(2) * u * u * u * (ig * ig) - u) * (T(1) / T(3)) *
                     fr3<T, IGA>(xR2 - xR - xL + xL2, xR2 + xR + xL + xL2, T(4));
                v += (fabs(u) * cb0 * ig - T(2) * u * u * cb0 * (ig * ig)) *
                     fr3<T, IGA>(a0 - b0 - e0 + f0, a0 + b0 + e0 + f0, T(4));
                v += (fabs(u) * cb2 * ig - T(2) * u * u * cb2 * (ig * ig)) *
                     fr3<T, IGA>(a2 - b2 - e2 + f2, a2 + b2 + e2 + f2, T(4));
                T num = T(0), den = T(0);
                for (int sd = 0; sd < 2; sd++) {
                    const int cc = sd ? c : c - BK;
                    T pp_ = ya(YC[cc + 1]), mp_ = ya(YA[cc + 1]), pm_ = ya(YC[cc - 1]), mm_ = ya(YA[cc - 1]);
                    num += pp_ - mp_ - pm_ + mm_;
                    den += pp_ + mp_ + pm_ + mm_;
                }
                v += -(T(2) / T(3)) * u * cb0 * cb2 * (ig * ig) * fr3<T, IGA>(num, den, T(8));
            }
            return v;
        };
        // V2 at plane p, wall between box lanes wk-1 | wk, row wj
        auto vel2 = [&](int wj, int wk, bool own) -> T {
            const int c = wj * BK + wk;
            T ig = igo[2];
            if (HAS_G && !own) {
                T one[1] = {T(1)}, gb[1] = {T(0.5) * (Gs[cs][c - 1] + Gs[cs][c])}, q[1];
                quotients<1>(one, gb, q);
                ig = q[0];
            }
            const T xL = ya(YB[c - 1]), xR = ya(YB[c]);
            const T u = C2s[cs][wj * (BK + 1) + wk];
            T A = fr3<T, IGA>(xR - xL, xR + xL, T(2));
            T v = (fabs(u) - u * u * ig) * A;
            const T cb0 = T(0.25) * ((C0s[ws][c - 1] + C0s[ws1][c - 1]) + (C0s[ws][c] + C0s[ws1][c]));
            const T cb1 = T(0.25) * ((C1s[cs][c - 1] + C1s[cs][c - 1 + BK]) + (C1s[cs][c] + C1s[cs][c + BK]));
            // o = 0 (i)
            T a0 = ya(YC[c]), b0 = ya(YC[c - 1]), e0 = ya(YA[c]), f0 = ya(YA[c - 1]);
            v -= T(0.5) * u * cb0 * ig * fr3<T, IGA>(a0 + b0 - e0 - f0, a0 + b0 + e0 + f0, T(4));
            // o = 1 (j)
            T a1 = ya(YB[c + BK]), b1 = ya(YB[c + BK - 1]), e1 = ya(YB[c - BK]), f1 = ya(YB[c - BK - 1]);
            v -= T(0.5) * u * cb1 * ig * fr3<T, IGA>(a1 + b1 - e1 - f1, a1 + b1 + e1 + f1, T(4));
            if (DFL) {
                // cells (p, wj, wk-1) and (p, wj, wk)
                const int w2 = wj * (BK + 1) + wk;
                T dv = (C0s[ws1][c - 1] - C0s[ws][c - 1]) + (C0s[ws1][c] - C0s[ws][c]);
                dv += (C1s[cs][c - 1 + BK] - C1s[cs][c - 1]) + (C1s[cs][c + BK] - C1s[cs][c]);
                dv += (C2s[cs][w2] - C2s[cs][w2 - 1]) + (C2s[cs][w2 + 1] - C2s[cs][w2]);
                if (IGA) dv *= T(0.5) * (xL + xR);
                v -= T(0.25) * u * ig * dv;
            }
            if (TOT) {
                const T xR2 = ya(YB[c + 1]), xL2 = ya(YB[c - 2]);
                v += (T(3) * u * fabs(u) * ig - T(2) * u * u * u * (ig * ig) - u) * (T(1) / T(3)) *
                     fr3<T, IGA>(xR2 - xR - xL + xL2, xR2 + xR + xL + xL2, T(4));
                v += (fabs(u) * cb0 * ig - T(2) * u * u * cb0 * (ig * ig)) *
                     fr3<T, IGA>(a0 - b0 - e0 + f0, a0 + b0 + e0 + f0, T(4));
                v += (fabs(u) * cb1 * ig - T(2) * u * u * cb1 * (ig * ig)) *
                     fr3<T, IGA>(a1 - b1 - e1 + f1, a1 + b1 + e1 + f1, T(4));
                T num = T(0), den = T(0);
                for (int sd = 0; sd < 2; sd++) {
                    const int cc = sd ? c : c - 1;
                    T pp_ = ya(YC[cc + BK]), mp_ = ya(YA[cc + BK]), pm_ = ya(YC[cc - BK]), mm_ = ya(YA[cc - BK]);
                    num += pp_ - mp_ - pm_ + mm_;
                    den += pp_ + mp_ + pm_ + mm_;
                }
                v += -(T(2) / T(3)) * u * cb0 * cb1 * (ig * ig) * fr3<T, IGA>(num, den, T(8));
            }
            return v;
        };

        const T v0_hi = vel0();
        if (vo.v0) {
            // output mode: the donor result and the raw pseudo-velocities of
            // the chunk's planes (V0 at its walls), each entry by its owner
            // -- the low walls of the tile's cells, and along an open
            // dimension the domain's far edge walls -- for the limiter's
            // kernels, instead of the corrective pass
            const int jj = j0 + r, kk = k0 + l;
            const int64_t n1 = g.n1, n2 = g.n2;
            const bool o0 = g.bc0 == BC_OPEN, o1 = g.bc1 == BC_OPEN, o2 = g.bc2 == BC_OPEN;
            const int w0 = p + 1;
            if (own_out && ((w0 >= i0 && w0 < i1) || (o0 && w0 == g.n0 && i1 == g.n0)))
                vo.v0[((int64_t)w0 * n1 + jj) * n2 + kk] = v0_hi;
            if (p >= i0 && p < i1) {
                if (own_out && vo.y1) vo.y1[((int64_t)p * n1 + jj) * n2 + kk] = YB[cy];
                const T v1o = vel1(bj, bk, true), v2o = vel2(bj, bk, true);
                if (kk < g.n2 && (jj < g.n1 || (o1 && jj == g.n1)))
                    vo.v1[((int64_t)p * (n1 + 1) + jj) * n2 + kk] = v1o;
                if (jj < g.n1 && (kk < g.n2 || (o2 && kk == g.n2)))
                    vo.v2[((int64_t)p * n1 + jj) * (n2 + 1) + kk] = v2o;
                if (BETA) {
                    // the coefficients read the high walls of the own cell
                    V1s[r * SK + l] = v1o;
                    V2s[r * (SK + 1) + l] = v2o;
                }
                if (tid < SK) {                                            // far j edge
                    const int je = j0 + SJ, ke = k0 + tid;
                    const bool wr = o1 && je == g.n1 && ke < g.n2;
                    if (BETA || wr) {
                        const T v = vel1(SJ + 2, tid + 2, false);
                        if (wr) vo.v1[((int64_t)p * (n1 + 1) + je) * n2 + ke] = v;
                        if (BETA) V1s[SJ * SK + tid] = v;
                    }
                } else if (tid < SK + SJ) {                                // far k edge
                    const int je = j0 + tid - SK, ke = k0 + SK;
                    const bool wr = o2 && ke == g.n2 && je < g.n1;
                    if (BETA || wr) {
                        const T v = vel2(tid - SK + 2, SK + 2, false);
                        if (wr) vo.v2[((int64_t)p * n1 + je) * (n2 + 1) + ke] = v;
                        if (BETA) V2s[(tid - SK) * (SK + 1) + SK] = v;
                    }
                }
            }
        } else {
            V1s[r * SK + l] = vel1(bj, bk, true);
            V2s[r * (SK + 1) + l] = vel2(bj, bk, true);
            if (tid < SK) V1s[SJ * SK + tid] = vel1(SJ + 2, tid + 2, false);  // far j edge
            else if (tid < SK + SJ)
                V2s[(tid - SK) * (SK + 1) + SK] = vel2(tid - SK + 2, SK + 2, false);
        }
        T g_own = T(1);
        if (HAS_G) g_own = Gs[cs][cy];
        // the pass input at the own cell of plane p and its face neighbours,
        // for the limiter coefficients (read before the barrier: in pass
        // mode the next iteration stores plane t+1 into the slot of p-1)
        T xn[7];
        if (BETA) {
            xn[0] = YB[cy];
            xn[1] = YA[cy];
            xn[2] = YC[cy];
            xn[3] = YB[cy - BK];
            xn[4] = YB[cy + BK];
            xn[5] = YB[cy - 1];
            xn[6] = YB[cy + 1];
        }
        // (B3) V1, V2 of plane p are in LDS; and (in both modes) no thread
        // stores the next planes into the rings before every thread is done
        // reading this iteration's
        __syncthreads();

        // ---- limiter coefficients of plane p (BETA; the arithmetic of the
        // cell kernel k_fct_beta term by term) ----
        if (BETA && p >= i0 && p < i1 && own_out) {
            // psi^n of the same cells (planes p-1..p+1 stay in the ring until
            // the iteration after next)
            T pn[7];
            const int qo = (r + 3) * PK + (l + 3);
            const T *P0 = Ps[slp(-2)];
            pn[0] = P0[qo];
            pn[1] = Ps[slp(-3)][qo];
            pn[2] = Ps[slp(-1)][qo];
            pn[3] = P0[qo - PK];
            pn[4] = P0[qo + PK];
            pn[5] = P0[qo - 1];
            pn[6] = P0[qo + 1];
            const T xi = xn[0];
            T mx = pn[0], mn = mx;
            mx = fmax(mx, xi);
            mn = fmin(mn, xi);
            // face neighbours in the order -e0, +e0, -e1, +e1, -e2, +e2
#pragma unroll
            for (int q = 0; q < 6; q++) {
                mx = fmax(fmax(mx, pn[1 + q]), xn[1 + q]);
                mn = fmin(fmin(mn, pn[1 + q]), xn[1 + q]);
            }
            const T vlo[3] = {v0_lo, V1s[r * SK + l], V2s[r * (SK + 1) + l]};
            const T vhi[3] = {v0_hi, V1s[(r + 1) * SK + l], V2s[r * (SK + 1) + l + 1]};
            T fin = T(0), fout = T(0);
#pragma unroll
            for (int d = 0; d < 3; d++) {
                const T wm = IGA ? T(1) : xn[1 + 2 * d], wp = IGA ? T(1) : xn[2 + 2 * d];
                const T wi = IGA ? T(1) : xi;
                fin += pos(vlo[d]) * wm - neg(vhi[d]) * wp;
                fout += pos(vhi[d]) * wi - neg(vlo[d]) * wi;
            }
            const T Gi = HAS_G ? g_own : T(1);
            const int64_t idx = ((int64_t)p * g.n1 + (j0 + r)) * g.n2 + (k0 + l);
            vo.bup[idx] = fin > T(0) ? Gi * (mx - xi) / fin : T(1);
            vo.bdn[idx] = fout > T(0) ? Gi * (xi - mn) / fout : T(1);
        }

        // ---- corrective pass at plane p ----
        if (!vo.v0 && p >= i0 && p < i1 && own_out) {
            const T xo = YB[cy];
            const T V0lo = v0_lo, V0hi = v0_hi;
            const T V1lo = V1s[r * SK + l], V1hi = V1s[(r + 1) * SK + l];
            const T V2lo = V2s[r * (SK + 1) + l], V2hi = V2s[r * (SK + 1) + l + 1];
            T f0lo, f0hi, f1lo, f1hi, f2lo, f2hi;
            if (IGA) {
                f0lo = V0lo; f0hi = V0hi; f1lo = V1lo; f1hi = V1hi; f2lo = V2lo; f2hi = V2hi;
            } else {
                f0lo = pos(V0lo) * YA[cy] + neg(V0lo) * xo;
                f0hi = pos(V0hi) * xo + neg(V0hi) * YC[cy];
                f1lo = pos(V1lo) * YB[cy - BK] + neg(V1lo) * xo;
                f1hi = pos(V1hi) * xo + neg(V1hi) * YB[cy + BK];
                f2lo = pos(V2lo) * YB[cy - 1] + neg(V2lo) * xo;
                f2hi = pos(V2hi) * xo + neg(V2hi) * YB[cy + 1];
            }
            T res;
            if (kahan) {
                T dv[3] = {f0hi - f0lo, f1hi - f1lo, f2hi - f2lo};
                if (HAS_G) {
                    if constexpr (std::is_same<T, double>::value) {
#pragma unroll
                        for (int d = 0; d < 3; d++) dv[d] = gfast ? dv[d] * igo[3] : dv[d] / g_own;
                    } else {
                        T gg[3] = {g_own, g_own, g_own}, qq[3];
                        quotients<3>(dv, gg, qq);
                        dv[0] = qq[0];
                        dv[1] = qq[1];
                        dv[2] = qq[2];
                    }
                }
                T ks = xo, kc = T(0);
#pragma unroll
                for (int d = 0; d < 3; d++) kahan_add(ks, kc, -dv[d]);
                res = ks;
            } else {
                T acc = T(0);
                acc += f0hi - f0lo;
                acc += f1hi - f1lo;
                acc += f2hi - f2lo;
                if (HAS_G) {
                    if constexpr (std::is_same<T, double>::value) {
                        acc = gfast ? acc * igo[3] : acc / g_own;
                    } else {
                        T nn[1] = {acc}, dd[1] = {g_own}, qq[1];
                        quotients<1>(nn, dd, qq);
                        acc = qq[0];
                    }
                }
                res = xo - acc;
            }
            out[((int64_t)p * g.n1 + (j0 + r)) * g.n2 + (k0 + l)] = res;
        }
        v0_lo = v0_hi;
    }
}

}  // namespace

bool step3d_supported(int nd, int n_iters, unsigned opts, const int64_t n[3])
{
    // (with the limiter or more than two passes the kernel runs pass by
    // pass in output mode, see fused3d_step)
    if (nd != 3 || n_iters < 2) return false;
    // 32-bit plane and row indices inside the kernel
    if (n[0] >= (1 << 30) || n[1] >= (1 << 30) || n[2] >= (1 << 30)) return false;
    return true;
}

template <typename T>
hipError_t step3d_launch(const Geom &geom, unsigned opts, const T *psi_n, T *psi_out, const T *c0,
                         const T *c1, const T *c2, const T *G, int tile_planes, hipStream_t s,
                         const Step3dOut<T> &vo)
{
    // the coefficients are formed only in output mode
    if (vo.bup && (!vo.bdn || !vo.v0)) return hipErrorInvalidValue;
    G3s g{(int)geom.n[0], (int)geom.n[1], (int)geom.n[2], geom.bc[0], geom.bc[1], geom.bc[2]};
    const int tiles_k = (g.n2 + SK - 1) / SK, tiles_j = (g.n1 + SJ - 1) / SJ;
    int th = tile_planes > 0 ? tile_planes : 96;
    if (th > g.n0) th = g.n0;
    const int64_t chunks = cdiv(g.n0, th);
    const int64_t blocks = (int64_t)tiles_k * tiles_j * chunks;
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    const int kahan = (opts & OPT_KAHAN) ? 1 : 0;
    const bool iga = opts & OPT_IGA, absf = opts & OPT_ABS, dfl = opts & OPT_DFL,
               tot = opts & OPT_TOT;
    auto go = [&](auto HG, auto IG, auto AB, auto DF, auto TO, auto XI, auto BE) {
        k_step3d<T, decltype(HG)::value, decltype(IG)::value, decltype(AB)::value,
                 decltype(DF)::value, decltype(TO)::value, decltype(XI)::value,
                 decltype(BE)::value><<<(unsigned)blocks, NT, 0, s>>>(
            g, th, tiles_k, tiles_j, (int)blocks, kahan, psi_n, c0, c1, c2, G, psi_out, vo);
    };
    using TT = std::true_type;
    using FF = std::false_type;
    // pass mode reads its input; with bup / bdn the coefficients too
    auto by_x = [&](auto HG, auto IG, auto AB, auto DF, auto TO) {
        if (vo.xin) {
            if (vo.bup) go(HG, IG, AB, DF, TO, TT{}, TT{});
            else go(HG, IG, AB, DF, TO, TT{}, FF{});
        } else {
            if (vo.bup) go(HG, IG, AB, DF, TO, FF{}, TT{});
            else go(HG, IG, AB, DF, TO, FF{}, FF{});
        }
    };
    auto by_t = [&](auto HG, auto IG, auto AB, auto DF) {
        if (tot) by_x(HG, IG, AB, DF, TT{});
        else by_x(HG, IG, AB, DF, FF{});
    };
    auto by_d = [&](auto HG, auto IG, auto AB) {
        if (dfl) by_t(HG, IG, AB, TT{});
        else by_t(HG, IG, AB, FF{});
    };
    auto by_m = [&](auto HG) {       // psi-fractions: plain, infinite gauge or |psi|
        if (iga) by_d(HG, TT{}, FF{});
        else if (absf) by_d(HG, FF{}, TT{});
        else by_d(HG, FF{}, FF{});
    };
    if (G) by_m(TT{});
    else by_m(FF{});
    return hipGetLastError();
}

template hipError_t step3d_launch<float>(const Geom &, unsigned, const float *, float *,
                                         const float *, const float *, const float *,
                                         const float *, int, hipStream_t,
                                         const Step3dOut<float> &);
template hipError_t step3d_launch<double>(const Geom &, unsigned, const double *, double *,
                                          const double *, const double *, const double *,
                                          const double *, int, hipStream_t,
                                          const Step3dOut<double> &);

}  // namespace mp
