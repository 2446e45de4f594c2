// fused3d.hip -- 3-D MPDATA step with two passes and no limiter in two
// launches (the three-dimensional workload: third-order terms, infinite
// gauge, variable G, open boundaries).
//
//   k_donor3d : donor-cell pass, psi^n -> y1 (workspace).  Each thread owns a
//               (j, k) column and marches along i over a chunk of planes,
//               keeping psi at i-1, i, i+1 and the dimension-0 walls in
//               registers; in-plane neighbours are read through L1/L2.
//   k_corr3d  : pseudo-velocity on every wall and the corrective pass,
//               y1 -> psi^{n+1}.  A workgroup of 16 x 32 (FP64) or 16 x 64
//               (FP32) threads owns a (j, k) tile with a halo of two cells and
//               marches along i.  Each thread keeps its own column's planes in
//               registers; the in-plane neighbours it needs come through LDS
//               (two barriers per plane).  The pseudo-velocity of each wall is
//               computed once: V0 by the cell above it, V1 / V2 by the cell
//               after it.
// Every global read goes through the boundary map (periodic wrap / open
// clamp), so halo positions hold mapped values and the computed walls equal
// the staged path's walls.  A thread's (j, k) part of every address is fixed,
// so the per-plane part is uniform scalar arithmetic.  Tiles are numbered so
// that neighbouring tiles run on the same XCD and share its L2 for their
// overlapping halo reads.
#include "common.hpp"
#include "kernels.hpp"

#include <type_traits>

namespace mp {
namespace {

constexpr int TR = 16;   // tile rows (j) incl. halo
constexpr int HALO = 2;
// tile lanes (k) incl. halo: 64 for FP32; 32 for FP64, whose per-thread
// state needs more than the 128 registers a 1024-thread workgroup allows
template <typename T> struct TileL {
    static constexpr int v = sizeof(T) == 8 ? 32 : 64;
};

struct G3 {
    int n0, n1, n2;
    int bc0, bc1, bc2;
};

// ---- donor-cell pass ----------------------------------------------------
constexpr int DONOR_PLANES = 16;   // planes per thread column

// Blocks of 64 (k) x 4 (j) columns over DONOR_PLANES planes; a 1-D grid of
// nblk blocks.  The hardware deals block b to XCD b % 8: block b takes tile
// number x * (nblk / 8) + ... (x = b % 8), so each XCD runs a contiguous
// range of tiles, k fastest, then j, and the rows a tile reads above and
// below its own (the in-plane neighbours) are mostly read by tiles on the
// same XCD, through its L2.
template <typename T, bool HAS_G>
__global__ void __launch_bounds__(256) k_donor3d(G3 g, int kahan, int tiles_k, int tiles_j,
                                                 int nblk, const T *__restrict__ x,
                                                 const T *__restrict__ c0,
                                                 const T *__restrict__ c1,
                                                 const T *__restrict__ c2,
                                                 const T *__restrict__ G, T *__restrict__ y)
{
    int b;
    {
        const int xcd = blockIdx.x & 7, per = nblk >> 3, rem = nblk & 7;
        b = xcd * per + (xcd < rem ? xcd : rem) + (blockIdx.x >> 3);
    }
    const int tk = b % tiles_k;
    b /= tiles_k;
    const int tj = b % tiles_j;
    const int ch = b / tiles_j;
    const int k = tk * 64 + (threadIdx.x & 63);
    const int j = tj * 4 + (threadIdx.x >> 6);
    const int i0 = ch * DONOR_PLANES;
    const int i1 = min(i0 + DONOR_PLANES, g.n0);
    if (k >= g.n2 || j >= g.n1) return;
    const int64_t pl = (int64_t)g.n1 * g.n2;                 // cell / c0 plane
    const int64_t pl1 = (int64_t)(g.n1 + 1) * g.n2;          // c1 plane
    const int64_t pl2 = (int64_t)g.n1 * (g.n2 + 1);          // c2 plane
    // in-plane offsets (fixed for the column)
    const int64_t o = (int64_t)j * g.n2 + k;
    const int64_t ojm = (int64_t)wrap_cell(j - 1, g.n1, g.bc1) * g.n2 + k;
    const int64_t ojp = (int64_t)wrap_cell(j + 1, g.n1, g.bc1) * g.n2 + k;
    const int64_t okm = (int64_t)j * g.n2 + wrap_cell(k - 1, g.n2, g.bc2);
    const int64_t okp = (int64_t)j * g.n2 + wrap_cell(k + 1, g.n2, g.bc2);
    const int64_t w1lo = (int64_t)j * g.n2 + k;
    const int64_t w1hi = (int64_t)wrap_wall(j + 1, g.n1, g.bc1) * g.n2 + k;
    const int64_t w2lo = (int64_t)j * (g.n2 + 1) + k;
    const int64_t w2hi = (int64_t)j * (g.n2 + 1) + wrap_wall(k + 1, g.n2, g.bc2);

    T xm = x[wrap_cell(i0 - 1, g.n0, g.bc0) * pl + o];
    T xc = x[i0 * pl + o];
    T ulo = c0[i0 * pl + o];
    for (int i = i0; i < i1; i++) {
        const int64_t pc = i * pl;
        T xp = x[wrap_cell(i + 1, g.n0, g.bc0) * pl + o];
        T uhi = c0[wrap_wall(i + 1, g.n0, g.bc0) * pl + o];
        T dv[3];
        {
            T flo = pos(ulo) * xm + neg(ulo) * xc;
            T fhi = pos(uhi) * xc + neg(uhi) * xp;
            dv[0] = fhi - flo;
        }
        {
            T ul = c1[i * pl1 + w1lo], uh = c1[i * pl1 + w1hi];
            T flo = pos(ul) * x[pc + ojm] + neg(ul) * xc;
            T fhi = pos(uh) * xc + neg(uh) * x[pc + ojp];
            dv[1] = fhi - flo;
        }
        {
            T ul = c2[i * pl2 + w2lo], uh = c2[i * pl2 + w2hi];
            T flo = pos(ul) * x[pc + okm] + neg(ul) * xc;
            T fhi = pos(uh) * xc + neg(uh) * x[pc + okp];
            dv[2] = fhi - flo;
        }
        if (kahan) {
            T ks = xc, kc = T(0);
#pragma unroll
            for (int d = 0; d < 3; d++) kahan_add(ks, kc, -(HAS_G ? dv[d] / G[pc + o] : dv[d]));
            y[pc + o] = ks;
        } else {
            T acc = T(0);
            acc += dv[0];
            acc += dv[1];
            acc += dv[2];
            y[pc + o] = xc - (HAS_G ? acc / G[pc + o] : acc);
        }
        xm = xc;
        xc = xp;
        ulo = uhi;
    }
}

template <typename T, bool IGA> __device__ inline T fr(T num, T den, T m)
{
    if (IGA) return num * (T(1) / m);
    return den == T(0) ? T(0) : num / den;
}

// ---- pseudo-velocity + corrective pass ---------------------------------
template <typename T, bool HAS_G, bool IGA, bool TOT>
__global__ void __launch_bounds__(TR * TileL<T>::v)
k_corr3d(G3 g, int th, int tiles_k, int tiles_j, int nblk, int kahan, const T *__restrict__ y1,
                                                    const T *__restrict__ c0,
                                                    const T *__restrict__ c1,
                                                    const T *__restrict__ c2,
                                                    const T *__restrict__ G,
                                                    T *__restrict__ out)
{
    constexpr int TL = TileL<T>::v;
    // LDS planes [TR][TL]
    __shared__ T Y[4][TR][TL];     // y1 planes (ring of four)
    __shared__ T S1[2][TR][TL];       // c1(t-2) + c1(t-1)        (V0 cross mean)
    __shared__ T S2[2][TR][TL];       // c2(t-2) + c2(t-1)
    __shared__ T Q0[2][TR][TL];       // c0(wall t-1) + c0(wall t)  (V1, V2 cross mean)
    __shared__ T C1P[2][TR][TL];      // c1(t-1)
    __shared__ T C2P[2][TR][TL];      // c2(t-1)
    __shared__ T GP[2][TR][TL];       // G(t-1)
    __shared__ T V1B[2][TR][TL];      // V1 at plane t-2
    __shared__ T V2B[2][TR][TL];      // V2 at plane t-2

    const int l = threadIdx.x % TL, r = threadIdx.x / TL;
    // The hardware deals workgroup b to XCD b % 8; tile q is numbered so
    // that consecutive tiles (which share halo cells) land on one XCD.
    int b;
    {
        const int x = blockIdx.x & 7, per = nblk >> 3, rem = nblk & 7;
        b = x * per + (x < rem ? x : rem) + (blockIdx.x >> 3);
    }
    const int tk = b % tiles_k;
    b /= tiles_k;
    const int tj = b % tiles_j;
    const int ch = b / tiles_j;
    const int k0 = tk * (TL - 2 * HALO), j0 = tj * (TR - 2 * HALO);
    const int kk = k0 - HALO + l, jj = j0 - HALO + r;
    const int i0 = ch * th, i1 = min(i0 + th, g.n0);
    const bool out_pos = r >= HALO && r < TR - HALO && l >= HALO && l < TL - HALO &&
                         jj < g.n1 && kk < g.n2;
    // the (j, k) part of this thread's addresses; planes add a uniform part
    const int jw = wrap_cell(jj, g.n1, g.bc1), kw = wrap_cell(kk, g.n2, g.bc2);
    const int64_t pl = (int64_t)g.n1 * g.n2, pl1 = (int64_t)(g.n1 + 1) * g.n2,
                  pl2 = (int64_t)g.n1 * (g.n2 + 1);
    const T *y1p = y1 + ((int64_t)jw * g.n2 + kw);
    const T *Gp = HAS_G ? G + ((int64_t)jw * g.n2 + kw) : nullptr;
    const T *c0p = c0 + ((int64_t)jw * g.n2 + kw);
    const T *c1p = c1 + ((int64_t)wrap_wall(jj, g.n1, g.bc1) * g.n2 + kw);
    const T *c2p = c2 + ((int64_t)jw * (g.n2 + 1) + wrap_wall(kk, g.n2, g.bc2));

    // own-column queues (index 0 = oldest)
    T yq[4] = {T(0), T(0), T(0), T(0)};  // y1 planes t-3..t
    T gq[3] = {T(1), T(1), T(1)};        // G planes t-2..t
    T c0q[3] = {T(0), T(0), T(0)};       // c0 walls t-2..t
    T c1q[3] = {T(0), T(0), T(0)};       // c1 planes t-2..t
    T c2q[3] = {T(0), T(0), T(0)};       // c2 planes t-2..t
    T v0q[2] = {T(0), T(0)};             // V0 walls t-2, t-1
    T v1_keep = T(0), v2_keep = T(0);    // V1, V2 at plane t-1 (to LDS next plane)

    const int t_begin = i0 - 2, t_end = i1 + 1;
    // plane t+1 is loaded while plane t is processed
    T y_nx, g_nx = T(1), c0_nx, c1_nx, c2_nx;
    auto load = [&](int t) {
        const int ic = wrap_cell(t, g.n0, g.bc0), iw = wrap_wall(t, g.n0, g.bc0);
        y_nx = y1p[ic * pl];
        if (HAS_G) g_nx = Gp[ic * pl];
        c0_nx = c0p[iw * pl];
        c1_nx = c1p[ic * pl1];
        c2_nx = c2p[ic * pl2];
    };
    load(t_begin);
    // One plane.  The LDS ring slot of plane t is its phase (t - t_begin)
    // mod 4 and the other per-plane arrays alternate between two sets, both
    // compile-time constants in each of the four unrolled copies.  With four
    // y1 slots and two sets, one barrier per plane suffices: a thread writing
    // plane t+2 has passed the barrier of plane t+1, which every thread
    // reaches only after it has finished reading plane t's arrays.
    auto plane = [&](auto phase, int t) {
        constexpr int s0 = decltype(phase)::value;
        constexpr int sm1 = (s0 + 3) % 4, sm2 = (s0 + 2) % 4, bs = s0 & 1;
        T y_new = y_nx, g_new = g_nx, c0_new = c0_nx, c1_new = c1_nx, c2_new = c2_nx;
        load(t + 1);   // wrapped: past the chunk it reads valid, unused planes
        yq[0] = yq[1]; yq[1] = yq[2]; yq[2] = yq[3]; yq[3] = y_new;
        gq[0] = gq[1]; gq[1] = gq[2]; gq[2] = g_new;
        c0q[0] = c0q[1]; c0q[1] = c0q[2]; c0q[2] = c0_new;
        c1q[0] = c1q[1]; c1q[1] = c1q[2]; c1q[2] = c1_new;
        c2q[0] = c2q[1]; c2q[1] = c2q[2]; c2q[2] = c2_new;

        // ---- write phase ----
        Y[s0][r][l] = y_new;
        S1[bs][r][l] = c1q[0] + c1q[1];
        S2[bs][r][l] = c2q[0] + c2q[1];
        Q0[bs][r][l] = c0q[1] + c0q[2];
        C1P[bs][r][l] = c1q[1];
        C2P[bs][r][l] = c2q[1];
        GP[bs][r][l] = gq[1];
        V1B[bs][r][l] = v1_keep;
        V2B[bs][r][l] = v2_keep;
        __syncthreads();

        // neighbour accessors (clamped to the tile; only halo lanes / rows
        // read past it, and their results are never used)
        const int rm1 = max(r - 1, 0), rm2 = max(r - 2, 0), rp1 = min(r + 1, TR - 1);
        const int lm1 = max(l - 1, 0), lm2 = max(l - 2, 0), lp1 = min(l + 1, TL - 1);

        // 1 / mean G at the three walls this thread owns (V0 at wall t-1,
        // V1 at wall jj and V2 at wall kk of plane t-1)
        T igw[3] = {T(1), T(1), T(1)};
        if (HAS_G) {
            T one[3] = {T(1), T(1), T(1)};
            T gb[3] = {T(0.5) * (gq[0] + gq[1]), T(0.5) * (GP[bs][rm1][l] + GP[bs][r][l]),
                       T(0.5) * (GP[bs][r][lm1] + GP[bs][r][l])};
            quotients<3>(one, gb, igw);
        }
        // ---- V0 at wall t-1 (planes t-2 | t-1), own (j, k) ----
        T v0;
        {
            T xL = yq[1], xR = yq[2];
            T ig = igw[0];
            T u = c0q[1];
            T A = fr<T, IGA>(xR - xL, xR + xL, T(2));
            T v = (fabs(u) - u * u * ig) * A;
            T cb1 = T(0.25) * (S1[bs][r][l] + S1[bs][rp1][l]);
            T cb2 = T(0.25) * (S2[bs][r][l] + S2[bs][r][lp1]);
            // o = 1 (j)
            T a1 = Y[sm1][rp1][l], b1 = Y[sm2][rp1][l], e1 = Y[sm1][rm1][l], f1 = Y[sm2][rm1][l];
            v -= T(0.5) * u * cb1 * ig * fr<T, IGA>(a1 + b1 - e1 - f1, a1 + b1 + e1 + f1, T(4));
            // o = 2 (k)
            T a2 = Y[sm1][r][lp1], b2 = Y[sm2][r][lp1], e2 = Y[sm1][r][lm1], f2 = Y[sm2][r][lm1];
            v -= T(0.5) * u * cb2 * ig * fr<T, IGA>(a2 + b2 - e2 - f2, a2 + b2 + e2 + f2, T(4));
            if (TOT) {
                T xR2 = yq[3], xL2 = yq[0];
                v += (T(3) * u * fabs(u) * ig - T(2) * u * u * u * (ig * ig) - u) * (T(1) / T(3)) *
                     fr<T, IGA>(xR2 - xR - xL + xL2, xR2 + xR + xL + xL2, T(4));
                v += (fabs(u) * cb1 * ig - T(2) * u * u * cb1 * (ig * ig)) *
                     fr<T, IGA>(a1 - b1 - e1 + f1, a1 + b1 + e1 + f1, T(4));
                v += (fabs(u) * cb2 * ig - T(2) * u * u * cb2 * (ig * ig)) *
                     fr<T, IGA>(a2 - b2 - e2 + f2, a2 + b2 + e2 + f2, T(4));
                // o1 = j, o2 = k, sides L = plane t-2, R = plane t-1
                T num = T(0), den = T(0);
                for (int sd = 0; sd < 2; sd++) {
                    int sl = sd ? sm1 : sm2;
                    T pp = Y[sl][rp1][lp1], mp_ = Y[sl][rm1][lp1], pm = Y[sl][rp1][lm1],
                      mm = Y[sl][rm1][lm1];
                    num += pp - mp_ - pm + mm;
                    den += pp + mp_ + pm + mm;
                }
                v += -(T(2) / T(3)) * u * cb1 * cb2 * (ig * ig) * fr<T, IGA>(num, den, T(8));
            }
            v0 = v;
        }
        // ---- V1 at plane t-1, wall jj (rows jj-1 | jj), own k ----
        T v1;
        {
            T xL = Y[sm1][rm1][l], xR = Y[sm1][r][l];
            T ig = igw[1];
            T u = C1P[bs][r][l];
            T A = fr<T, IGA>(xR - xL, xR + xL, T(2));
            T v = (fabs(u) - u * u * ig) * A;
            T cb0 = T(0.25) * (Q0[bs][rm1][l] + Q0[bs][r][l]);
            T cb2 = T(0.25) * ((C2P[bs][rm1][l] + C2P[bs][rm1][lp1]) + (C2P[bs][r][l] + C2P[bs][r][lp1]));
            // o = 0 (i): R+e0 = plane t at r, L+e0 = plane t at r-1, minus plane t-2
            T a0 = Y[s0][r][l], b0 = Y[s0][rm1][l], e0 = Y[sm2][r][l], f0 = Y[sm2][rm1][l];
            v -= T(0.5) * u * cb0 * ig * fr<T, IGA>(a0 + b0 - e0 - f0, a0 + b0 + e0 + f0, T(4));
            // o = 2 (k)
            T a2 = Y[sm1][r][lp1], b2 = Y[sm1][rm1][lp1], e2 = Y[sm1][r][lm1],
              f2 = Y[sm1][rm1][lm1];
            v -= T(0.5) * u * cb2 * ig * fr<T, IGA>(a2 + b2 - e2 - f2, a2 + b2 + e2 + f2, T(4));
            if (TOT) {
                T xR2 = Y[sm1][rp1][l], xL2 = Y[sm1][rm2][l];
                v += (T(3) * u * fabs(u) * ig - T(2) * u * u * u * (ig * ig) - u) * (T(1) / T(3)) *
                     fr<T, IGA>(xR2 - xR - xL + xL2, xR2 + xR + xL + xL2, T(4));
                v += (fabs(u) * cb0 * ig - T(2) * u * u * cb0 * (ig * ig)) *
                     fr<T, IGA>(a0 - b0 - e0 + f0, a0 + b0 + e0 + f0, T(4));
                v += (fabs(u) * cb2 * ig - T(2) * u * u * cb2 * (ig * ig)) *
                     fr<T, IGA>(a2 - b2 - e2 + f2, a2 + b2 + e2 + f2, T(4));
                // o1 = i, o2 = k, sides L = row r-1, R = row r
                T num = T(0), den = T(0);
                for (int sd = 0; sd < 2; sd++) {
                    int rr = sd ? r : rm1;
                    T pp = Y[s0][rr][lp1], mp_ = Y[sm2][rr][lp1], pm = Y[s0][rr][lm1],
                      mm = Y[sm2][rr][lm1];
                    num += pp - mp_ - pm + mm;
                    den += pp + mp_ + pm + mm;
                }
                v += -(T(2) / T(3)) * u * cb0 * cb2 * (ig * ig) * fr<T, IGA>(num, den, T(8));
            }
            v1 = v;
        }
        // ---- V2 at plane t-1, wall kk (lanes kk-1 | kk), own j ----
        T v2;
        {
            T xL = Y[sm1][r][lm1], xR = Y[sm1][r][l];
            T ig = igw[2];
            T u = C2P[bs][r][l];
            T A = fr<T, IGA>(xR - xL, xR + xL, T(2));
            T v = (fabs(u) - u * u * ig) * A;
            T cb0 = T(0.25) * (Q0[bs][r][lm1] + Q0[bs][r][l]);
            T cb1 = T(0.25) * ((C1P[bs][r][lm1] + C1P[bs][rp1][lm1]) + (C1P[bs][r][l] + C1P[bs][rp1][l]));
            // o = 0 (i)
            T a0 = Y[s0][r][l], b0 = Y[s0][r][lm1], e0 = Y[sm2][r][l], f0 = Y[sm2][r][lm1];
            v -= T(0.5) * u * cb0 * ig * fr<T, IGA>(a0 + b0 - e0 - f0, a0 + b0 + e0 + f0, T(4));
            // o = 1 (j)
            T a1 = Y[sm1][rp1][l], b1 = Y[sm1][rp1][lm1], e1 = Y[sm1][rm1][l],
              f1 = Y[sm1][rm1][lm1];
            v -= T(0.5) * u * cb1 * ig * fr<T, IGA>(a1 + b1 - e1 - f1, a1 + b1 + e1 + f1, T(4));
            if (TOT) {
                T xR2 = Y[sm1][r][lp1], xL2 = Y[sm1][r][lm2];
                v += (T(3) * u * fabs(u) * ig - T(2) * u * u * u * (ig * ig) - u) * (T(1) / T(3)) *
                     fr<T, IGA>(xR2 - xR - xL + xL2, xR2 + xR + xL + xL2, T(4));
                v += (fabs(u) * cb0 * ig - T(2) * u * u * cb0 * (ig * ig)) *
                     fr<T, IGA>(a0 - b0 - e0 + f0, a0 + b0 + e0 + f0, T(4));
                v += (fabs(u) * cb1 * ig - T(2) * u * u * cb1 * (ig * ig)) *
                     fr<T, IGA>(a1 - b1 - e1 + f1, a1 + b1 + e1 + f1, T(4));
                // o1 = i, o2 = j, sides L = lane l-1, R = lane l
                T num = T(0), den = T(0);
                for (int sd = 0; sd < 2; sd++) {
                    int ll = sd ? l : lm1;
                    T pp = Y[s0][rp1][ll], mp_ = Y[sm2][rp1][ll], pm = Y[s0][rm1][ll],
                      mm = Y[sm2][rm1][ll];
                    num += pp - mp_ - pm + mm;
                    den += pp + mp_ + pm + mm;
                }
                v += -(T(2) / T(3)) * u * cb0 * cb1 * (ig * ig) * fr<T, IGA>(num, den, T(8));
            }
            v2 = v;
        }

        // ---- corrective pass at plane t-2 ----
        v0q[0] = v0q[1];
        v0q[1] = v0;
        const int p = t - 2;
        if (p >= i0 && p < i1 && out_pos) {
            T x = yq[1];
            T V0lo = v0q[0], V0hi = v0q[1];
            T V1lo = V1B[bs][r][l], V1hi = V1B[bs][rp1][l];
            T V2lo = V2B[bs][r][l], V2hi = V2B[bs][r][lp1];
            T f0lo, f0hi, f1lo, f1hi, f2lo, f2hi;
            if (IGA) {
                f0lo = V0lo; f0hi = V0hi; f1lo = V1lo; f1hi = V1hi; f2lo = V2lo; f2hi = V2hi;
            } else {
                f0lo = pos(V0lo) * yq[0] + neg(V0lo) * x;
                f0hi = pos(V0hi) * x + neg(V0hi) * yq[2];
                f1lo = pos(V1lo) * Y[sm2][rm1][l] + neg(V1lo) * x;
                f1hi = pos(V1hi) * x + neg(V1hi) * Y[sm2][rp1][l];
                f2lo = pos(V2lo) * Y[sm2][r][lm1] + neg(V2lo) * x;
                f2hi = pos(V2hi) * x + neg(V2hi) * Y[sm2][r][lp1];
            }
            T res;
            if (kahan) {
                T dv[3] = {f0hi - f0lo, f1hi - f1lo, f2hi - f2lo};
                if (HAS_G) {
                    T gg[3] = {gq[0], gq[0], gq[0]}, qq[3];
                    quotients<3>(dv, gg, qq);
                    dv[0] = qq[0];
                    dv[1] = qq[1];
                    dv[2] = qq[2];
                }
                T ks = x, kc = T(0);
#pragma unroll
                for (int d = 0; d < 3; d++) kahan_add(ks, kc, -dv[d]);
                res = ks;
            } else {
                T acc = T(0);
                acc += f0hi - f0lo;
                acc += f1hi - f1lo;
                acc += f2hi - f2lo;
                if (HAS_G) {
                    T nn[1] = {acc}, dd[1] = {gq[0]}, qq[1];
                    quotients<1>(nn, dd, qq);
                    acc = qq[0];
                }
                res = x - acc;
            }
            out[((int64_t)p * g.n1 + jj) * g.n2 + kk] = res;
        }
        v1_keep = v1;
        v2_keep = v2;
    };
    // whole blocks of four planes; iterations past t_end store nothing
    for (int t = t_begin; t <= t_end; t += 4) {
        plane(std::integral_constant<int, 0>{}, t);
        plane(std::integral_constant<int, 1>{}, t + 1);
        plane(std::integral_constant<int, 2>{}, t + 2);
        plane(std::integral_constant<int, 3>{}, t + 3);
    }
}

}  // namespace

bool fused3d_supported(int nd, int n_iters, unsigned opts, const int64_t n[3], const int bc[3])
{
    if (nd != 3 || !(n_iters == 1 || n_iters == 2) || (opts & (OPT_FCT | OPT_ABS | OPT_DFL))) return false;
    if (n[0] >= 65536 || n[1] >= (1 << 30) || n[2] >= (1 << 30)) return false;
    // halo coordinates (and the planes read past a chunk) must stay within
    // one period of a periodic dimension
    if (bc[0] == BC_PERIODIC && n[0] < 6) return false;
    if (bc[1] == BC_PERIODIC && n[1] < TR) return false;
    if (bc[2] == BC_PERIODIC && n[2] < 64) return false;
    return true;
}

template <typename T>
hipError_t fused3d_step(const Geom &geom, int n_iters, unsigned opts, const T *psi_n, T *psi_out,
                        const T *c0, const T *c1, const T *c2, const T *G, T *y1buf, int tile_planes,
                        hipStream_t s)
{
    G3 g{(int)geom.n[0], (int)geom.n[1], (int)geom.n[2], geom.bc[0], geom.bc[1], geom.bc[2]};
    const int dk = (int)cdiv(g.n2, 64), dj = (int)cdiv(g.n1, 4);
    const int64_t dblk = (int64_t)dk * dj * cdiv(g.n0, DONOR_PLANES);
    if (dblk > INT32_MAX) return hipErrorInvalidValue;
    T *y1 = (n_iters == 1) ? psi_out : y1buf;
    const int kahan = (opts & OPT_KAHAN) ? 1 : 0;
    if (G)
        k_donor3d<T, true><<<(unsigned)dblk, 256, 0, s>>>(g, kahan, dk, dj, (int)dblk, psi_n, c0,
                                                          c1, c2, G, y1);
    else
        k_donor3d<T, false><<<(unsigned)dblk, 256, 0, s>>>(g, kahan, dk, dj, (int)dblk, psi_n, c0,
                                                           c1, c2, G, y1);
    if (n_iters == 1) return hipGetLastError();
    constexpr int TL = TileL<T>::v;
    int tiles_k = (g.n2 + TL - 2 * HALO - 1) / (TL - 2 * HALO);
    int tiles_j = (g.n1 + TR - 2 * HALO - 1) / (TR - 2 * HALO);
    int th = tile_planes > 0 ? tile_planes : 48;
    if (th > g.n0) th = g.n0;
    int chunks = (g.n0 + th - 1) / th;
    unsigned blocks = (unsigned)tiles_k * tiles_j * chunks;
    const bool iga = opts & OPT_IGA, tot = opts & OPT_TOT;
#define MP_CORR(HG, IG, TO) \
    k_corr3d<T, HG, IG, TO><<<blocks, TR * TL, 0, s>>>(g, th, tiles_k, tiles_j, (int)blocks, \
                                                      kahan, y1, \
                                                      c0, c1, c2, G, psi_out)
    if (G) {
        if (iga) { if (tot) MP_CORR(true, true, true); else MP_CORR(true, true, false); }
        else { if (tot) MP_CORR(true, false, true); else MP_CORR(true, false, false); }
    } else {
        if (iga) { if (tot) MP_CORR(false, true, true); else MP_CORR(false, true, false); }
        else { if (tot) MP_CORR(false, false, true); else MP_CORR(false, false, false); }
    }
#undef MP_CORR
    return hipGetLastError();
}

template hipError_t fused3d_step<float>(const Geom &, int, unsigned, const float *, float *,
                                        const float *, const float *, const float *,
                                        const float *, float *, int, hipStream_t);
template hipError_t fused3d_step<double>(const Geom &, int, unsigned, const double *, double *,
                                         const double *, const double *, const double *,
                                         const double *, double *, int, hipStream_t);

}  // namespace mp
