// staged.hip -- the MPDATA step as one kernel launch per stage.
//
// Every stage is a plain gather: one thread per output cell or wall, every
// input read through the boundary map.  Intermediate fields (pass results,
// pseudo-velocities, limiter coefficients) round-trip through the caller's
// workspace.  This is the general path (1-3 D, every option, both boundary
// types, FP32/FP64) and the cross-check for the fused kernels.
#include "common.hpp"
#include "dual.hpp"
#include "kernels.hpp"

#include <type_traits>

namespace mp {
namespace {

struct Idx3 {
    int v[3];
};

__device__ inline Idx3 unflat(int64_t t, const int64_t e[3])
{
    Idx3 p;
    unflat3(t, e, p.v);
    return p;
}

__device__ inline Idx3 shifted(Idx3 p, int d, int s)
{
    p.v[d] += s;
    return p;
}

template <typename T>
__device__ inline T cell(const Geom &g, const T *a, const Idx3 &p)
{
    int i = wrap_cell(p.v[0], (int)g.n[0], g.bc[0]);
    int j = wrap_cell(p.v[1], (int)g.n[1], g.bc[1]);
    int k = wrap_cell(p.v[2], (int)g.n[2], g.bc[2]);
    return a[((int64_t)i * g.n[1] + j) * g.n[2] + k];
}

template <typename T>
__device__ inline T gcell(const Geom &g, const T *G, const Idx3 &p)
{
    return G ? cell(g, G, p) : T(1);
}

// wall value of the dimension-d advector component at p (p.v[d] = wall)
template <typename T>
__device__ inline T wall(const Geom &g, int d, const T *a, const Idx3 &p)
{
    int64_t e[3] = {g.n[0], g.n[1], g.n[2]};
    e[d] += 1;
    int q[3];
    for (int t = 0; t < 3; t++)
        q[t] = (t == d) ? wrap_wall(p.v[t], (int)g.n[t], g.bc[t])
                        : wrap_cell(p.v[t], (int)g.n[t], g.bc[t]);
    return a[((int64_t)q[0] * e[1] + q[1]) * e[2] + q[2]];
}

// Boundary-mapped coordinates of the positions p + o, o = -2..2, along each
// of the first ND dimensions, as cells and as walls, formed once per thread.
// The stencils read at constant offsets from p (their loops unroll), so a
// read costs its index arithmetic only, not a boundary map per dimension.
template <int ND> struct Near {
    Idx3 p;
    int c[3][5], w[3][5];
    __device__ __forceinline__ Near(const Geom &g, const Idx3 &p_) : p(p_)
    {
#pragma unroll
        for (int t = 0; t < 3; t++)
#pragma unroll
            for (int o = 0; o < 5; o++) {
                c[t][o] = t < ND ? wrap_cell(p.v[t] + o - 2, (int)g.n[t], g.bc[t]) : 0;
                w[t][o] = t < ND ? wrap_wall(p.v[t] + o - 2, (int)g.n[t], g.bc[t]) : 0;
            }
    }
    __device__ __forceinline__ int off(const Idx3 &q, int t) const { return q.v[t] - p.v[t] + 2; }
    // cell array at q
    template <typename T> __device__ __forceinline__ T cell(const Geom &g, const T *a, const Idx3 &q) const
    {
        const int i = c[0][off(q, 0)], j = c[1][off(q, 1)], k = c[2][off(q, 2)];
        return a[((int64_t)i * g.n[1] + j) * g.n[2] + k];
    }
    template <typename T> __device__ __forceinline__ T gcell(const Geom &g, const T *G, const Idx3 &q) const
    {
        return G ? cell(g, G, q) : T(1);
    }
    // dimension-d wall array at q (q.v[d] a wall coordinate)
    template <typename T>
    __device__ __forceinline__ T wall(const Geom &g, int d, const T *a, const Idx3 &q) const
    {
        const int i = d == 0 ? w[0][off(q, 0)] : c[0][off(q, 0)];
        const int j = d == 1 ? w[1][off(q, 1)] : c[1][off(q, 1)];
        const int k = d == 2 ? w[2][off(q, 2)] : c[2][off(q, 2)];
        const int64_t e1 = g.n[1] + (d == 1 ? 1 : 0), e2 = g.n[2] + (d == 2 ? 1 : 0);
        return a[((int64_t)i * e1 + j) * e2 + k];
    }
};

template <typename T>
__device__ inline T frac(bool iga, T num, T den, T m)
{
    if (iga) return num / m;
    return den == T(0) ? T(0) : num / den;
}

// donor-cell pass (eqs. upstream, F).  mode bit 0: the wall flux is the
// advector itself (infinite-gauge corrective pass); bit 1: Kahan-compensated
// update (terms -(F(hi) - F(lo)) / G, dimensions in increasing order)
template <typename T, int ND>
__global__ void __launch_bounds__(256) k_donor(Geom g, const T *__restrict__ x, const T *c0, const T *c1,
                        const T *c2, const T *G, int mode, T *__restrict__ out)
{
    int64_t N = g.n[0] * g.n[1] * g.n[2];
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N) return;
    const bool flux_is_vel = mode & 1, kahan = mode & 2;
    const Idx3 p = unflat(t, g.n);
    const Near<ND> nr(g, p);
    const T *c[3] = {c0, c1, c2};
    T acc = T(0);
    T ks = x[t], kc = T(0);
#pragma unroll
    for (int d = 0; d < ND; d++) {
        T fl[2];
#pragma unroll
        for (int s = 0; s < 2; s++) {
            Idx3 w = shifted(p, d, s);
            T u = nr.wall(g, d, c[d], w);
            if (flux_is_vel)
                fl[s] = u;
            else
                fl[s] = upwind(u, nr.cell(g, x, shifted(w, d, -1)), nr.cell(g, x, w));
        }
        acc += fl[1] - fl[0];
        if (kahan) {
            T term = fl[1] - fl[0];
            if (G) term = term / G[t];
            kahan_add(ks, kc, -term);
        }
    }
    if (kahan) {
        out[t] = ks;
        return;
    }
    T r = G ? acc / G[t] : acc;
    out[t] = x[t] - r;
}

// antidiffusive pseudo-velocity at every dimension-d wall (eq. adf_vel, its
// cross terms and the third-order terms)
template <typename T, int ND, int WD>
__global__ void __launch_bounds__(256) k_pseudo(Geom g, unsigned opts, const T *__restrict__ x, const T *c0,
                         const T *c1, const T *c2, const T *G, T *__restrict__ V)
{
    constexpr int d = WD;   // wall dimension (compile time: no dynamic indexing)
    int64_t e[3] = {g.n[0], g.n[1], g.n[2]};
    e[d] += 1;
    int64_t M = e[0] * e[1] * e[2];
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= M) return;
    const bool iga = opts & OPT_IGA, tot = opts & OPT_TOT, absf = opts & OPT_ABS;
    // psi value entering a psi-fraction: |psi| under the abs option
    const Idx3 p = unflat(t, e);
    const Near<ND> nr(g, p);
    auto xv = [&](const Idx3 &q) -> T {
        T v = nr.cell(g, x, q);
        return absf ? fabs(v) : v;
    };
    const T *c[3] = {c0, c1, c2};
    Idx3 L = shifted(p, d, -1), R = p;
    T u = nr.wall(g, d, c[d], p);
    T ig = T(1);                                                   // 1 / mean G
    if (G) ig = T(1) / (T(0.5) * (nr.cell(g, G, L) + nr.cell(g, G, R)));
    T xL = xv(L), xR = xv(R);
    T V_ = (fabs(u) - u * u * ig) * frac(iga, xR - xL, xR + xL, T(2));

    T cb[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int o = 0; o < ND; o++) {
        if (o == d) continue;
        cb[o] = T(0.25) * (nr.wall(g, o, c[o], L) + nr.wall(g, o, c[o], shifted(L, o, 1)) +
                           nr.wall(g, o, c[o], R) + nr.wall(g, o, c[o], shifted(R, o, 1)));
        T a = xv(shifted(R, o, 1)), b = xv(shifted(L, o, 1));
        T e_ = xv(shifted(R, o, -1)), f = xv(shifted(L, o, -1));
        V_ -= T(0.5) * u * cb[o] * ig * frac(iga, a + b - e_ - f, a + b + e_ + f, T(4));
    }
    if (opts & OPT_DFL) {
        // divergent-flow term: -c / (2 Gb) times the mean of the two cells'
        // advector divergences sum_o (c_o(hi) - c_o(lo))
        T dv = T(0);
#pragma unroll
        for (int o = 0; o < ND; o++)
            dv += (nr.wall(g, o, c[o], shifted(L, o, 1)) - nr.wall(g, o, c[o], L)) +
                  (nr.wall(g, o, c[o], shifted(R, o, 1)) - nr.wall(g, o, c[o], R));
        // under iga the pseudo-velocity is a unit-field flux, so this
        // psi-free term carries the wall mean of psi
        if (iga) dv *= T(0.5) * (xL + xR);
        V_ -= T(0.25) * u * ig * dv;
    }
    if (tot) {
        T xR2 = xv(shifted(R, d, 1)), xL2 = xv(shifted(L, d, -1));
        T D = frac(iga, xR2 - xR - xL + xL2, xR2 + xR + xL + xL2, T(4));
        V_ += (T(3) * u * fabs(u) * ig - T(2) * u * u * u * (ig * ig) - u) * (T(1) / T(3)) * D;
#pragma unroll
        for (int o = 0; o < ND; o++) {
            if (o == d) continue;
            T a = xv(shifted(R, o, 1)), b = xv(shifted(L, o, 1));
            T e_ = xv(shifted(R, o, -1)), f = xv(shifted(L, o, -1));
            T E = frac(iga, a - b - e_ + f, a + b + e_ + f, T(4));
            V_ += (fabs(u) * cb[o] * ig - T(2) * u * u * cb[o] * (ig * ig)) * E;
        }
        if (ND == 3) {
            int o1 = (d == 0) ? 1 : 0;
            int o2 = (d == 2) ? 1 : 2;
            T num = T(0), den = T(0);
#pragma unroll
            for (int s = 0; s < 2; s++) {
                Idx3 S = s ? R : L;
                T vpp = xv(shifted(shifted(S, o1, 1), o2, 1));
                T vmp = xv(shifted(shifted(S, o1, -1), o2, 1));
                T vpm = xv(shifted(shifted(S, o1, 1), o2, -1));
                T vmm = xv(shifted(shifted(S, o1, -1), o2, -1));
                num += vpp - vmp - vpm + vmm;
                den += vpp + vmp + vpm + vmm;
            }
            V_ += -(T(2) / T(3)) * u * cb[o1] * cb[o2] * (ig * ig) * frac(iga, num, den, T(8));
        }
    }
    V[t] = V_;
}

// limiter coefficients per cell (Sect. 3.1.4)
template <typename T, int ND>
__global__ void __launch_bounds__(256) k_fct_beta(Geom g, unsigned opts, const T *__restrict__ psi_n,
                           const T *__restrict__ x, const T *V0, const T *V1, const T *V2,
                           const T *G, T *__restrict__ bup, T *__restrict__ bdn)
{
    int64_t N = g.n[0] * g.n[1] * g.n[2];
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N) return;
    const bool iga = opts & OPT_IGA;
    const T *V[3] = {V0, V1, V2};
    const Idx3 p = unflat(t, g.n);
    const Near<ND> nr(g, p);
    T xi = x[t];
    T mx = psi_n[t], mn = mx;
    mx = fmax(mx, xi);
    mn = fmin(mn, xi);
#pragma unroll
    for (int d = 0; d < ND; d++)
#pragma unroll
        for (int s = -1; s <= 1; s += 2) {
            Idx3 q = shifted(p, d, s);
            T a = nr.cell(g, psi_n, q), b = nr.cell(g, x, q);
            mx = fmax(fmax(mx, a), b);
            mn = fmin(fmin(mn, a), b);
        }
    T fin = T(0), fout = T(0);
#pragma unroll
    for (int d = 0; d < ND; d++) {
        T vlo = nr.wall(g, d, V[d], p), vhi = nr.wall(g, d, V[d], shifted(p, d, 1));
        T wm = iga ? T(1) : nr.cell(g, x, shifted(p, d, -1));
        T wp = iga ? T(1) : nr.cell(g, x, shifted(p, d, 1));
        T wi = iga ? T(1) : xi;
        fin += pos(vlo) * wm - neg(vhi) * wp;
        fout += pos(vhi) * wi - neg(vlo) * wi;
    }
    T Gi = G ? G[t] : T(1);
    bup[t] = fin > T(0) ? Gi * (mx - xi) / fin : T(1);
    bdn[t] = fout > T(0) ? Gi * (xi - mn) / fout : T(1);
}

// 3-D limiter coefficients, the arithmetic of k_fct_beta term by term, with
// one thread per (j, k) column marching along i over BETA_PLANES planes:
// psi^n and x of the planes i-1, i, i+1 and the dimension-0 walls stay in
// registers (read once per plane instead of once per neighbour), the
// in-plane neighbours come through L1/L2, and no flat index is divided
// back into coordinates.  Blocks of 64 (k) x 4 (j) columns, numbered so
// that each XCD runs a contiguous range of tiles (see fused3d.hip).
constexpr int BETA_PLANES = 16;

template <typename T>
__global__ void __launch_bounds__(256)
k_fct_beta3d(Geom g, unsigned opts, int tiles_k, int tiles_j, int nblk,
             const T *__restrict__ psi_n, const T *__restrict__ x, const T *__restrict__ V0,
             const T *__restrict__ V1, const T *__restrict__ V2, const T *__restrict__ G,
             T *__restrict__ bup, T *__restrict__ bdn)
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
    const int n0 = (int)g.n[0], n1 = (int)g.n[1], n2 = (int)g.n[2];
    const int k = tk * 64 + (threadIdx.x & 63);
    const int j = tj * 4 + (threadIdx.x >> 6);
    const int i0 = ch * BETA_PLANES;
    const int i1 = min(i0 + BETA_PLANES, n0);
    if (k >= n2 || j >= n1) return;
    const bool iga = opts & OPT_IGA;
    const int64_t pl = (int64_t)n1 * n2, pl1 = (int64_t)(n1 + 1) * n2,
                  pl2 = (int64_t)n1 * (n2 + 1);
    // in-plane offsets of the column and its neighbours (boundary-mapped)
    const int64_t o = (int64_t)j * n2 + k;
    const int64_t ojm = (int64_t)wrap_cell(j - 1, n1, g.bc[1]) * n2 + k;
    const int64_t ojp = (int64_t)wrap_cell(j + 1, n1, g.bc[1]) * n2 + k;
    const int64_t okm = (int64_t)j * n2 + wrap_cell(k - 1, n2, g.bc[2]);
    const int64_t okp = (int64_t)j * n2 + wrap_cell(k + 1, n2, g.bc[2]);
    const int64_t w1lo = (int64_t)j * n2 + k;
    const int64_t w1hi = (int64_t)wrap_wall(j + 1, n1, g.bc[1]) * n2 + k;
    const int64_t w2lo = (int64_t)j * (n2 + 1) + k;
    const int64_t w2hi = (int64_t)j * (n2 + 1) + wrap_wall(k + 1, n2, g.bc[2]);

    const int64_t im = (int64_t)wrap_cell(i0 - 1, n0, g.bc[0]) * pl;
    T pm = psi_n[im + o], xm = x[im + o];
    T pc = psi_n[i0 * pl + o], xc = x[i0 * pl + o];
    T v0lo = V0[(int64_t)wrap_wall(i0, n0, g.bc[0]) * pl + o];
    for (int i = i0; i < i1; i++) {
        const int64_t ic = (int64_t)i * pl;
        const int64_t ip = (int64_t)wrap_cell(i + 1, n0, g.bc[0]) * pl;
        const T pp = psi_n[ip + o], xp = x[ip + o];
        const T v0hi = V0[(int64_t)wrap_wall(i + 1, n0, g.bc[0]) * pl + o];
        const T xjm = x[ic + ojm], xjp = x[ic + ojp], xkm = x[ic + okm], xkp = x[ic + okp];
        const T xi = xc;
        T mx = pc, mn = mx;
        mx = fmax(mx, xi);
        mn = fmin(mn, xi);
        // face neighbours in the order -e0, +e0, -e1, +e1, -e2, +e2
        const T na[6] = {pm, pp, psi_n[ic + ojm], psi_n[ic + ojp], psi_n[ic + okm],
                         psi_n[ic + okp]};
        const T nb[6] = {xm, xp, xjm, xjp, xkm, xkp};
#pragma unroll
        for (int q = 0; q < 6; q++) {
            mx = fmax(fmax(mx, na[q]), nb[q]);
            mn = fmin(fmin(mn, na[q]), nb[q]);
        }
        const T vlo[3] = {v0lo, V1[(int64_t)i * pl1 + w1lo], V2[(int64_t)i * pl2 + w2lo]};
        const T vhi[3] = {v0hi, V1[(int64_t)i * pl1 + w1hi], V2[(int64_t)i * pl2 + w2hi]};
        T fin = T(0), fout = T(0);
#pragma unroll
        for (int d = 0; d < 3; d++) {
            const T wm = iga ? T(1) : nb[2 * d], wp = iga ? T(1) : nb[2 * d + 1];
            const T wi = iga ? T(1) : xi;
            fin += pos(vlo[d]) * wm - neg(vhi[d]) * wp;
            fout += pos(vhi[d]) * wi - neg(vlo[d]) * wi;
        }
        const T Gi = G ? G[ic + o] : T(1);
        bup[ic + o] = fin > T(0) ? Gi * (mx - xi) / fin : T(1);
        bdn[ic + o] = fout > T(0) ? Gi * (xi - mn) / fout : T(1);
        pm = pc;
        pc = pp;
        xm = xc;
        xc = xp;
        v0lo = v0hi;
    }
}

// limited pseudo-velocity at every dimension-d wall
template <typename T, int ND, int WD>
__global__ void __launch_bounds__(256) k_fct_limit(Geom g, const T *__restrict__ V, const T *__restrict__ bup,
                            const T *__restrict__ bdn, T *__restrict__ W)
{
    constexpr int d = WD;   // wall dimension (compile time)
    int64_t e[3] = {g.n[0], g.n[1], g.n[2]};
    e[d] += 1;
    int64_t M = e[0] * e[1] * e[2];
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= M) return;
    const Idx3 p = unflat(t, e);
    const Near<ND> nr(g, p);
    Idx3 L = shifted(p, d, -1), R = p;
    T v = V[t];
    T up = fmin(fmin(T(1), nr.cell(g, bdn, L)), nr.cell(g, bup, R));
    T dn = fmin(fmin(T(1), nr.cell(g, bup, L)), nr.cell(g, bdn, R));
    W[t] = pos(v) * up + neg(v) * dn;
}

// limited velocities at the cell's walls and the corrective donor-cell
// update in one kernel (one thread per cell): the arithmetic of k_fct_limit
// followed by k_donor, term by term, without the limited velocities going
// through memory -- unless a following pass needs them as its advector:
// then W0..W2 (non-NULL) receive each cell's low walls and, along an open
// dimension, the far edge wall.  mode bit 0: the flux is the limited
// velocity itself (infinite gauge); bit 1: Kahan-compensated update.
template <typename T, int ND>
__global__ void __launch_bounds__(256)
k_limcorr(Geom g, const T *__restrict__ x, const T *V0, const T *V1, const T *V2,
          const T *__restrict__ bup, const T *__restrict__ bdn, const T *G, int mode,
          T *__restrict__ out, T *W0, T *W1, T *W2)
{
    const int64_t N = g.n[0] * g.n[1] * g.n[2];
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N) return;
    const bool flux_is_vel = mode & 1, kahan = mode & 2;
    const Idx3 p = unflat(t, g.n);
    const Near<ND> nr(g, p);
    const T *V[3] = {V0, V1, V2};
    T *Wo[3] = {W0, W1, W2};
    T acc = T(0);
    T ks = x[t], kc = T(0);
#pragma unroll
    for (int d = 0; d < ND; d++) {
        T fl[2];
#pragma unroll
        for (int s = 0; s < 2; s++) {
            const Idx3 w = shifted(p, d, s);
            const Idx3 L = shifted(w, d, -1), R = w;
            const T v = nr.wall(g, d, V[d], w);
            const T up = fmin(fmin(T(1), nr.cell(g, bdn, L)), nr.cell(g, bup, R));
            const T dn = fmin(fmin(T(1), nr.cell(g, bup, L)), nr.cell(g, bdn, R));
            const T u = pos(v) * up + neg(v) * dn;
            if (Wo[d] && (s == 0 || (g.bc[d] == BC_OPEN && p.v[d] == (int)g.n[d] - 1))) {
                int64_t e[3] = {g.n[0], g.n[1], g.n[2]};
                e[d] += 1;
                Wo[d][((int64_t)w.v[0] * e[1] + w.v[1]) * e[2] + w.v[2]] = u;
            }
            fl[s] = flux_is_vel ? u : upwind(u, nr.cell(g, x, L), nr.cell(g, x, R));
        }
        acc += fl[1] - fl[0];
        if (kahan) {
            T term = fl[1] - fl[0];
            if (G) term = term / G[t];
            kahan_add(ks, kc, -term);
        }
    }
    if (kahan) {
        out[t] = ks;
        return;
    }
    T r = G ? acc / G[t] : acc;
    out[t] = x[t] - r;
}

template <typename T>
int64_t wall_count(const Geom &g, int d)
{
    int64_t e[3] = {g.n[0], g.n[1], g.n[2]};
    e[d] += 1;
    return e[0] * e[1] * e[2];
}

}  // namespace

// ---- single-stage launchers (used by the adjoint's forward recompute) ----
template <typename T>
hipError_t launch_donor(const Geom &g, const T *x, const T *const c[3], const T *G,
                        int mode, T *out, hipStream_t s)
{
    int64_t N = g.n[0] * g.n[1] * g.n[2];
    with_nd(g.nd, [&](auto ND) {
        k_donor<T, decltype(ND)::value><<<(unsigned)cdiv(N, 256), 256, 0, s>>>(
            g, x, c[0], c[1], c[2], G, mode, out);
    });
    return hipGetLastError();
}

// Run f with the dimension count as a compile-time constant.
template <typename F> void with_nd(int nd, F f)
{
    if (nd == 1)
        f(std::integral_constant<int, 1>{});
    else if (nd == 2)
        f(std::integral_constant<int, 2>{});
    else
        f(std::integral_constant<int, 3>{});
}

// ... and with a wall dimension d < nd as a second one.
template <typename F> void with_nd_d(int nd, int d, F f)
{
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I3c = std::integral_constant<int, 3>;
    using D0 = std::integral_constant<int, 0>;
    using D1 = std::integral_constant<int, 1>;
    using D2 = std::integral_constant<int, 2>;
    if (nd == 1)
        f(I1{}, D0{});
    else if (nd == 2) {
        if (d == 0) f(I2{}, D0{}); else f(I2{}, D1{});
    } else {
        if (d == 0) f(I3c{}, D0{}); else if (d == 1) f(I3c{}, D1{}); else f(I3c{}, D2{});
    }
}

// k_pseudo for the runtime (n_dims, d): the dimension count and the wall
// dimension are template parameters so every stencil index is static
template <typename T>
void pseudo_dispatch(const Geom &g, int d, unsigned wb, unsigned tb, hipStream_t s, unsigned opts,
                     const T *x, const T *c0, const T *c1, const T *c2, const T *G, T *V)
{
#define MP_P(ND, D) k_pseudo<T, ND, D><<<wb, tb, 0, s>>>(g, opts, x, c0, c1, c2, G, V)
    if (g.nd == 1) MP_P(1, 0);
    else if (g.nd == 2) { if (d == 0) MP_P(2, 0); else MP_P(2, 1); }
    else { if (d == 0) MP_P(3, 0); else if (d == 1) MP_P(3, 1); else MP_P(3, 2); }
#undef MP_P
}

template <typename T>
hipError_t launch_pseudo(const Geom &g, unsigned opts, const T *x, const T *const c[3],
                         const T *G, T *const V[3], hipStream_t s)
{
    for (int d = 0; d < g.nd; d++) {
        unsigned wb = (unsigned)cdiv(wall_count<T>(g, d), 256);
        pseudo_dispatch<T>(g, d, wb, 256, s, opts, x, c[0], c[1], c[2], G, V[d]);
    }
    return hipGetLastError();
}

template <typename T>
void fct_beta_launch(const Geom &g, unsigned opts, const T *psi_n, const T *x,
                     const T *const V[3], const T *G, T *bup, T *bdn, hipStream_t s)
{
    const int64_t tk = cdiv(g.n[2], 64), tj = cdiv(g.n[1], 4);
    const int64_t nb = tk * tj * cdiv(g.n[0], BETA_PLANES);
    if (g.nd == 3 && nb <= INT32_MAX) {
        k_fct_beta3d<T><<<(unsigned)nb, 256, 0, s>>>(g, opts, (int)tk, (int)tj, (int)nb, psi_n,
                                                       x, V[0], V[1], V[2], G, bup, bdn);
        return;
    }
    const int64_t N = g.n[0] * g.n[1] * g.n[2];
    with_nd(g.nd, [&](auto ND) {
        k_fct_beta<T, decltype(ND)::value><<<(unsigned)cdiv(N, 256), 256, 0, s>>>(
            g, opts, psi_n, x, V[0], V[1], V[2], G, bup, bdn);
    });
}

template <typename T>
hipError_t launch_fct(const Geom &g, unsigned opts, const T *psi_n, const T *x,
                      const T *const V[3], const T *G, T *bup, T *bdn, T *const W[3],
                      hipStream_t s)
{
    fct_beta_launch<T>(g, opts, psi_n, x, V, G, bup, bdn, s);
    for (int d = 0; d < g.nd; d++) {
        unsigned wb = (unsigned)cdiv(wall_count<T>(g, d), 256);
        with_nd_d(g.nd, d, [&](auto ND, auto WD) {
            k_fct_limit<T, decltype(ND)::value, decltype(WD)::value><<<wb, 256, 0, s>>>(
                g, V[d], bup, bdn, W[d]);
        });
    }
    return hipGetLastError();
}

template <typename T>
hipError_t limcorr_launch(const Geom &g, unsigned opts, const T *x, const T *const V[3],
                          const T *G, const T *bup, const T *bdn, T *y, T *const W[3],
                          hipStream_t s)
{
    const int64_t N = g.n[0] * g.n[1] * g.n[2];
    const unsigned cb = (unsigned)cdiv(N, 256);
    const int mode = ((opts & OPT_IGA) ? 1 : 0) | ((opts & OPT_KAHAN) ? 2 : 0);
    with_nd(g.nd, [&](auto ND) {
        constexpr int nd = decltype(ND)::value;
        k_limcorr<T, nd><<<cb, 256, 0, s>>>(g, x, V[0], V[1], V[2], bup, bdn, G, mode, y, W[0],
                                            W[1], W[2]);
    });
    return hipGetLastError();
}

#define MP_INST(T)                                                                            \
    template hipError_t launch_donor<T>(const Geom &, const T *, const T *const[3], const T *, \
                                        int, T *, hipStream_t);                               \
    template hipError_t launch_pseudo<T>(const Geom &, unsigned, const T *, const T *const[3], \
                                         const T *, T *const[3], hipStream_t);                \
    template hipError_t launch_fct<T>(const Geom &, unsigned, const T *, const T *,            \
                                      const T *const[3], const T *, T *, T *, T *const[3],    \
                                      hipStream_t);                                           \
    template hipError_t limcorr_launch<T>(const Geom &, unsigned, const T *, const T *const[3], \
                                          const T *, const T *, const T *, T *, T *const[3],   \
                                          hipStream_t);
MP_INST(float)
MP_INST(double)
#undef MP_INST

// One full step psi_n -> psi_out through the staged kernels.
template <typename T>
hipError_t staged_step(const StagedArgs<T> &a, hipStream_t s)
{
    const Geom &g = a.g;
    const int B = 256;
    int64_t N = g.n[0] * g.n[1] * g.n[2];
    unsigned cblocks = (unsigned)cdiv(N, B);
    const bool fct = a.opts & OPT_FCT, iga = a.opts & OPT_IGA;

    T *out1 = (a.n_iters == 1) ? a.psi_out : a.tmp[0];
    const int km = (a.opts & OPT_KAHAN) ? 2 : 0;
    with_nd(g.nd, [&](auto ND) {
        k_donor<T, decltype(ND)::value><<<cblocks, B, 0, s>>>(g, a.psi_n, a.c[0], a.c[1], a.c[2],
                                                              a.G, km, out1);
    });
    const T *cprev[3] = {a.c[0], a.c[1], a.c[2]};
    const T *x = out1;
    int set = 0;
    for (int it = 2; it <= a.n_iters; it++) {
        // raw pseudo-velocity into the face set not holding cprev
        T *const *raw = a.faces[set];
        for (int d = 0; d < g.nd; d++) {
            unsigned wb = (unsigned)cdiv(wall_count<T>(g, d), B);
            pseudo_dispatch<T>(g, d, wb, B, s, a.opts, x, cprev[0], cprev[1], cprev[2], a.G,
                                         raw[d]);
        }
        T *const *adv = raw;
        if (fct) {
            T *const *lim = a.faces[set ^ 1];
            with_nd(g.nd, [&](auto ND) {
                k_fct_beta<T, decltype(ND)::value><<<cblocks, B, 0, s>>>(
                    g, a.opts, a.psi_n, x, raw[0], raw[1], raw[2], a.G, a.bup, a.bdn);
            });
            for (int d = 0; d < g.nd; d++) {
                unsigned wb = (unsigned)cdiv(wall_count<T>(g, d), B);
                with_nd_d(g.nd, d, [&](auto ND, auto WD) {
                    k_fct_limit<T, decltype(ND)::value, decltype(WD)::value><<<wb, B, 0, s>>>(
                        g, raw[d], a.bup, a.bdn, lim[d]);
                });
            }
            adv = lim;
        } else {
            set ^= 1;
        }
        T *y = (it == a.n_iters) ? a.psi_out : a.tmp[(it - 1) & 1];
        with_nd(g.nd, [&](auto ND) {
            k_donor<T, decltype(ND)::value><<<cblocks, B, 0, s>>>(g, x, adv[0], adv[1], adv[2],
                                                                  a.G, (iga ? 1 : 0) | km, y);
        });
        for (int d = 0; d < 3; d++) cprev[d] = adv[d];
        x = y;
    }
    return hipGetLastError();
}

template hipError_t staged_step<float>(const StagedArgs<float> &, hipStream_t);
template hipError_t staged_step<double>(const StagedArgs<double> &, hipStream_t);
// the tangent-linear step: value and derivative through the same stages
template hipError_t staged_step<Dual<float>>(const StagedArgs<Dual<float>> &, hipStream_t);
template hipError_t staged_step<Dual<double>>(const StagedArgs<Dual<double>> &, hipStream_t);

}  // namespace mp
