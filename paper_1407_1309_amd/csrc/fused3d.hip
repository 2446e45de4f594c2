// fused3d.hip -- the 3-D donor-cell step (n_iters = 1) in one launch, and
// the dispatch of the 3-D steps: two passes without the limiter are one
// launch of the kernel of step3d.hip; with the limiter, or more passes, the
// same kernel forms each pass's raw pseudo-velocities (and the limiter
// coefficients) and a cell kernel of staged.hip applies the limited
// velocities and the corrective pass, pass by pass.
//
//   k_donor3d : donor-cell pass, psi^n -> y.  Each thread owns a (j, k)
//               column and marches along i over a chunk of planes, keeping
//               psi at i-1, i, i+1 and the dimension-0 walls in registers;
//               in-plane neighbours are read through L1/L2.
// Every global read goes through the boundary map (periodic wrap / open
// clamp).  Tiles are numbered so that neighbouring tiles run on the same
// XCD and share its L2 for their overlapping neighbour reads.
#include "common.hpp"
#include "kernels.hpp"


namespace mp {
namespace {

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
            T flo = upwind_fp(ulo, xm, xc);
            T fhi = upwind_fp(uhi, xc, xp);
            dv[0] = fhi - flo;
        }
        {
            T ul = c1[i * pl1 + w1lo], uh = c1[i * pl1 + w1hi];
            T flo = upwind_fp(ul, x[pc + ojm], xc);
            T fhi = upwind_fp(uh, xc, x[pc + ojp]);
            dv[1] = fhi - flo;
        }
        {
            T ul = c2[i * pl2 + w2lo], uh = c2[i * pl2 + w2hi];
            T flo = upwind_fp(ul, x[pc + okm], xc);
            T fhi = upwind_fp(uh, xc, x[pc + okp]);
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

}  // namespace

bool fused3d_supported(int nd, int n_iters, unsigned opts, const int64_t n[3], const int bc[3])
{
    (void)bc;
    // (n_iters = 1: the limiter, abs and dfl have nothing to act on)
    if (nd != 3 || n_iters < 1) return false;
    if (n_iters >= 2) return step3d_supported(nd, n_iters, opts, n);
    return n[0] < (1 << 30) && n[1] < (1 << 30) && n[2] < (1 << 30);
}

template <typename T>
hipError_t fused3d_step(const Geom &geom, int n_iters, unsigned opts, const T *psi_n, T *psi_out,
                        const T *c0, const T *c1, const T *c2, const T *G, int tile_planes,
                        hipStream_t s, const Fused3DWork<T> &w)
{
    if (n_iters >= 2) {
        if (!step3d_supported(geom.nd, n_iters, opts, geom.n)) return hipErrorNotSupported;
        const bool fct = opts & OPT_FCT;
        if (n_iters == 2 && !fct)
            return step3d_launch<T>(geom, opts, psi_n, psi_out, c0, c1, c2, G, tile_planes, s);
        // pass by pass: the 3-D kernel forms the pass's raw
        // pseudo-velocities (pass 2 from the donor pass it forms itself,
        // which it also writes; later passes from the previous result) and
        // the limiter coefficients, then a cell kernel applies the limited
        // velocities and the corrective pass.
        // Buffers: the pass input in cell[xs], its advector in wall[as]
        // (the input advector for pass 2), its raw velocities into the
        // other wall set, its limited velocities (the next advector) into
        // wall[as] once the raw ones are formed.
        const int mode = ((opts & OPT_IGA) ? 1 : 0) | ((opts & OPT_KAHAN) ? 2 : 0);
        const T *x = nullptr;
        const T *adv[3] = {c0, c1, c2};
        int xs = 0, as = 1;
        for (int it = 2; it <= n_iters; it++) {
            const bool last = it == n_iters;
            const int vs = 1 - as;                   // wall set for this pass's raw velocities
            Step3dOut<T> vo;
            vo.xin = x;
            if (!x) vo.y1 = w.cell[0];               // pass 2: keep the donor result
            vo.v0 = w.wall[vs][0];
            vo.v1 = w.wall[vs][1];
            vo.v2 = w.wall[vs][2];
            // with the limiter the same launch forms the coefficients
            if (fct) {
                vo.bup = w.bup;
                vo.bdn = w.bdn;
            }
            hipError_t e = step3d_launch<T>(geom, opts & ~OPT_FCT, psi_n, nullptr, adv[0], adv[1],
                                            adv[2], G, tile_planes, s, vo);
            if (e != hipSuccess) return e;
            const T *xp = x ? x : w.cell[0];
            T *y = last ? psi_out : w.cell[1 - xs];
            const T *V[3] = {w.wall[vs][0], w.wall[vs][1], w.wall[vs][2]};
            if (fct) {
                T *W[3] = {nullptr, nullptr, nullptr};
                if (!last)
                    for (int d = 0; d < 3; d++) W[d] = w.wall[as][d];
                // (the next pass's advector W stays in wall[as]; its raw
                // velocities go to the set that held V)
                e = limcorr_launch<T>(geom, opts, xp, V, G, w.bup, w.bdn, y, W, s);
                for (int d = 0; d < 3; d++) adv[d] = W[d];
            } else {
                e = launch_donor<T>(geom, xp, V, G, mode, y, s);
                for (int d = 0; d < 3; d++) adv[d] = V[d];
                as = vs;                             // the next advector is V
            }
            if (e != hipSuccess) return e;
            x = y;
            xs = 1 - xs;
        }
        return hipGetLastError();
    }
    if (n_iters != 1) return hipErrorNotSupported;
    G3 g{(int)geom.n[0], (int)geom.n[1], (int)geom.n[2], geom.bc[0], geom.bc[1], geom.bc[2]};
    const int dk = (int)cdiv(g.n2, 64), dj = (int)cdiv(g.n1, 4);
    const int64_t dblk = (int64_t)dk * dj * cdiv(g.n0, DONOR_PLANES);
    if (dblk > INT32_MAX) return hipErrorInvalidValue;
    const int kahan = (opts & OPT_KAHAN) ? 1 : 0;
    if (G)
        k_donor3d<T, true><<<(unsigned)dblk, 256, 0, s>>>(g, kahan, dk, dj, (int)dblk, psi_n, c0,
                                                          c1, c2, G, psi_out);
    else
        k_donor3d<T, false><<<(unsigned)dblk, 256, 0, s>>>(g, kahan, dk, dj, (int)dblk, psi_n, c0,
                                                           c1, c2, G, psi_out);
    return hipGetLastError();
}

template hipError_t fused3d_step<float>(const Geom &, int, unsigned, const float *, float *,
                                        const float *, const float *, const float *,
                                        const float *, int, hipStream_t,
                                        const Fused3DWork<float> &);
template hipError_t fused3d_step<double>(const Geom &, int, unsigned, const double *, double *,
                                         const double *, const double *, const double *,
                                         const double *, int, hipStream_t,
                                         const Fused3DWork<double> &);

}  // namespace mp
