// sw.hip -- prognosed velocity (Sect. 5.1-5.2) and the pressure-gradient
// forcing of the shallow-water equations (eqs. shw1d, shw2d).
//
// Both kernels are elementwise with small stencils and bound by HBM
// traffic; each thread handles one wall (advector) or one cell (forcing) in
// a grid-stride loop.  Contraction into FMA is off in this file, so in FP64
// every value is the correctly rounded result of the same operations in the
// same order as a plain evaluation of the formulas.
#include "common.hpp"
#include "kernels.hpp"

#pragma clang fp contract(off)

namespace mp {
namespace {

constexpr int SB = 256;

// cell velocity: num / den, 0 where den <= eps; num itself without den
template <typename T>
__device__ inline T vel(const T *__restrict__ num, const T *__restrict__ den, int64_t i, T eps)
{
    if (!den) return num[i];
    T h = den[i];
    return h > eps ? num[i] / h : T(0);
}

// Advector component WD at every wall: the velocity extrapolated to n+1/2,
// 1.5 u^n - 0.5 u^(n-1), averaged over the wall's two cells (through the
// boundary map), times k = dt / dx_WD.
template <typename T, int WD>
__global__ void k_vip(Geom g, const T *__restrict__ num, const T *__restrict__ den,
                      const T *__restrict__ nump, const T *__restrict__ denp, T eps, T k,
                      T *__restrict__ c)
{
    int64_t e[3] = {g.n[0], g.n[1], g.n[2]};
    e[WD] += 1;
    const int64_t M = e[0] * e[1] * e[2];
    const int64_t stride = WD == 2 ? 1 : (WD == 1 ? g.n[2] : g.n[1] * g.n[2]);
    for (int64_t t = (int64_t)blockIdx.x * SB + threadIdx.x; t < M;
         t += (int64_t)gridDim.x * SB) {
        int v[3];
        unflat3(t, e, v);
        const int64_t f = v[WD];
        v[WD] = 0;
        const int64_t base = ((int64_t)v[0] * g.n[1] + v[1]) * g.n[2] + v[2];
        const int64_t iL = base + map_cell(f - 1, g.n[WD], g.bc[WD]) * stride;
        const int64_t iR = base + map_cell(f, g.n[WD], g.bc[WD]) * stride;
        T uL = T(1.5) * vel(num, den, iL, eps) - T(0.5) * vel(nump, denp, iL, eps);
        T uR = T(1.5) * vel(num, den, iR, eps) - T(0.5) * vel(nump, denp, iR, eps);
        c[t] = k * (T(0.5) * (uL + uR));
    }
}

// Momentum forcing: q_d += (dt/2) (-g h dh/dx_d), the derivative as the
// centred difference through the boundary map.  With save set, the
// previous level is taken first: q_prev_d = q_d, h_prev = h.
template <typename T>
__global__ void k_sw_force(Geom g, const T *__restrict__ h, T *__restrict__ h_prev, T *q0,
                           T *q1, T *q2, T *qp0, T *qp1, T *qp2, T ngrav, T tdx0, T tdx1,
                           T tdx2, T half_dt, int save)
{
    const int64_t e[3] = {g.n[0], g.n[1], g.n[2]};
    const int64_t M = e[0] * e[1] * e[2];
    const int64_t st[3] = {e[1] * e[2], e[2], 1};
    T *q[3] = {q0, q1, q2};
    T *qp[3] = {qp0, qp1, qp2};
    const T tdx[3] = {tdx0, tdx1, tdx2};
    for (int64_t t = (int64_t)blockIdx.x * SB + threadIdx.x; t < M;
         t += (int64_t)gridDim.x * SB) {
        int v[3];
        unflat3(t, e, v);
        const T hc = h[t];
        if (save) h_prev[t] = hc;
#pragma unroll
        for (int d = 0; d < 3; d++) {
            if (d >= g.nd) break;
            const int64_t base = t - (int64_t)v[d] * st[d];
            const T hp = h[base + map_cell(v[d] + 1, e[d], g.bc[d]) * st[d]];
            const T hm = h[base + map_cell(v[d] - 1, e[d], g.bc[d]) * st[d]];
            const T f = ngrav * hc * (hp - hm) / tdx[d];
            const T qc = q[d][t];
            if (save) qp[d][t] = qc;
            q[d][t] = qc + half_dt * f;
        }
    }
}

// The save-phase forcing of one momentum component d written elsewhere: out
// = q + (dt/2)(-g h dh/dx_d) (the same expressions as above), q itself left
// at level n and copied to qp; h_prev, when given, receives h.  The step
// then advects out into q, with no copy of q into the workspace.
template <typename T>
__global__ void k_sw_force1(Geom g, int d, const T *__restrict__ h, T *__restrict__ h_prev,
                            const T *__restrict__ q, T *__restrict__ qp, T *__restrict__ out,
                            T ngrav, T tdx, T half_dt)
{
    const int64_t e[3] = {g.n[0], g.n[1], g.n[2]};
    const int64_t M = e[0] * e[1] * e[2];
    const int64_t st[3] = {e[1] * e[2], e[2], 1};
    for (int64_t t = (int64_t)blockIdx.x * SB + threadIdx.x; t < M;
         t += (int64_t)gridDim.x * SB) {
        int v[3];
        unflat3(t, e, v);
        const T hc = h[t];
        if (h_prev) h_prev[t] = hc;
        const int64_t base = t - (int64_t)v[d] * st[d];
        const T hp = h[base + map_cell(v[d] + 1, e[d], g.bc[d]) * st[d]];
        const T hm = h[base + map_cell(v[d] - 1, e[d], g.bc[d]) * st[d]];
        const T f = ngrav * hc * (hp - hm) / tdx;
        const T qc = q[t];
        qp[t] = qc;
        out[t] = qc + half_dt * f;
    }
}

unsigned blocks_for(int64_t n)
{
    int64_t b = cdiv(n, SB);
    return (unsigned)(b < 16384 ? (b > 0 ? b : 1) : 16384);
}

}  // namespace

template <typename T>
hipError_t vip_launch(const Geom &g, const T *const num[3], const T *den, const T *const nump[3],
                      const T *denp, double eps, const double k[3], T *const c[3], hipStream_t s)
{
    for (int d = 0; d < g.nd; d++) {
        int64_t e[3] = {g.n[0], g.n[1], g.n[2]};
        e[d] += 1;
        const unsigned nb = blocks_for(e[0] * e[1] * e[2]);
        if (d == 0)
            k_vip<T, 0><<<nb, SB, 0, s>>>(g, num[0], den, nump[0], denp, (T)eps, (T)k[0], c[0]);
        else if (d == 1)
            k_vip<T, 1><<<nb, SB, 0, s>>>(g, num[1], den, nump[1], denp, (T)eps, (T)k[1], c[1]);
        else
            k_vip<T, 2><<<nb, SB, 0, s>>>(g, num[2], den, nump[2], denp, (T)eps, (T)k[2], c[2]);
        hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

template <typename T>
hipError_t sw_force_launch(const Geom &g, const T *h, T *h_prev, T *const q[3],
                           T *const q_prev[3], double grav, const double dx[3], double dt,
                           int save, hipStream_t s)
{
    const int64_t M = g.n[0] * g.n[1] * g.n[2];
    k_sw_force<T><<<blocks_for(M), SB, 0, s>>>(g, h, h_prev, q[0], q[1], q[2], q_prev[0],
                                               q_prev[1], q_prev[2], (T)(-grav),
                                               (T)(2.0 * dx[0]), (T)(2.0 * dx[1]),
                                               (T)(2.0 * dx[2]), (T)(0.5 * dt), save);
    return hipGetLastError();
}

template <typename T>
hipError_t sw_force1_launch(const Geom &g, int d, const T *h, T *h_prev, const T *q, T *q_prev,
                            T *out, double grav, const double dx[3], double dt, hipStream_t s)
{
    if (d < 0 || d >= g.nd || !q || !q_prev || !out) return hipErrorInvalidValue;
    const int64_t M = g.n[0] * g.n[1] * g.n[2];
    k_sw_force1<T><<<blocks_for(M), SB, 0, s>>>(g, d, h, h_prev, q, q_prev, out, (T)(-grav),
                                                (T)(2.0 * dx[d]), (T)(0.5 * dt));
    return hipGetLastError();
}

template hipError_t vip_launch<float>(const Geom &, const float *const[3], const float *,
                                      const float *const[3], const float *, double,
                                      const double[3], float *const[3], hipStream_t);
template hipError_t vip_launch<double>(const Geom &, const double *const[3], const double *,
                                       const double *const[3], const double *, double,
                                       const double[3], double *const[3], hipStream_t);
template hipError_t sw_force_launch<float>(const Geom &, const float *, float *, float *const[3],
                                           float *const[3], double, const double[3], double,
                                           int, hipStream_t);
template hipError_t sw_force_launch<double>(const Geom &, const double *, double *,
                                            double *const[3], double *const[3], double,
                                            const double[3], double, int, hipStream_t);
template hipError_t sw_force1_launch<float>(const Geom &, int, const float *, float *,
                                            const float *, float *, float *, double,
                                            const double[3], double, hipStream_t);
template hipError_t sw_force1_launch<double>(const Geom &, int, const double *, double *,
                                             const double *, double *, double *, double,
                                             const double[3], double, hipStream_t);

}  // namespace mp
