// resident1d.hip -- 1-D MPDATA steps with the whole grid resident in LDS.
//
// A 1-D grid of up to a few hundred cells is far too small to fill the chip,
// so its cost is launch latency.  One workgroup keeps psi, the advector, G
// and every intermediate field in LDS and runs all n_steps of a call in a
// single launch, stage by stage with workgroup barriers in between.  Every
// option (tot, iga, fct, G, periodic / open) is supported.
#include "common.hpp"
#include "kernels.hpp"

namespace mp {
namespace {

constexpr int RB = 512;            // threads
constexpr size_t LDS_BYTES = 160 * 1024;   // upper bound; the device's limit applies

__device__ inline int mc(int q, int n, int bc)
{
    if (bc == BC_PERIODIC) {
        q %= n;
        return q < 0 ? q + n : q;
    }
    return q < 0 ? 0 : (q >= n ? n - 1 : q);
}

__device__ inline int mw(int f, int n, int bc)
{
    if (bc == BC_PERIODIC) {
        f %= n;
        return f < 0 ? f + n : f;
    }
    return f < 0 ? 0 : (f > n ? n : f);
}

template <typename T> __device__ inline T rfrac(bool iga, T num, T den, T m)
{
    if (iga) return num / m;
    return den == T(0) ? T(0) : num / den;
}

// With phi != nullptr the kernel advances the translating oscillator pair
// (psi, phi) with the trapezoidal coupling of strength osc_a (= dt omega / 2):
// explicit half, one MPDATA step of each field, implicit half in closed form.
template <typename T>
__global__ void __launch_bounds__(RB) k_resident1d(int n, int bc, int n_iters, unsigned opts,
                                                   T *psi, const T *__restrict__ cin,
                                                   const T *__restrict__ Gin, int n_steps,
                                                   T *phi, T osc_a)
{
    extern __shared__ char lds_raw[];
    T *P = (T *)lds_raw;          // psi at the start of the step
    T *Q = P + n;                 // phi (oscillator only)
    T *X = Q + (phi ? n : 0);     // pass input
    T *Y = X + n;                 // pass output
    T *BU = Y + n;
    T *BD = BU + n;
    T *GG = BD + n;               // G (n values, only with Gin)
    T *C = GG + (Gin ? n : 0);    // input advector (n+1)
    T *W0 = C + (n + 1);          // three wall buffers
    T *W1 = W0 + (n + 1);
    T *W2 = W1 + (n + 1);
    const bool fct = opts & OPT_FCT, iga = opts & OPT_IGA, tot = opts & OPT_TOT;
    const bool kahan = opts & OPT_KAHAN, absf = opts & OPT_ABS, dfl = opts & OPT_DFL;
    // donor-cell update from the flux difference acc (straightforward, or
    // Kahan-compensated: psi + (-acc / G) as a compensated sum)
    auto upd = [&](T x, T acc, int i) -> T {
        if (kahan) {
            T s = x, c = T(0);
            kahan_add(s, c, -(Gin ? acc / GG[i] : acc));
            return s;
        }
        return x - (Gin ? acc / GG[i] : acc);
    };
    const int tid = threadIdx.x;

    for (int i = tid; i < n; i += RB) {
        P[i] = psi[i];
        if (phi) Q[i] = phi[i];
        if (Gin) GG[i] = Gin[i];
    }
    for (int f = tid; f <= n; f += RB) C[f] = cin[f];
    __syncthreads();

    auto gv = [&](int i) -> T { return Gin ? GG[mc(i, n, bc)] : T(1); };

    // one MPDATA step of the field F in place (F -> Y -> F)
    auto advect = [&](T *F) {
        // donor-cell pass: F -> Y
        for (int i = tid; i < n; i += RB) {
            T ul = C[mw(i, n, bc)], uh = C[mw(i + 1, n, bc)];
            T flo = upwind_fp(ul, F[mc(i - 1, n, bc)], F[i]);
            T fhi = upwind_fp(uh, F[i], F[mc(i + 1, n, bc)]);
            T acc = fhi - flo;
            Y[i] = upd(F[i], acc, i);
        }
        __syncthreads();
        const T *cprev = C;
        for (int it = 2; it <= n_iters; it++) {
            // move Y into X; raw and limited velocities go to the two wall
            // buffers that do not hold the previous pass's advector
            for (int i = tid; i < n; i += RB) X[i] = Y[i];
            T *cand[3] = {W0, W1, W2};
            T *V = nullptr, *Wl = nullptr;
            for (int k = 0; k < 3; k++) {
                if (cand[k] == cprev) continue;
                if (!V)
                    V = cand[k];
                else if (!Wl)
                    Wl = cand[k];
            }
            __syncthreads();
            // pseudo-velocity at every wall
            for (int f = tid; f <= n; f += RB) {
                int L = f - 1, R = f;
                T u = cprev[mw(f, n, bc)];
                T Gb = T(0.5) * (gv(L) + gv(R));
                // |psi| in the psi-fractions under the abs option
                T xL = X[mc(L, n, bc)], xR = X[mc(R, n, bc)];
                if (absf) {
                    xL = fabs(xL);
                    xR = fabs(xR);
                }
                T v = (fabs(u) - u * u / Gb) * rfrac(iga, xR - xL, xR + xL, T(2));
                if (tot) {
                    T xR2 = X[mc(R + 1, n, bc)], xL2 = X[mc(L - 1, n, bc)];
                    if (absf) {
                        xR2 = fabs(xR2);
                        xL2 = fabs(xL2);
                    }
                    T D = rfrac(iga, xR2 - xR - xL + xL2, xR2 + xR + xL + xL2, T(4));
                    v += (T(3) * u * fabs(u) / Gb - T(2) * u * u * u / (Gb * Gb) - u) / T(3) * D;
                }
                if (dfl) {
                    // divergent-flow term: -c/(2 Gb) times the mean divergence
                    // (c(f+1) - c(f)) + (c(f) - c(f-1)) of the two cells
                    T dv = (cprev[mw(f + 1, n, bc)] - cprev[mw(f, n, bc)]) +
                           (cprev[mw(f, n, bc)] - cprev[mw(f - 1, n, bc)]);
                    // under iga: times the wall mean of psi (unit-field flux)
                    if (iga) dv *= T(0.5) * (xL + xR);
                    v -= T(0.25) * u / Gb * dv;
                }
                V[f] = v;
            }
            __syncthreads();
            const T *adv = V;
            if (fct) {
                for (int i = tid; i < n; i += RB) {
                    T xi = X[i];
                    T mx = fmax(F[i], xi), mn = fmin(F[i], xi);
                    for (int s = -1; s <= 1; s += 2) {
                        int q = mc(i + s, n, bc);
                        mx = fmax(fmax(mx, F[q]), X[q]);
                        mn = fmin(fmin(mn, F[q]), X[q]);
                    }
                    T vlo = V[mw(i, n, bc)], vhi = V[mw(i + 1, n, bc)];
                    T wm = iga ? T(1) : X[mc(i - 1, n, bc)];
                    T wp = iga ? T(1) : X[mc(i + 1, n, bc)];
                    T wc = iga ? T(1) : xi;
                    T fin = pos(vlo) * wm - neg(vhi) * wp;
                    T fout = pos(vhi) * wc - neg(vlo) * wc;
                    T Gi = Gin ? GG[i] : T(1);
                    BU[i] = fin > T(0) ? Gi * (mx - xi) / fin : T(1);
                    BD[i] = fout > T(0) ? Gi * (xi - mn) / fout : T(1);
                }
                __syncthreads();
                for (int f = tid; f <= n; f += RB) {
                    int L = mc(f - 1, n, bc), R = mc(f, n, bc);
                    T v = V[f];
                    T up = fmin(fmin(T(1), BD[L]), BU[R]);
                    T dn = fmin(fmin(T(1), BU[L]), BD[R]);
                    Wl[f] = pos(v) * up + neg(v) * dn;
                }
                __syncthreads();
                adv = Wl;
            }
            // corrective donor-cell pass: X -> Y
            for (int i = tid; i < n; i += RB) {
                T ul = adv[mw(i, n, bc)], uh = adv[mw(i + 1, n, bc)];
                T flo, fhi;
                if (iga) {
                    flo = ul;
                    fhi = uh;
                } else {
                    flo = pos(ul) * X[mc(i - 1, n, bc)] + neg(ul) * X[i];
                    fhi = pos(uh) * X[i] + neg(uh) * X[mc(i + 1, n, bc)];
                }
                T acc = fhi - flo;
                Y[i] = upd(X[i], acc, i);
            }
            cprev = adv;
            __syncthreads();
        }
        for (int i = tid; i < n; i += RB) F[i] = Y[i];
        __syncthreads();
    };

    for (int step = 0; step < n_steps; step++) {
        if (phi) {
            // explicit half of the coupling: (psi, phi) += a (phi, -psi)
            for (int i = tid; i < n; i += RB) {
                T x = P[i], y = Q[i];
                P[i] = x + osc_a * y;
                Q[i] = y - osc_a * x;
            }
            __syncthreads();
            advect(P);
            advect(Q);
            // implicit half in closed form
            const T den = T(1) + osc_a * osc_a;
            for (int i = tid; i < n; i += RB) {
                T x = P[i], y = Q[i];
                P[i] = (x + osc_a * y) / den;
                Q[i] = (y - osc_a * x) / den;
            }
            __syncthreads();
        } else {
            advect(P);
        }
    }
    for (int i = tid; i < n; i += RB) {
        psi[i] = P[i];
        if (phi) phi[i] = Q[i];
    }
}

size_t lds_need(int n, size_t es, bool has_g, bool two)
{
    return es * ((5 + (has_g ? 1 : 0) + (two ? 1 : 0)) * (size_t)n + 4 * ((size_t)n + 1));
}

// LDS a workgroup may use on the current device (160 KB on gfx950)
size_t lds_limit()
{
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 64 * 1024;
    }
    return (size_t)v < LDS_BYTES ? (size_t)v : LDS_BYTES;
}

template <typename T>
hipError_t launch_resident(int64_t n, int bc, int n_iters, unsigned opts, T *psi, const T *c,
                           const T *G, int n_steps, T *phi, double a, hipStream_t s)
{
    size_t lds = lds_need((int)n, sizeof(T), G != nullptr, phi != nullptr);
    if (lds > lds_limit()) return hipErrorInvalidValue;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)k_resident1d<T>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    k_resident1d<T><<<1, RB, lds, s>>>((int)n, bc, n_iters, opts, psi, c, G, n_steps, phi, (T)a);
    return hipGetLastError();
}

}  // namespace

bool resident1d_supported(int nd, int64_t n, int dtype_is_f64, int has_g, int two_fields)
{
    if (nd != 1 || n < 1 || n > (1 << 20)) return false;
    return lds_need((int)n, dtype_is_f64 ? 8 : 4, has_g != 0, two_fields != 0) <= lds_limit();
}

template <typename T>
hipError_t resident1d_steps(int64_t n, int bc, int n_iters, unsigned opts, T *psi, const T *c,
                            const T *G, int n_steps, hipStream_t s)
{
    return launch_resident<T>(n, bc, n_iters, opts, psi, c, G, n_steps, nullptr, 0.0, s);
}

template <typename T>
hipError_t resident1d_osc(int64_t n, int bc, int n_iters, unsigned opts, T *psi, T *phi,
                          const T *c, const T *G, double a, int n_steps, hipStream_t s)
{
    return launch_resident<T>(n, bc, n_iters, opts, psi, c, G, n_steps, phi, a, s);
}

template hipError_t resident1d_steps<float>(int64_t, int, int, unsigned, float *, const float *,
                                            const float *, int, hipStream_t);
template hipError_t resident1d_steps<double>(int64_t, int, int, unsigned, double *,
                                             const double *, const double *, int, hipStream_t);
template hipError_t resident1d_osc<float>(int64_t, int, int, unsigned, float *, float *,
                                          const float *, const float *, double, int, hipStream_t);
template hipError_t resident1d_osc<double>(int64_t, int, int, unsigned, double *, double *,
                                           const double *, const double *, double, int,
                                           hipStream_t);

}  // namespace mp
