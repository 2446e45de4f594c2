// tlm.hip -- the tangent-linear step (forward-mode derivative of the full
// nonlinear MPDATA step; an extension of the method, not in the paper).
//
// psi and its tangent dpsi, the advector and its tangent dc are packed into
// dual numbers (dual.hpp), advanced by the stage-by-stage kernels
// instantiated on the dual type, and unpacked.  G is a constant (zero
// tangent).  The dual arrays live in the plan's workspace.
#include "common.hpp"
#include "dual.hpp"
#include "kernels.hpp"

namespace mp {
namespace {

constexpr int TB = 256;

template <typename T>
__global__ void k_pack(Dual<T> *__restrict__ out, const T *__restrict__ v,
                       const T *__restrict__ d, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TB)
        out[i] = Dual<T>(v[i], d ? d[i] : T(0));
}

template <typename T>
__global__ void k_unpack(const Dual<T> *__restrict__ in, T *__restrict__ v, T *__restrict__ d,
                         int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * TB) {
        const Dual<T> x = in[i];
        v[i] = x.v;
        d[i] = x.d;
    }
}

unsigned blocks(int64_t n)
{
    const int64_t b = cdiv(n, TB);
    return (unsigned)(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

size_t up256(size_t v) { return (v + 255) / 256 * 256; }

int64_t walls(const Geom &g, int d)
{
    int64_t e[3] = {g.n[0], g.n[1], g.n[2]};
    e[d] += 1;
    return e[0] * e[1] * e[2];
}

// workspace carving (sizing with base == nullptr)
template <typename T> struct TlmWs {
    Dual<T> *psi, *alt, *G, *c[3], *tmp[2], *faces[2][3], *bup, *bdn;
    size_t bytes;
};

template <typename T> TlmWs<T> carve(const Geom &g, bool has_g, char *base)
{
    TlmWs<T> w{};
    size_t off = 0;
    auto take = [&](int64_t n) -> Dual<T> * {
        Dual<T> *p = base ? (Dual<T> *)(base + off) : nullptr;
        off += up256((size_t)n * sizeof(Dual<T>));
        return p;
    };
    const int64_t N = g.n[0] * g.n[1] * g.n[2];
    w.psi = take(N);
    w.alt = take(N);
    w.G = has_g ? take(N) : nullptr;
    for (int d = 0; d < 3; d++) w.c[d] = d < g.nd ? take(walls(g, d)) : nullptr;
    w.tmp[0] = take(N);
    w.tmp[1] = take(N);
    for (int s = 0; s < 2; s++)
        for (int d = 0; d < 3; d++) w.faces[s][d] = d < g.nd ? take(walls(g, d)) : nullptr;
    w.bup = take(N);
    w.bdn = take(N);
    w.bytes = off;
    return w;
}

}  // namespace

size_t tlm_workspace_bytes(const Geom &g, int f64, int has_g)
{
    return f64 ? carve<double>(g, has_g != 0, nullptr).bytes
               : carve<float>(g, has_g != 0, nullptr).bytes;
}

template <typename T>
hipError_t tlm_steps(const Geom &g, int n_iters, unsigned opts, T *psi, T *dpsi, const T *G,
                     const T *const c[3], const T *const dc[3], int n_steps, void *ws,
                     hipStream_t s)
{
    TlmWs<T> w = carve<T>(g, G != nullptr, (char *)ws);
    const int64_t N = g.n[0] * g.n[1] * g.n[2];
    k_pack<T><<<blocks(N), TB, 0, s>>>(w.psi, psi, dpsi, N);
    if (G) k_pack<T><<<blocks(N), TB, 0, s>>>(w.G, G, nullptr, N);
    for (int d = 0; d < g.nd; d++)
        k_pack<T><<<blocks(walls(g, d)), TB, 0, s>>>(w.c[d], c[d], dc[d], walls(g, d));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    StagedArgs<Dual<T>> a;
    a.g = g;
    a.n_iters = n_iters;
    a.opts = opts;
    for (int d = 0; d < 3; d++) a.c[d] = w.c[d];
    a.G = w.G;
    a.tmp[0] = w.tmp[0];
    a.tmp[1] = w.tmp[1];
    for (int t = 0; t < 2; t++)
        for (int d = 0; d < 3; d++) a.faces[t][d] = w.faces[t][d];
    a.bup = w.bup;
    a.bdn = w.bdn;
    // the last pass reads only pass results, so with two or more passes the
    // step may write in place; a single pass alternates with the spare buffer
    Dual<T> *cur = w.psi, *nxt = n_iters >= 2 ? w.psi : w.alt;
    for (int st = 0; st < n_steps; st++) {
        a.psi_n = cur;
        a.psi_out = nxt;
        e = staged_step<Dual<T>>(a, s);
        if (e != hipSuccess) return e;
        if (n_iters < 2) {
            Dual<T> *t = cur;
            cur = nxt;
            nxt = t;
        }
    }
    k_unpack<T><<<blocks(N), TB, 0, s>>>(cur, psi, dpsi, N);
    return hipGetLastError();
}

template hipError_t tlm_steps<float>(const Geom &, int, unsigned, float *, float *, const float *,
                                     const float *const[3], const float *const[3], int, void *,
                                     hipStream_t);
template hipError_t tlm_steps<double>(const Geom &, int, unsigned, double *, double *,
                                      const double *, const double *const[3],
                                      const double *const[3], int, void *, hipStream_t);

}  // namespace mp
