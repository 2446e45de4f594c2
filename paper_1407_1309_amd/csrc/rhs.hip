// rhs.hip -- elementwise kernels around the MPDATA step for the inhomogeneous
// transport equation (Sect. 4.1: source terms applied before and / or after
// the advection) and for the translating oscillator's trapezoidal coupling
// (Sect. 4.3).  Grid-stride loops over the cells; each kernel reads and
// writes every cell once.
#include "common.hpp"
#include "kernels.hpp"

namespace mp {
namespace {

constexpr int EB = 256;

template <typename T> __global__ void k_axpy(T *y, const T *__restrict__ x, T a, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * EB + threadIdx.x; i < n; i += (int64_t)gridDim.x * EB)
        y[i] += a * x[i];
}

// explicit half of the coupling: (psi, phi) <- (psi + a phi, phi - a psi)
template <typename T> __global__ void k_osc_explicit(T *psi, T *phi, T a, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * EB + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * EB) {
        T x = psi[i], y = phi[i];
        psi[i] = x + a * y;
        phi[i] = y - a * x;
    }
}

// implicit half, solved in closed form (eq. final_osc):
// (psi, phi) <- ((psi + a phi), (phi - a psi)) / (1 + a^2)
template <typename T> __global__ void k_osc_implicit(T *psi, T *phi, T a, T den, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * EB + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * EB) {
        T x = psi[i], y = phi[i];
        psi[i] = (x + a * y) / den;
        phi[i] = (y - a * x) / den;
    }
}

unsigned grid_for(int64_t n)
{
    int64_t b = cdiv(n, EB);
    return (unsigned)(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

}  // namespace

template <typename T> hipError_t axpy_launch(T *y, const T *x, double a, int64_t n, hipStream_t s)
{
    k_axpy<T><<<grid_for(n), EB, 0, s>>>(y, x, (T)a, n);
    return hipGetLastError();
}

template <typename T>
hipError_t osc_couple_launch(T *psi, T *phi, double a, int implicit, int64_t n, hipStream_t s)
{
    if (implicit)
        k_osc_implicit<T><<<grid_for(n), EB, 0, s>>>(psi, phi, (T)a, (T)(1.0 + a * a), n);
    else
        k_osc_explicit<T><<<grid_for(n), EB, 0, s>>>(psi, phi, (T)a, n);
    return hipGetLastError();
}

template hipError_t axpy_launch<float>(float *, const float *, double, int64_t, hipStream_t);
template hipError_t axpy_launch<double>(double *, const double *, double, int64_t, hipStream_t);
template hipError_t osc_couple_launch<float>(float *, float *, double, int, int64_t, hipStream_t);
template hipError_t osc_couple_launch<double>(double *, double *, double, int, int64_t,
                                              hipStream_t);

}  // namespace mp
