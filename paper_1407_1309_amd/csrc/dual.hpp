// dual.hpp -- first-order dual numbers for the tangent-linear step.
//
// Dual<T>{v, d} carries a value and its directional derivative.  Running the
// stage-by-stage kernels on Dual<T> evaluates the step and its derivative
// along (dpsi, dc) together (forward mode).  The derivative conventions at
// the method's kinks are those of the reverse mode:
//   d[u]+/du = [u > 0] and d[u]-/du = [u < 0] (a comparison picks a branch
//   by value, so the branch's own derivative is taken);
//   d|u|/du = [u > 0] - [u < 0];
//   max / min pass the derivative of the operand they return, ties to the
//   first operand (the running extremum, i.e. the earliest in scan order);
//   a branch chosen by a zero test (zero denominator, no flux) has the
//   derivative of its constant.
#pragma once

#include <hip/hip_runtime.h>

namespace mp {

template <typename T> struct Dual {
    T v, d;
    __host__ __device__ Dual() : v(0), d(0) {}
    __host__ __device__ Dual(T value) : v(value), d(0) {}   // constant
    __host__ __device__ Dual(T value, T deriv) : v(value), d(deriv) {}

    friend __host__ __device__ Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
    friend __host__ __device__ Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
    friend __host__ __device__ Dual operator-(Dual a) { return {-a.v, -a.d}; }
    friend __host__ __device__ Dual operator*(Dual a, Dual b)
    {
        return {a.v * b.v, a.v * b.d + a.d * b.v};
    }
    friend __host__ __device__ Dual operator/(Dual a, Dual b)
    {
        const T q = a.v / b.v;
        return {q, (a.d - q * b.d) / b.v};
    }
    __host__ __device__ Dual &operator+=(Dual b) { return *this = *this + b; }
    __host__ __device__ Dual &operator-=(Dual b) { return *this = *this - b; }
    __host__ __device__ Dual &operator*=(Dual b) { return *this = *this * b; }
    __host__ __device__ Dual &operator/=(Dual b) { return *this = *this / b; }

    friend __host__ __device__ bool operator<(Dual a, Dual b) { return a.v < b.v; }
    friend __host__ __device__ bool operator>(Dual a, Dual b) { return a.v > b.v; }
    friend __host__ __device__ bool operator<=(Dual a, Dual b) { return a.v <= b.v; }
    friend __host__ __device__ bool operator>=(Dual a, Dual b) { return a.v >= b.v; }
    friend __host__ __device__ bool operator==(Dual a, Dual b) { return a.v == b.v; }
    friend __host__ __device__ bool operator!=(Dual a, Dual b) { return a.v != b.v; }

    friend __host__ __device__ Dual fabs(Dual a)
    {
        return {a.v < T(0) ? -a.v : a.v, a.v > T(0) ? a.d : (a.v < T(0) ? -a.d : T(0))};
    }
    friend __host__ __device__ Dual fmax(Dual a, Dual b) { return a.v >= b.v ? a : b; }
    friend __host__ __device__ Dual fmin(Dual a, Dual b) { return a.v <= b.v ? a : b; }
};

}  // namespace mp
