// adjoint.hip -- reverse-mode MPDATA step (placeholder until implemented).
#include "adjoint.hpp"

namespace mp {

size_t adj_extra_bytes(const Geom &, size_t, int, int, int) { return 0; }

template <typename T> hipError_t adjoint_run(const AdjArgs<T> &, hipStream_t)
{
    return hipErrorNotSupported;
}

template hipError_t adjoint_run<float>(const AdjArgs<float> &, hipStream_t);
template hipError_t adjoint_run<double>(const AdjArgs<double> &, hipStream_t);

}  // namespace mp
