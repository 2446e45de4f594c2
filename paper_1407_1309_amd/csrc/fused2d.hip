// fused2d.hip -- placeholder until the fused kernel lands.
#include "kernels.hpp"

namespace mp {

bool fused2d_supported(int, int, unsigned, int) { return false; }
int fused2d_tile_rows() { return 64; }
int fused2d_tile_cols() { return 64; }

template <typename T>
hipError_t fused2d_step(const Fused2DShape &, int, unsigned, const T *, T *, const T *,
                        const T *, const T *, hipStream_t)
{
    return hipErrorNotSupported;
}

template <typename T>
hipError_t fused2d_batched_step(const BatchGrid *, int, int, int, int, unsigned, const T *, T *,
                                const T *, const T *, hipStream_t)
{
    return hipErrorNotSupported;
}

template hipError_t fused2d_step<float>(const Fused2DShape &, int, unsigned, const float *, float *,
                                        const float *, const float *, const float *, hipStream_t);
template hipError_t fused2d_step<double>(const Fused2DShape &, int, unsigned, const double *,
                                         double *, const double *, const double *, const double *,
                                         hipStream_t);
template hipError_t fused2d_batched_step<float>(const BatchGrid *, int, int, int, int, unsigned,
                                                const float *, float *, const float *,
                                                const float *, hipStream_t);
template hipError_t fused2d_batched_step<double>(const BatchGrid *, int, int, int, int, unsigned,
                                                 const double *, double *, const double *,
                                                 const double *, hipStream_t);

}  // namespace mp
