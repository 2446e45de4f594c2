// fused2d_f32.hip -- FP32 instances of the fused 2-D step (fused2d.hpp).
#include "fused2d.hpp"

namespace mp {

template hipError_t fused2d_step<float>(const Fused2DShape &, int, unsigned, const float *, float *,
                                        const float *, const float *, const float *, hipStream_t,
                                        double *, int *);
template hipError_t fused2d_batched_step<float>(const BatchGrid *, int, int, int, int, unsigned,
                                                int, int, const float *, float *, const float *,
                                                const float *, hipStream_t);

}  // namespace mp
