// fused2d_f64.hip -- FP64 instances of the fused 2-D step (fused2d.hpp) and
// the host-side queries of what the fused kernel covers.
#include "fused2d.hpp"

namespace mp {

bool fused2d_supported(int nd, int n_iters, unsigned opts, int has_g, int bc0, int bc1)
{
    if (nd != 2 || has_g || bc0 != BC_PERIODIC || bc1 != BC_PERIODIC) return false;
    if (opts & ~(OPT_FCT | OPT_KAHAN | OPT_ABS)) return false;   // tot / iga / dfl: staged path
    if ((opts & OPT_ABS) && n_iters > 3) return false;
    return n_iters >= 1 && n_iters <= 4;
}

int fused2d_tile_rows() { return 64; }

int64_t fused2d_max_parts(int64_t n0, int64_t n1, int n_iters, unsigned opts, int min_rows)
{
    return cdiv(n1, fused2d_strip_cols(n_iters, opts)) * cdiv(n0, min_rows);
}

int fused2d_strip_cols(int n_iters, unsigned opts)
{
    int np = n_iters - 1;
    int h = 1 + ((opts & OPT_FCT) ? 2 : 1) * np;
    return WAVE - 2 * h;
}

template hipError_t fused2d_step<double>(const Fused2DShape &, int, unsigned, const double *,
                                         double *, const double *, const double *, const double *,
                                         hipStream_t, double *, int *);
template hipError_t fused2d_batched_step<double>(const BatchGrid *, int, int, int, int, unsigned,
                                                 int, int, const double *, double *,
                                                 const double *, const double *, hipStream_t);

}  // namespace mp
