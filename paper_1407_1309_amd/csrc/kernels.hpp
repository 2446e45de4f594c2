// kernels.hpp -- internal launcher interfaces between the C ABI (capi.hip)
// and the kernel translation units.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace mp {

// Arguments of one step through the staged (one launch per stage) path.
template <typename T> struct StagedArgs {
    Geom g;
    int n_iters;
    unsigned opts;
    const T *psi_n;     // step input (read by every pass under the limiter)
    T *psi_out;         // step output, distinct from psi_n
    const T *c[3];      // advector components (NULL beyond nd)
    const T *G;         // NULL: G == 1
    T *tmp[2];          // pass results, cell arrays
    T *faces[2][3];     // two sets of wall arrays
    T *bup, *bdn;       // limiter coefficients, cell arrays
};

template <typename T> hipError_t staged_step(const StagedArgs<T> &a, hipStream_t s);

// single stages of the staged path (arrays as in StagedArgs)
template <typename T>
hipError_t launch_donor(const Geom &g, const T *x, const T *const c[3], const T *G,
                        int mode, T *out, hipStream_t s);   // mode: 1 flux = advector, 2 Kahan
template <typename T>
hipError_t launch_pseudo(const Geom &g, unsigned opts, const T *x, const T *const c[3],
                         const T *G, T *const V[3], hipStream_t s);
template <typename T>
hipError_t launch_fct(const Geom &g, unsigned opts, const T *psi_n, const T *x,
                      const T *const V[3], const T *G, T *bup, T *bdn, T *const W[3],
                      hipStream_t s);

// Diagnostics: per-block partials into `part` (4 doubles per block, at most
// diag_max_blocks blocks), then one finalising block writing out[0..3] =
// (sum G psi, min, max, non-finite count as double).
int diag_max_blocks();
template <typename T>
hipError_t diag_launch(const T *psi, const T *G, int64_t N, double *part, double *out,
                       hipStream_t s);
// the final merge alone, over nparts partials written by another kernel
hipError_t diag_final_launch(const double *part, int nparts, double *out, hipStream_t s);

// out[0] = max over cells of sum_d max(|c_d| lo, |c_d| hi) / G where it is
// finite; out[1] = the number of cells where it is not.
template <typename T>
hipError_t courant_launch(const Geom &g, const T *c0, const T *c1, const T *c2, const T *G,
                          double *part, double *out, hipStream_t s);

// ---- fused 2-D kernel (all passes of a step in one launch) ---------------
struct Fused2DShape {
    int64_t n0, n1;      // rows (slow), columns (fast)
    int bc0, bc1;
    int tile_rows;       // rows per wavefront chunk; 0 = built-in default
};

// true if a fused kernel exists for this configuration
bool fused2d_supported(int nd, int n_iters, unsigned opts, int has_g, int bc0, int bc1);

// dpart != NULL: the launch also writes the diagnostics of the cells it
// stores, one partial per wave (5 doubles: sum, compensation, min, max,
// non-finite count) into dpart, and their number into *dparts; the final
// merge is diag_final_launch
template <typename T>
hipError_t fused2d_step(const Fused2DShape &sh, int n_iters, unsigned opts, const T *psi_n,
                        T *psi_out, const T *c0, const T *c1, const T *G, hipStream_t s,
                        double *dpart = nullptr, int *dparts = nullptr);
// the wave partials the fused 2-D step writes per 64-column strip chunk: an
// upper bound for chunks of at least min_rows rows
int64_t fused2d_max_parts(int64_t n0, int64_t n1, int n_iters, unsigned opts, int min_rows);

// ---- 3-D: a two-pass step without the limiter is one launch (step3d.hip;
// the donor-only step is k_donor3d in fused3d.hip).  With the limiter, or
// more passes, the same kernel forms each pass's raw pseudo-velocities (the
// first pass's input by its donor pass, a later pass's read from memory)
// and, with the limiter, the limiter coefficients; a cell kernel applies
// the limited velocities and the corrective pass (staged.hip:
// limcorr_launch, or launch_donor without the limiter).
// Modes of the 3-D step kernel: xin non-NULL: the pass input is read from
// xin (and c0..c2 are that pass's advector) instead of formed by the donor
// pass; v0 non-NULL (output mode): instead of the corrective pass, the raw
// pseudo-velocities v0, v1, v2 (walls, n_d + 1 along d) and, when y1 is
// non-NULL, the donor result y1 are written; bup / bdn non-NULL (output
// mode without xin): the limiter coefficients of the pass as well (cells).
template <typename T> struct Step3dOut {
    const T *xin = nullptr;
    T *y1 = nullptr, *v0 = nullptr, *v1 = nullptr, *v2 = nullptr;
    T *bup = nullptr, *bdn = nullptr;
};
bool step3d_supported(int nd, int n_iters, unsigned opts, const int64_t n[3]);
template <typename T>
hipError_t step3d_launch(const Geom &g, unsigned opts, const T *psi_n, T *psi_out, const T *c0,
                         const T *c1, const T *c2, const T *G, int tile_planes, hipStream_t s,
                         const Step3dOut<T> &vo = Step3dOut<T>());
// workspace of the 3-D step by passes: two cell fields, two sets of wall
// fields, the limiter coefficients
template <typename T> struct Fused3DWork {
    T *cell[2], *wall[2][3], *bup, *bdn;
};
bool fused3d_supported(int nd, int n_iters, unsigned opts, const int64_t n[3], const int bc[3]);
template <typename T>
hipError_t fused3d_step(const Geom &g, int n_iters, unsigned opts, const T *psi_n, T *psi_out,
                        const T *c0, const T *c1, const T *c2, const T *G, int tile_planes,
                        hipStream_t s, const Fused3DWork<T> &w);
// the limited corrective donor-cell pass of a pass from its input x, raw
// pseudo-velocities V and limiter coefficients: x -> y; W (entries NULL: not
// wanted) receives the limited velocities, the next pass's advector
template <typename T>
hipError_t limcorr_launch(const Geom &g, unsigned opts, const T *x, const T *const V[3],
                          const T *G, const T *bup, const T *bdn, T *y, T *const W[3],
                          hipStream_t s);

// ---- one corrective pass of a 2-D step in one launch (pass2d.hip) --------
// no third-order terms, any boundaries; x: previous pass's result, c0/c1:
// previous pass's advector, G: NULL for G = 1, y (distinct from x and
// psi_n): result; w0/w1 (both or neither): limited velocities for a
// following pass
// Optional records of a pass for the adjoint (written with w0 / w1): raw
// pseudo-velocities at the same walls, limiter coefficients of the cells.
template <typename T> struct PassRecord {
    T *v0 = nullptr, *v1 = nullptr, *bu = nullptr, *bd = nullptr;
    T *xd = nullptr;   // the folded donor pass's result (psi_n NULL launches only)
};
bool pass2d_supported(int nd, int n_iters, unsigned opts, int has_g, const int64_t n[3]);
// y may be NULL (no result needed); psi_n NULL: x is psi^n and the donor
// pass is folded in (the first corrective pass; rec.xd, when given,
// receives the donor result); tile_rows:
// rows per wavefront chunk (0 = built-in default)
template <typename T>
hipError_t pass2d_launch(const Geom &g, unsigned opts, const T *x, const T *c0, const T *c1,
                         const T *psi_n, const T *G, T *y, T *w0, T *w1, hipStream_t s,
                         const PassRecord<T> &rec = PassRecord<T>(), int tile_rows = 0);
// donor-cell pass of a 2-D grid, G = 1 (Kahan per opts); copy (optional)
// receives x unchanged
template <typename T>
hipError_t donor2d_launch(const Geom &g, unsigned opts, const T *x, const T *c0, const T *c1,
                          T *out, T *copy, hipStream_t s);

// ---- tangent-linear step (tlm.hip) ----------------------------------------
// workspace bytes of tlm_steps for the geometry and dtype
size_t tlm_workspace_bytes(const Geom &g, int f64, int has_g);
// n_steps steps of psi and its tangent dpsi (in place) along the advector
// tangent dc (entries NULL: zero); G constant; stage-by-stage kernels on
// dual numbers
template <typename T>
hipError_t tlm_steps(const Geom &g, int n_iters, unsigned opts, T *psi, T *dpsi, const T *G,
                     const T *const c[3], const T *const dc[3], int n_steps, void *ws,
                     hipStream_t s);

// ---- 1-D grid resident in LDS: all steps of a call in one launch --------
// two_fields: room for the oscillator pair (resident1d_osc)
bool resident1d_supported(int nd, int64_t n, int dtype_is_f64, int has_g, int two_fields = 0);
template <typename T>
hipError_t resident1d_steps(int64_t n, int bc, int n_iters, unsigned opts, T *psi, const T *c,
                            const T *G, int n_steps, hipStream_t s);
// n_steps trapezoidal steps of the translating oscillator pair (psi, phi)
template <typename T>
hipError_t resident1d_osc(int64_t n, int bc, int n_iters, unsigned opts, T *psi, T *phi,
                          const T *c, const T *G, double a, int n_steps, hipStream_t s);

// ---- batched fused 2-D: one launch over all tiles of all grids ---------
struct BatchGrid {
    int64_t n0, n1;
    int64_t off_psi, off_c0, off_c1;   // element offsets into packed buffers
    int tile_begin;                    // first tile of this grid in the work list
    int tiles_w;                       // tiles along columns
};

// tile_rows: rows per tile (the chunk length the table was built with);
// xcd_order != 0 numbers the tiles so that consecutive ones run on one XCD
template <typename T>
hipError_t fused2d_batched_step(const BatchGrid *grids_dev, int n_grids, int n_tiles, int bc,
                                int n_iters, unsigned opts, int tile_rows, int xcd_order,
                                const T *psi_n, T *psi_out, const T *c0, const T *c1,
                                hipStream_t s);

int fused2d_tile_rows();                             // default rows per batched tile
int fused2d_strip_cols(int n_iters, unsigned opts);  // output columns per strip

// ---- source terms and the oscillator coupling (rhs.hip) ----------------
template <typename T> hipError_t axpy_launch(T *y, const T *x, double a, int64_t n, hipStream_t s);
template <typename T>
hipError_t osc_couple_launch(T *psi, T *phi, double a, int implicit, int64_t n, hipStream_t s);

// ---- prognosed velocity and the shallow-water forcing (sw.hip) ----------
// c[d] = k[d] * wall mean of (1.5 u^n - 0.5 u^(n-1)), u = num / den (0 where
// den <= eps; num itself when den is NULL), for d < g.nd
template <typename T>
hipError_t vip_launch(const Geom &g, const T *const num[3], const T *den, const T *const nump[3],
                      const T *denp, double eps, const double k[3], T *const c[3], hipStream_t s);
// q[d] += dt/2 * (-grav h dh/dx_d); with save, first q_prev[d] = q[d], h_prev = h
template <typename T>
hipError_t sw_force_launch(const Geom &g, const T *h, T *h_prev, T *const q[3],
                           T *const q_prev[3], double grav, const double dx[3], double dt,
                           int save, hipStream_t s);
// One momentum component's save-phase forcing written to `out` (q kept at
// level n and copied to q_prev; h copied to h_prev when h_prev is not NULL).
template <typename T>
hipError_t sw_force1_launch(const Geom &g, int d, const T *h, T *h_prev, const T *q, T *q_prev,
                            T *out, double grav, const double dx[3], double dt, hipStream_t s);

}  // namespace mp
