/*
 * mpdata.h -- C ABI of libmpdata, the MI355X (gfx950) MPDATA time step.
 *
 * The step solves the homogeneous generalised transport equation in the form
 *     d(psi)/dt + (1/G) div(G u psi) = 0              (paper eq. gte_final)
 * with G constant in time, on the staggered Arakawa-C grid of Sect. 2.3:
 * psi and G live at cell centres, the advector (G-weighted Courant number
 * GC = G u dt/dx, Sect. 3.1.1) lives on the cell walls.
 *
 * One step is a donor-cell pass (eqs. upstream and F) followed by n_iters-1
 * corrective passes that advect the previous pass's result with the
 * antidiffusive pseudo-velocity (eq. adf_vel and its multi-dimensional
 * form), optionally with the third-order terms (Sect. 3.1.2), the infinite-
 * gauge variant (Sect. 3.1.5) and the non-oscillatory limiter (Sect. 3.1.4).
 * Summation is the "straightforward" one of Sect. 3.1.1.
 *
 * Memory and ownership
 *   - Every array argument is a DEVICE pointer to C-contiguous (row-major,
 *     last dimension fastest, Sect. 3.2) data of the plan's dtype, owned by
 *     the caller.  The library never allocates device memory: scratch space
 *     comes from the caller's workspace (mpdata_workspace_bytes).
 *   - psi and G have the plan's shape (n0[, n1[, n2]]).
 *   - Advector component c_d has the plan's shape with n_d + 1 entries along
 *     dimension d; entry f is the wall between cells f-1 and f.  With
 *     periodic boundaries wall n_d is the same wall as wall 0 and is never
 *     read; with open boundaries walls 0 and n_d are the domain edges.
 *   - g == NULL means G == 1.
 *
 * Boundaries (Sect. 2.2): periodic wraps every array; open gives every cell
 * array a zero-gradient halo and every wall array copies its edge wall.
 *
 * Execution and errors
 *   - Calls enqueue work on the plan's HIP stream and return without
 *     waiting, except mpdata_diag, mpdata_courant_max and mpdata_adv_adj,
 *     which wait for their results.
 *   - Every call returns MPDATA_OK or a negative status; nothing throws.
 *     mpdata_last_error() gives the message of the calling thread's last
 *     failure.  A device fault surfaces at the next synchronising call.
 *   - A plan is not thread-safe; calls on one plan must be serialised.
 */
#ifndef MPDATA_H
#define MPDATA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum mpdata_status {
    MPDATA_OK = 0,
    MPDATA_EINVAL = -1,       /* bad argument (null pointer, shape, flag)   */
    MPDATA_EWORKSPACE = -2,   /* workspace missing, too small or unaligned  */
    MPDATA_EHIP = -3,         /* a HIP runtime call or launch failed        */
    MPDATA_ENONFINITE = -4,   /* mpdata_diag found NaN or Inf values        */
    MPDATA_ECANCELLED = -5,   /* stopped by the plan's cancel flag          */
    MPDATA_EUNSUPPORTED = -6  /* valid but not provided (see mpdata_init)   */
};

/* option bits (Sect. 3.4) */
enum {
    MPDATA_OPT_FCT = 1u << 0, /* non-oscillatory limiter, Sect. 3.1.4       */
    MPDATA_OPT_IGA = 1u << 1, /* infinite gauge, Sect. 3.1.5                */
    MPDATA_OPT_TOT = 1u << 2, /* third-order terms, Sect. 3.1.2             */
    /* |psi| replaces psi in every psi-fraction of the pseudo-velocity, for
     * variable-sign fields (Sect. 3.1.5).  Not combinable with IGA (the other
     * variable-sign option: MPDATA_EINVAL); mpdata_adv_adj rejects it
     * (MPDATA_EUNSUPPORTED). */
    MPDATA_OPT_ABS = 1u << 3,
    /* divergent-flow term (Sect. 3.1.3): the pseudo-velocity at a wall gains
     * -c/(2 Gb) times the mean over the wall's two cells of the pass
     * advector's divergence sum_o (c_o(hi) - c_o(lo)).  Staged and resident
     * 1-D kernels; mpdata_adv_adj rejects it (MPDATA_EUNSUPPORTED). */
    MPDATA_OPT_DFL = 1u << 4,
    /* Kahan-compensated donor-cell update (Sect. 3.1.1): every donor-cell pass
     * forms psi + sum_d -(F_d(i+1/2) - F_d(i-1/2)) / G with Kahan's
     * compensated summation, dimensions in increasing order, instead of
     * psi - [sum_d (F_d(i+1/2) - F_d(i-1/2))] / G.  Round-off only; the
     * adjoint differentiates the exact sum. */
    MPDATA_OPT_KAHAN = 1u << 5
};

enum { MPDATA_BC_PERIODIC = 0, MPDATA_BC_OPEN = 1 };
enum { MPDATA_F32 = 0, MPDATA_F64 = 1 };

/* kernel selection for mpdata_set_kernel */
enum {
    MPDATA_KERNEL_AUTO = 0,    /* fused kernel where one exists, else the 2-D
                                  single-pass kernel, else staged           */
    MPDATA_KERNEL_STAGED = 1,  /* one launch per stage (cross-check path)    */
    MPDATA_KERNEL_FUSED = 2,   /* all passes of a step in one launch         */
    MPDATA_KERNEL_PASS = 3     /* 2-D: one launch per corrective pass (the
                                  kernel the adjoint records with)          */
};

typedef struct mpdata_desc {
    int n_dims;           /* 1, 2 or 3                                       */
    int64_t shape[3];     /* cells per dimension; entries >= n_dims ignored  */
    int dtype;            /* MPDATA_F32 or MPDATA_F64                         */
    int n_iters;          /* passes per step incl. the donor pass, 1..8      */
    uint32_t opts;        /* MPDATA_OPT_* bits                               */
    int bc[3];            /* MPDATA_BC_* per dimension                       */
    int has_g;            /* nonzero if steps will pass a G array            */
} mpdata_desc;

typedef struct mpdata_plan mpdata_plan; /* opaque host object */

/* Bytes of device workspace a plan for *desc needs (0 on invalid desc). */
size_t mpdata_workspace_bytes(const mpdata_desc *desc);

/* Validate *desc and create a plan bound to `workspace` (device memory of at
 * least mpdata_workspace_bytes(desc) bytes, 256-byte aligned, owned by the
 * caller and kept alive until mpdata_destroy) and `hip_stream` (a
 * hipStream_t; NULL = the default stream).
 * Rejects: n_dims outside 1..3, a shape < 1 (< 3 along a periodic dimension)
 * or >= 2^30 (cells and walls of a dimension are indexed in 32 bits with
 * halo offsets), more than 2^40 cells,
 * n_iters outside 1..8, unknown option bits, bc or dtype values
 * (MPDATA_EINVAL); the infinite gauge with n_iters > 2 (MPDATA_EUNSUPPORTED:
 * its pseudo-velocity is a flux, not a Courant number, so it cannot drive a
 * third pass). */
int mpdata_init(const mpdata_desc *desc, void *workspace, size_t ws_bytes,
                void *hip_stream, mpdata_plan **out);

/* Re-bind the plan to another HIP stream (NULL = the default stream). */
int mpdata_set_stream(mpdata_plan *plan, void *hip_stream);

/* Choose the step kernel (MPDATA_KERNEL_*).  FUSED returns
 * MPDATA_EUNSUPPORTED when no fused kernel covers the plan, PASS when the
 * plan is not 2-D with n_iters >= 2.  FUSED and PASS give the same bits
 * where both apply (2-D periodic, G = 1, no tot / iga / dfl). */
int mpdata_set_kernel(mpdata_plan *plan, int kernel);

/* Rows per wavefront chunk of the fused 2-D kernel and of the 2-D
 * single-pass kernel (0 = built-in default).
 * Results do not depend on it (bit for bit); only the speed does. */
int mpdata_set_tile_rows(mpdata_plan *plan, int rows);

/* Autotuner: time the fused step on the caller's inputs for a set of chunk
 * lengths (psi is read, not modified; results go to workspace) and keep the
 * fastest in the plan.  *out_tile_rows receives the choice (0 when the plan
 * runs the staged path, which has nothing to tune).  Waits for completion. */
int mpdata_autotune(mpdata_plan *plan, const void *psi, const void *g,
                    const void *c0, const void *c1, const void *c2,
                    int *out_tile_rows);

/* Advance psi (in place) by n_steps steps (n_steps >= 0) with the advector
 * c0..c2 held fixed over the call (the caller passes the advector at the
 * intermediate time level n+1/2, Sect. 3.1.1).  c_d must be non-NULL for
 * d < n_dims and NULL otherwise; g must be non-NULL iff the plan has_g.
 * Successive calls continue the integration exactly (resumable like the
 * paper's advance()). */
int mpdata_step(mpdata_plan *plan, void *psi, const void *g, const void *c0,
                const void *c1, const void *c2, int n_steps);

/* Stop flag for the step loop of mpdata_step (the paper's solvers stop
 * after the current step when a flag is raised: Sect. 3.2, public
 * methods).  flag is a host address (plain or pinned memory, owned by the
 * caller, read with volatile loads; NULL removes it).  While a flag is set
 * on the plan, mpdata_step waits for each step to finish before it reads
 * the flag and launches the next one, so a flag raised from another thread
 * or a signal handler stops the run after the step in progress: the call
 * then returns MPDATA_ECANCELLED with psi holding the last completed step.
 * The 1-D kernel that runs every step of a call in one launch reads the
 * flag only before that launch. */
int mpdata_set_cancel_flag(mpdata_plan *plan, const volatile int *flag);

/* Number of steps the last mpdata_step call on this plan completed
 * (n_steps unless it was cancelled or failed). */
int mpdata_steps_done(const mpdata_plan *plan, int64_t *out);

/* One step of the inhomogeneous transport equation (Sect. 4.1):
 * psi <- ADV(psi + a_pre * r_pre) + a_post * r_post, ADV one mpdata_step.
 * r_pre / r_post are cell fields of the plan's dtype (either may be NULL:
 * that term is skipped).  The paper's schemes: euler_a (r_post = R^n,
 * a_post = dt), euler_b (r_pre = R^n, a_pre = dt), trapez (r_pre = R^n,
 * a_pre = dt/2, r_post = R^{n+1}, a_post = dt/2; a forcing that depends on
 * psi^{n+1} is applied by the caller after the call instead). */
int mpdata_step_rhs(mpdata_plan *plan, void *psi, const void *g, const void *c0,
                    const void *c1, const void *c2, const void *r_pre, double a_pre,
                    const void *r_post, double a_post);

/* n_steps steps of the translating oscillator (Sect. 4.3):
 * d psi/dt + div(u psi) = omega phi, d phi/dt + div(u phi) = -omega psi with
 * the trapezoidal rule, a = dt * omega / 2 (eqs. osc_disc, trapez_osc,
 * final_osc): psi* = ADV(psi + a phi), phi* = ADV(phi - a psi), then
 * psi = (psi* + a phi*) / (1 + a^2), phi = (phi* - a psi*) / (1 + a^2).
 * psi and phi are distinct cell buffers, updated in place.  (The printed
 * trapez_osc has phi^n in the second argument where psi^n belongs.) */
int mpdata_osc_step(mpdata_plan *plan, void *psi, void *phi, const void *g,
                    const void *c0, const void *c1, const void *c2, double a,
                    int n_steps);

/* Advector at n+1/2 from prognosed velocity (Sect. 5.1-5.2).  The cell
 * velocity component d is num[d] / den, set to 0 where den <= eps (den ==
 * NULL: num[d] is the velocity itself; den and den_prev are both given or
 * both NULL).  It is extrapolated in time from levels n (num, den) and n-1
 * (num_prev, den_prev) as 1.5 u^n - 0.5 u^(n-1), averaged over the two
 * cells of each dimension-d wall through the boundary map (open: an edge
 * wall takes its cell's value), and multiplied by dt / dx[d].
 * num, num_prev: arrays of n_dims cell-array pointers; c: n_dims wall-array
 * pointers (written, distinct from every input).  dt > 0, dx[d] > 0 for
 * d < n_dims, eps >= 0, all finite (else MPDATA_EINVAL).  The infinite
 * gauge of the advected fields does not enter here; G is not used. */
int mpdata_vip_advector(mpdata_plan *plan, const void *const num[3], const void *den,
                        const void *const num_prev[3], const void *den_prev, double dt,
                        const double dx[3], double eps, void *const c[3]);

/* n_steps steps of the shallow-water system (eqs. shw1d, shw2d; Sect.
 * 5.3-5.4): depth h and momenta q[d] = u_d h, gravity grav.  Each step
 *   c = mpdata_vip_advector(q, h, q_prev, h_prev)        (den = h)
 *   q_prev = q, h_prev = h
 *   q[d] += dt/2 R_d(h),  R_d(h) = -grav h dh/dx_d (centred difference
 *                                   through the boundary map)
 *   h = ADV(h),  q[d] = ADV(q[d])   (the plan's step, advector c)
 *   q[d] += dt/2 R_d(h)             (forcing at n+1 from the new depth)
 * i.e. the trapezoidal source-term scheme with h advected first.  h, q,
 * h_prev, q_prev hold levels n and n-1 on entry and n + n_steps and
 * n + n_steps - 1 on return; before the first step of a run the previous
 * level is a copy of the current one.  c (n_dims wall arrays) is scratch
 * that holds the last step's advector on return.  All buffers distinct
 * (else MPDATA_EINVAL).  The plan must be made without G
 * (MPDATA_EUNSUPPORTED: prognosed velocity is defined for G = 1); its
 * options and n_iters apply to every advection (the paper's example uses
 * iga + fct + dfl or abs + fct, two passes). */
int mpdata_sw_step(mpdata_plan *plan, void *h, void *const q[3], void *h_prev,
                   void *const q_prev[3], void *const c[3], double dt, const double dx[3],
                   double grav, double eps, int n_steps);

/* Diagnostics of every step call's result, formed by the step itself.  With
 * on != 0, each later mpdata_step call on the plan also forms the
 * diagnostics of mpdata_diag (sum of G*psi, min, max, non-finite count) of
 * the field it leaves in psi, and mpdata_step_diag returns those of the last
 * call (waits for them).  The fused 2-D step accumulates them in its last
 * launch while it stores each cell (one partial per wavefront, then one
 * small merge launch: no second read of psi); the other kernels are
 * followed by a diagnostics pass over psi.  mpdata_step_diag returns
 * MPDATA_EINVAL when no step call has formed them since they were switched
 * on, and MPDATA_ENONFINITE (after filling the outputs) when the field holds
 * NaN or Inf values.  The conserved sum is the flux form's invariant
 * (Sect. 1); the non-finite count is the run-time counterpart of the NaN
 * checks of Sect. 2.4.  Switching off (on = 0) drops the last result. */
int mpdata_set_step_diag(mpdata_plan *plan, int on);
int mpdata_step_diag(mpdata_plan *plan, double out_sum_min_max[3], int64_t *n_nonfinite);

/* Diagnostics of psi (waits for the result): out[0] = sum of G*psi over the
 * finite cells (FP64, compensated), out[1] = min, out[2] = max of the finite
 * values, *n_nonfinite = number of NaN/Inf cells.  Returns MPDATA_ENONFINITE
 * (after filling the outputs) when *n_nonfinite > 0.  g may be NULL.
 * The sum is the conserved quantity of the flux form (Sect. 1: the scheme is
 * conservative); the non-finite count is the run-time counterpart of the
 * paper's NaN checks in debug builds (Sect. 2.4).  Every step kernel lets a
 * NaN or infinity in psi or in the advector reach psi of the next step
 * (the donor-cell flux is formed as a product with the advector), so a
 * failed run shows here. */
int mpdata_diag(mpdata_plan *plan, const void *psi, const void *g,
                double out_sum_min_max[3], int64_t *n_nonfinite);

/* mpdata_diag for callers that cannot allocate device memory or hold a
 * plan's workspace (code under HIP stream capture, tight serving loops,
 * harnesses that forbid allocation): the same kernels and outputs, with the
 * block partials and the result in a fixed device array of the library
 * (41 KB per device, kept until the process ends); no plan, no workspace,
 * no allocation.  psi (and g, or NULL) are device arrays of n_cells values
 * of `dtype` (MPDATA_F32 / MPDATA_F64), 1 <= n_cells <= 2^40 (else
 * MPDATA_EINVAL); work is enqueued on hip_stream (a hipStream_t, NULL =
 * default) and the call waits for the result.  Returns MPDATA_ENONFINITE
 * (after filling the outputs) when *n_nonfinite > 0.  Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (from several
 * threads or streams) race and must be serialised by the caller. */
int mpdata_diag_noalloc(int dtype, int64_t n_cells, const void *psi, const void *g,
                        void *hip_stream, double out_sum_min_max[3], int64_t *n_nonfinite);

/* max over cells of sum_d max(|c_d| on the two d-walls of the cell) / G
 * (waits for the result).  A value above 1 means the donor-cell pass can
 * empty a cell, so sign preservation (Sect. 1) is no longer guaranteed.
 * Cells whose walls or G hold a NaN or infinity are left out of the
 * maximum and make the call return MPDATA_ENONFINITE (after *out is
 * written): the input check before a run. */
int mpdata_courant_max(mpdata_plan *plan, const void *g, const void *c0,
                       const void *c1, const void *c2, double *out);

/* Gradient of a scalar J(psi_T), psi_T = n_steps steps from psi0, with
 * respect to psi0 and the advector (reverse mode of the full nonlinear step:
 * pseudo-velocity, cross/third-order terms and limiter included; G is held
 * constant).  lambda_T = dJ/dpsi_T.  grad_psi0 and grad_c0..grad_c2
 * (NULL for d >= n_dims) are overwritten.  The forward trajectory is kept
 * only every ckpt_every steps (1 <= ckpt_every <= n_steps) and recomputed in
 * between, one segment at a time, keeping that segment's states and per-pass
 * records; memory for the checkpoints and the segment comes from the plan's
 * workspace, sized by mpdata_adj_workspace_bytes (it grows with ckpt_every
 * as about 1 + 7 (n_iters - 1) cell fields per step of a segment in 2-D,
 * with the limiter).  Waits for completion.  Periodic walls:
 * the gradient of the shared wall 0 / wall n_d is returned in entry 0, and
 * entry n_d is zero.
 * Derivatives at non-differentiable points: d[u]+/du = 1 only for u > 0,
 * d[u]-/du = 1 only for u < 0; a max/min passes its derivative to the first
 * argument attaining it in the order the method lists its arguments; the
 * zero-denominator and no-flux branches of the fractions and limiter
 * coefficients have zero derivative. */
int mpdata_adv_adj(mpdata_plan *plan, const void *psi0, const void *g,
                   const void *c0, const void *c1, const void *c2,
                   int n_steps, int ckpt_every, const void *lambda_T,
                   void *grad_psi0, void *grad_c0, void *grad_c1,
                   void *grad_c2);

/* Tangent-linear steps (forward-mode derivative of the full nonlinear step,
 * the directional counterpart of mpdata_adv_adj): psi advances by n_steps
 * steps as in mpdata_step and dpsi becomes the derivative of the result
 * along the direction (dpsi, dc0..dc2) of (psi0, c0..c2); G is constant.
 * psi and dpsi are distinct cell buffers updated in place; dc_d may be
 * NULL (zero tangent), else it has c_d's layout.  Derivatives at
 * non-differentiable points follow the conventions of mpdata_adv_adj, so
 * <tangent(v), w> = <v, adjoint(w)> holds to rounding.  Runs the
 * stage-by-stage kernels on (value, derivative) pairs held in the plan's
 * workspace, which must have mpdata_tlm_workspace_bytes bytes
 * (MPDATA_EWORKSPACE otherwise). */
int mpdata_tlm_step(mpdata_plan *plan, void *psi, void *dpsi, const void *g,
                    const void *c0, const void *c1, const void *c2, const void *dc0,
                    const void *dc1, const void *dc2, int n_steps);

/* Workspace bytes mpdata_tlm_step needs (0 on an invalid desc). */
size_t mpdata_tlm_workspace_bytes(const mpdata_desc *desc);

/* Workspace bytes mpdata_adv_adj needs for n_steps / ckpt_every (0 on bad
 * arguments); a plan meant for the adjoint must be created with at least
 * this much workspace. */
size_t mpdata_adj_workspace_bytes(const mpdata_desc *desc, int n_steps,
                                  int ckpt_every);

/* ---------------------------------------------------------------------- */
/* Batched step: many independent 2-D grids (ensemble members, tracers)    */
/* advanced together, one launch per step over every tile of every grid.   */
/* ---------------------------------------------------------------------- */

/* shapes[2*i], shapes[2*i+1] = (n0, n1) of grid i.  Grids are packed one
 * after another in three device buffers: psi (sum n0*n1 values), c0 (sum
 * (n0+1)*n1) and c1 (sum n0*(n1+1)), each grid C-contiguous, in order.
 * Every grid shares dtype, n_iters, opts and one boundary type for both
 * dimensions.  The workspace must hold mpdata_batched_workspace_bytes. */
size_t mpdata_batched_workspace_bytes(int n_grids, const int64_t *shapes,
                                      int dtype, int n_iters, uint32_t opts,
                                      int bc);
int mpdata_batched_init(int n_grids, const int64_t *shapes, int dtype,
                        int n_iters, uint32_t opts, int bc, void *workspace,
                        size_t ws_bytes, void *hip_stream, mpdata_plan **out);

/* Advance every grid by n_steps steps (in place).  With use_graph != 0 the
 * n_steps launches are captured once into a HIP graph per (buffers,
 * n_steps) and replayed; otherwise they are launched directly. */
int mpdata_step_batched(mpdata_plan *plan, void *psi_packed,
                        const void *c0_packed, const void *c1_packed,
                        int n_steps, int use_graph);

/* Tiling of the batched launch: chunks of tile_rows rows (0 = the default,
 * 64) and the tile order (xcd_order = 0: grid by grid; 1: numbered so that
 * consecutive tiles, which share halo columns, run on the same XCD).
 * Results do not depend on either (bit for bit).  Rebuilds the work list in
 * the workspace (waits for the plan's stream) and drops cached graphs. */
int mpdata_set_batched_tiling(mpdata_plan *plan, int tile_rows, int xcd_order);

/* Batched autotuner: times one batched step on the caller's buffers for
 * every candidate chunk length (16..256 rows) and both tile orders (psi is
 * read, not modified; the result goes to workspace), keeps the fastest and
 * returns it.  Waits for completion. */
int mpdata_autotune_batched(mpdata_plan *plan, const void *psi_packed,
                            const void *c0_packed, const void *c1_packed,
                            int *out_tile_rows, int *out_xcd_order);

/* Same update, one ordinary launch sequence per grid (the baseline the
 * batched launch is measured against). */
int mpdata_step_per_grid(mpdata_plan *plan, void *psi_packed,
                         const void *c0_packed, const void *c1_packed,
                         int n_steps);

/* Timing of the step kernels, for roofline accounting.  mpdata_timing(plan,
 * m) with m > 0 clears earlier records and times the next m step launches
 * made by mpdata_step (the fused 2-D kernel, the 3-D donor + corrective
 * pair, the resident 1-D kernel -- one launch for all steps of a call -- or
 * the staged kernel sequence): a HIP event on the plan's stream before the
 * first of them and one after the m-th (or, if fewer were made, one
 * recorded by mpdata_timing_read), with no event in between, so time
 * between the launches of separate mpdata_step calls is included.  m = 0
 * switches timing off.
 * Timing does not change results.  mpdata_timing_read waits for the
 * recorded launches and returns the elapsed milliseconds of the window,
 * the number of launches in it and the name of what was launched (a static
 * string; kernel may be NULL).  Single-grid plans only. */
int mpdata_timing(mpdata_plan *plan, int max_launches);
int mpdata_timing_read(mpdata_plan *plan, double *total_ms, int *launches,
                       const char **kernel);

void mpdata_destroy(mpdata_plan *plan);

/* Message of the calling thread's last failed call ("" if none). */
const char *mpdata_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
