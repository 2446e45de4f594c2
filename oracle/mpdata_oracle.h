/*
 * mpdata_oracle.h -- plain FP64 CPU reference of the MPDATA time step.
 *
 * TEST INFRASTRUCTURE ONLY.  This header and the library built from
 * mpdata_oracle.c are loaded by the test suite, by the package smoke check and
 * by the CPU-baseline leg of the benchmark.  The product library (HIP) never
 * includes, links or calls anything here, and this code includes nothing of
 * the product.
 *
 * Conventions (shared by meaning, not by code, with the product ABI):
 *   - arrays are C-contiguous, last dimension fastest (row-major);
 *   - a grid of ndims dimensions has extents n[0..ndims-1]; the oracle pads
 *     unused trailing dimensions with extent 1;
 *   - psi and G are cell arrays of n[0]*n[1]*n[2] values;
 *   - the advector component c_d is a face array with n[d]+1 entries along
 *     dimension d (entry f is the wall between cells f-1 and f) and the cell
 *     extents along the other dimensions;
 *   - c_d holds the G-weighted Courant number G*u_d*dt/dx_d.
 */
#ifndef MPDATA_ORACLE_H
#define MPDATA_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_BC_PERIODIC = 0, ORC_BC_OPEN = 1 };
/* KAHAN: every donor-cell pass sums its update terms with Kahan's
 * compensated summation (the library default the paper describes in
 * Sect. 3.1.1) instead of straightforwardly. */
/* ABS: |psi| replaces psi in every psi-fraction of the pseudo-velocity
 * (variable-sign fields, Sect. 3.1.5); not combinable with IGA, forward
 * only (orc_adjoint rejects it). */
/* DFL: the pseudo-velocity gains the divergent-flow term -c/(2 Gb) * div,
 * div the mean over the wall's two cells of sum_o (c_o(hi) - c_o(lo)) of
 * the pass's advector (Sect. 3.1.3).  Forward only (orc_adjoint rejects it). */
enum { ORC_OPT_FCT = 1u << 0, ORC_OPT_IGA = 1u << 1, ORC_OPT_TOT = 1u << 2,
       ORC_OPT_ABS = 1u << 3, ORC_OPT_DFL = 1u << 4, ORC_OPT_KAHAN = 1u << 5 };

/* Advance psi (in place) by n_steps MPDATA steps.  g may be NULL (G = 1).
 * c[d] must be non-NULL for d < ndims.  Returns 0, or -1 on bad arguments. */
int orc_step(int ndims, const long n[3], const int bc[3], int n_iters,
             unsigned opts, double *psi, const double *g,
             const double *c0, const double *c1, const double *c2,
             long n_steps);

/* Sum of G*psi (Neumaier-compensated, row-major order), min and max of psi,
 * and the count of non-finite psi values. */
int orc_diag(int ndims, const long n[3], const double *psi, const double *g,
             double out_sum_min_max[3], long *n_nonfinite);

/* max over cells of sum_d max(|c_d| on the two d-walls of the cell) / G. */
int orc_courant_max(int ndims, const long n[3], const int bc[3],
                    const double *g, const double *c0, const double *c1,
                    const double *c2, double *out);

/* Reverse-mode gradient of J(psi_T) through n_steps steps started from psi0.
 * lambda_T = dJ/dpsi_T (cell array).  Outputs are overwritten:
 * grad_psi0 (cells) and grad_c[d] (faces, d < ndims).  The reverse sweep
 * keeps a checkpoint every ckpt_every steps and recomputes in between.
 * Derivative conventions at non-differentiable points are documented in the
 * source.  Returns 0 or -1. */
int orc_adjoint(int ndims, const long n[3], const int bc[3], int n_iters,
                unsigned opts, const double *psi0, const double *g,
                const double *c0, const double *c1, const double *c2,
                long n_steps, long ckpt_every, const double *lambda_T,
                double *grad_psi0, double *grad_c0, double *grad_c1,
                double *grad_c2);

/* Threads the stage loops of orc_step use: 1, or the OpenMP thread count
 * when the file is built with -fopenmp (the multi-core CPU baseline). */
int orc_threads(void);

#ifdef __cplusplus
}
#endif
#endif
