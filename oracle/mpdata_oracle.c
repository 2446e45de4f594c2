/*
 * mpdata_oracle.c -- plain, slow, FP64 CPU reference of the MPDATA time step
 * (libmpdata++ 0.1 paper, Sect. 3.1).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark.  It shares no code with the HIP library.
 *
 * Organisation: every stage of the method is one loop over the whole grid
 * that reads full arrays through a boundary map and writes a full array, in
 * the order the method states (donor-cell pass, then per corrective pass the
 * pseudo-velocity, the optional limiter and the corrective donor-cell pass).
 * No blocking, no fusion, no reordering.
 *
 * Readings where the paper only cites the formulae (frozen; the GPU path
 * obeys the same ones):
 *   - boundaries (Sect. 2.2, "cyclic" / "open"): every array, including the
 *     intermediate ones (pseudo-velocities, limiter coefficients), is read
 *     through the same map: periodic wraps cell q to q mod n and wall f to
 *     f mod n (so wall n is wall 0); open clamps cell q into [0, n-1] and
 *     wall f into [0, n];
 *   - psi-fractions n/d are 0 when d == 0, with no epsilon; under the infinite
 *     gauge they become n/m with m the number of values summed in d;
 *   - multi-dimensional cross terms, third-order terms and the limiter follow
 *     the forms written next to each function below;
 *   - options beyond the basic scheme: Kahan-compensated donor-cell updates
 *     (Sect. 3.1.1), the divergent-flow term (Sect. 3.1.3, its form derived
 *     from the donor-cell truncation error, see pseudo_velocity) and |psi| in
 *     the psi-fractions (abs, Sect. 3.1.5).
 */
#include "mpdata_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* The outermost loop of each stage (over dimension 0) may be shared among
 * threads: built with -fopenmp this file is the multi-core CPU baseline.
 * Every iteration writes its own cells or walls only and reads arrays that
 * the stage does not write, so any thread count gives the same bits. */
#define ROWS_IN_PARALLEL _Pragma("omp parallel for schedule(static)")

typedef struct {
    int ndims;
    long n[3];
    int bc[3];
    int iga, tot, fct, kahan, abs, dfl;
} grid_t;

/* ------------------------------------------------------------------------ */
/* boundary map (Sect. 2.2 boundary conditions; Sect. 2.3 grid)             */
/* ------------------------------------------------------------------------ */

static long map_cell(const grid_t *g, int d, long q)
{
    long n = g->n[d];
    if (g->bc[d] == ORC_BC_PERIODIC) {
        q %= n;
        if (q < 0) q += n;
        return q;
    }
    if (q < 0) return 0;
    if (q > n - 1) return n - 1;
    return q;
}

static long map_wall(const grid_t *g, int d, long f)
{
    long n = g->n[d];
    if (g->bc[d] == ORC_BC_PERIODIC) {
        f %= n;
        if (f < 0) f += n;
        return f;
    }
    if (f < 0) return 0;
    if (f > n) return n;
    return f;
}

static long cells(const grid_t *g) { return g->n[0] * g->n[1] * g->n[2]; }

static long walls(const grid_t *g, int d)
{
    long e[3] = {g->n[0], g->n[1], g->n[2]};
    e[d] += 1;
    return e[0] * e[1] * e[2];
}

/* flat index of the cell at p (after the boundary map) */
static long cidx(const grid_t *g, const long p[3])
{
    long i = map_cell(g, 0, p[0]), j = map_cell(g, 1, p[1]),
         k = map_cell(g, 2, p[2]);
    return (i * g->n[1] + j) * g->n[2] + k;
}

/* flat index of the wall p of a dimension-d wall array; p[d] is the wall
 * index (wall f separates cells f-1 and f), the other entries are cells. */
static long widx(const grid_t *g, int d, const long p[3])
{
    long e[3] = {g->n[0], g->n[1], g->n[2]};
    long q[3];
    e[d] += 1;
    for (int t = 0; t < 3; t++)
        q[t] = (t == d) ? map_wall(g, t, p[t]) : map_cell(g, t, p[t]);
    return (q[0] * e[1] + q[1]) * e[2] + q[2];
}

static double at(const grid_t *g, const double *a, const long p[3])
{
    return a[cidx(g, p)];
}

static double gat(const grid_t *g, const double *G, const long p[3])
{
    return G ? G[cidx(g, p)] : 1.0;
}

static double wat(const grid_t *g, int d, const double *a, const long p[3])
{
    return a[widx(g, d, p)];
}

/* p shifted by s along dimension d */
static void sh(long out[3], const long p[3], int d, long s)
{
    out[0] = p[0];
    out[1] = p[1];
    out[2] = p[2];
    out[d] += s;
}

/* p shifted by s along d and t along e */
static void sh2(long out[3], const long p[3], int d, long s, int e, long t)
{
    sh(out, p, d, s);
    out[e] += t;
}

static double pos(double u) { return u > 0.0 ? u : 0.0; } /* [u]^+ */
static double neg(double u) { return u < 0.0 ? u : 0.0; } /* [u]^- */

/* psi-fraction of the pseudo-velocity formulae (eq. adf_vel): num/den, or 0
 * for a zero denominator; the infinite-gauge variant (Sect. 3.1.5) replaces
 * the denominator by the count m of summed values. */
static double frac(const grid_t *g, double num, double den, double m)
{
    if (g->iga) return num / m;
    return den == 0.0 ? 0.0 : num / den;
}

/* psi value entering a psi-fraction: |psi| under the abs option (Sect. 3.1.5,
 * variable-sign fields), psi otherwise */
static double xat(const grid_t *g, const double *x, const long p[3])
{
    double v = at(g, x, p);
    return g->abs ? fabs(v) : v;
}

/* ------------------------------------------------------------------------ */
/* donor-cell pass, eq. (upstream) with the flux function eq. (F)            */
/* ------------------------------------------------------------------------ */

/* flux through wall p of dimension d: [c]^+ x(left) + [c]^- x(right) */
static double donor_flux(const grid_t *g, int d, const double *x,
                         const double *c, const long p[3])
{
    long L[3], R[3];
    sh(L, p, d, -1);
    sh(R, p, d, 0);
    double u = wat(g, d, c, p);
    return pos(u) * at(g, x, L) + neg(u) * at(g, x, R);
}

/* out(i) = x(i) - [sum_d (F_d(i+1/2) - F_d(i-1/2))] / G(i), dimensions summed
 * in increasing order.  When iga_flux is set the corrective-pass flux is the
 * pseudo-velocity itself (infinite-gauge limit, F = V).
 * With the Kahan option (Sect. 3.1.1) the update is the compensated sum of
 * x(i) and the terms -(F_d(i+1/2) - F_d(i-1/2)) / G(i), d increasing:
 * s = x(i), c = 0; per term t: y = t - c, u = s + y, c = (u - s) - y, s = u. */
static void donor_pass(const grid_t *g, const double *x, double *const c[3],
                       const double *G, int iga_flux, double *out)
{
    ROWS_IN_PARALLEL
    for (long i0 = 0; i0 < g->n[0]; i0++) {
        long p[3] = {i0, 0, 0};
        for (p[1] = 0; p[1] < g->n[1]; p[1]++)
            for (p[2] = 0; p[2] < g->n[2]; p[2]++) {
                double acc = 0.0;
                double ks = at(g, x, p), kc = 0.0;   /* Kahan sum and compensation */
                for (int d = 0; d < g->ndims; d++) {
                    long lo[3], hi[3];
                    sh(lo, p, d, 0);
                    sh(hi, p, d, 1);
                    double flo, fhi;
                    if (iga_flux) {
                        flo = wat(g, d, c[d], lo);
                        fhi = wat(g, d, c[d], hi);
                    } else {
                        flo = donor_flux(g, d, x, c[d], lo);
                        fhi = donor_flux(g, d, x, c[d], hi);
                    }
                    acc += fhi - flo;
                    if (g->kahan) {
                        double t = fhi - flo;
                        if (G) t = t / at(g, G, p);
                        double y = -t - kc;
                        double u = ks + y;
                        kc = (u - ks) - y;
                        ks = u;
                    }
                }
                if (g->kahan) {
                    out[cidx(g, p)] = ks;
                } else {
                    double r = G ? acc / at(g, G, p) : acc;
                    out[cidx(g, p)] = at(g, x, p) - r;
                }
            }
    }
}

/* ------------------------------------------------------------------------ */
/* antidiffusive pseudo-velocity (eq. adf_vel and its multi-D / third-order  */
/* extensions cited in Sects. 3.1.1-3.1.2)                                   */
/* ------------------------------------------------------------------------ */

/* Mean of the dimension-o advector over the four walls of cells L and R that
 * are normal to o (the cross-velocity at a dimension-d wall). */
static double cross_mean(const grid_t *g, int o, const double *co,
                         const long L[3], const long R[3])
{
    long a[3], b[3], e[3], f[3];
    sh(a, L, o, 0);
    sh(b, L, o, 1);
    sh(e, R, o, 0);
    sh(f, R, o, 1);
    return 0.25 * (wat(g, o, co, a) + wat(g, o, co, b) + wat(g, o, co, e) +
                   wat(g, o, co, f));
}

/* Pseudo-velocity at wall p of dimension d from the previous pass's field x
 * and advector c.  With Gb = (G(L)+G(R))/2 and cb_o the cross means:
 *   V  = (|c| - c^2/Gb) A                                   (eq. adf_vel)
 *      - sum_{o!=d} c cb_o / (2 Gb) B_o                     (cross terms)
 * and with the third-order option:
 *   V += (3c|c|/Gb - 2c^3/Gb^2 - c)/3 D
 *      + sum_{o!=d} (|c| cb_o/Gb - 2 c^2 cb_o/Gb^2) E_o
 *      - (2/3) c cb_o1 cb_o2 / Gb^2 T                      (3-D only)
 * where A, B_o, D, E_o, T are psi-fractions of the first difference along d,
 * the centred difference along o, the third difference along d, the mixed
 * d-o difference and the mixed o1-o2 difference. */
static double pseudo_velocity(const grid_t *g, int d, const double *x,
                              double *const c[3], const double *G,
                              const long p[3])
{
    long L[3], R[3];
    sh(L, p, d, -1);
    sh(R, p, d, 0);
    double u = wat(g, d, c[d], p);
    double Gb = 0.5 * (gat(g, G, L) + gat(g, G, R));
    double xL = xat(g, x, L), xR = xat(g, x, R);

    double A = frac(g, xR - xL, xR + xL, 2.0);
    double V = (fabs(u) - u * u / Gb) * A;

    double cb[3] = {0.0, 0.0, 0.0};
    for (int o = 0; o < g->ndims; o++) {
        if (o == d) continue;
        cb[o] = cross_mean(g, o, c[o], L, R);
        long Rp[3], Lp[3], Rm[3], Lm[3];
        sh(Rp, R, o, 1);
        sh(Lp, L, o, 1);
        sh(Rm, R, o, -1);
        sh(Lm, L, o, -1);
        double a = xat(g, x, Rp), b = xat(g, x, Lp), e = xat(g, x, Rm),
               f = xat(g, x, Lm);
        double B = frac(g, a + b - e - f, a + b + e + f, 4.0);
        V -= 0.5 * u * cb[o] / Gb * B;
    }

    if (g->dfl) {
        /* divergent-flow term (Sect. 3.1.3): -c/(2 Gb) times the advector's
         * divergence at the wall, the mean of the two cells' divergences
         * sum_o (c_o(hi) - c_o(lo)) */
        double dv = 0.0;
        for (int o = 0; o < g->ndims; o++) {
            long Lh[3], Rh[3];
            sh(Lh, L, o, 1);
            sh(Rh, R, o, 1);
            dv += (wat(g, o, c[o], Lh) - wat(g, o, c[o], L)) +
                  (wat(g, o, c[o], Rh) - wat(g, o, c[o], R));
        }
        /* under iga the pseudo-velocity is the flux of a unit field (the
         * psi-fractions become halved differences), so this psi-free term
         * takes the wall mean of psi to stay the same flux */
        double w = g->iga ? 0.5 * (xL + xR) : 1.0;
        V -= 0.25 * u / Gb * dv * w;
    }

    if (g->tot) {
        long R2[3], L2[3];
        sh(R2, R, d, 1);
        sh(L2, L, d, -1);
        double xR2 = xat(g, x, R2), xL2 = xat(g, x, L2);
        double D = frac(g, xR2 - xR - xL + xL2, xR2 + xR + xL + xL2, 4.0);
        V += (3.0 * u * fabs(u) / Gb - 2.0 * u * u * u / (Gb * Gb) - u) /
             3.0 * D;

        for (int o = 0; o < g->ndims; o++) {
            if (o == d) continue;
            long Rp[3], Lp[3], Rm[3], Lm[3];
            sh(Rp, R, o, 1);
            sh(Lp, L, o, 1);
            sh(Rm, R, o, -1);
            sh(Lm, L, o, -1);
            double a = xat(g, x, Rp), b = xat(g, x, Lp), e = xat(g, x, Rm),
                   f = xat(g, x, Lm);
            double E = frac(g, a - b - e + f, a + b + e + f, 4.0);
            V += (fabs(u) * cb[o] / Gb - 2.0 * u * u * cb[o] / (Gb * Gb)) * E;
        }

        if (g->ndims == 3) {
            int o1 = (d == 0) ? 1 : 0;
            int o2 = (d == 2) ? 1 : 2;
            double num = 0.0, den = 0.0;
            const long *side[2] = {L, R};
            for (int s = 0; s < 2; s++) {
                long pp[3], mp[3], pm[3], mm[3];
                sh2(pp, side[s], o1, 1, o2, 1);
                sh2(mp, side[s], o1, -1, o2, 1);
                sh2(pm, side[s], o1, 1, o2, -1);
                sh2(mm, side[s], o1, -1, o2, -1);
                double vpp = xat(g, x, pp), vmp = xat(g, x, mp),
                       vpm = xat(g, x, pm), vmm = xat(g, x, mm);
                num += vpp - vmp - vpm + vmm;
                den += vpp + vmp + vpm + vmm;
            }
            double T = frac(g, num, den, 8.0);
            V += -(2.0 / 3.0) * u * cb[o1] * cb[o2] / (Gb * Gb) * T;
        }
    }
    return V;
}

static void antidiffusive_velocity(const grid_t *g, const double *x,
                                   double *const c[3], const double *G,
                                   double *V[3])
{
    for (int d = 0; d < g->ndims; d++) {
        long e[3] = {g->n[0], g->n[1], g->n[2]};
        e[d] += 1;
        ROWS_IN_PARALLEL
        for (long i0 = 0; i0 < e[0]; i0++) {
            long p[3] = {i0, 0, 0};
            for (p[1] = 0; p[1] < e[1]; p[1]++)
                for (p[2] = 0; p[2] < e[2]; p[2]++)
                    V[d][(p[0] * e[1] + p[1]) * e[2] + p[2]] =
                        pseudo_velocity(g, d, x, c, G, p);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* non-oscillatory option (Sect. 3.1.4): flux-corrected limiting of V        */
/* ------------------------------------------------------------------------ */

/* Local bounds from the step's input field psi_n and the previous pass's x
 * over the cell and its face neighbours; inflow/outflow sums of the
 * corrective fluxes (weight x, or 1 under the infinite gauge); limiter
 * coefficients
 *   beta_up = G (psi_max - x) / f_in   (1 when f_in == 0)
 *   beta_dn = G (x - psi_min) / f_out  (1 when f_out == 0)
 * and the limited pseudo-velocity at the wall between cells L and R:
 *   [V]^+ min(1, beta_dn(L), beta_up(R)) + [V]^- min(1, beta_up(L), beta_dn(R)).
 */
static void fct_limit(const grid_t *g, const double *psi_n, const double *x,
                      const double *G, double *V[3], double *const Vlim[3],
                      double *beta_up, double *beta_dn)
{
    ROWS_IN_PARALLEL
    for (long i0 = 0; i0 < g->n[0]; i0++) {
        long p[3] = {i0, 0, 0};
        for (p[1] = 0; p[1] < g->n[1]; p[1]++)
            for (p[2] = 0; p[2] < g->n[2]; p[2]++) {
                double mx = at(g, psi_n, p), mn = mx;
                double v = at(g, x, p);
                if (v > mx) mx = v;
                if (v < mn) mn = v;
                for (int d = 0; d < g->ndims; d++)
                    for (int s = -1; s <= 1; s += 2) {
                        long q[3];
                        sh(q, p, d, s);
                        double a = at(g, psi_n, q), b = at(g, x, q);
                        if (a > mx) mx = a;
                        if (a < mn) mn = a;
                        if (b > mx) mx = b;
                        if (b < mn) mn = b;
                    }

                double fin = 0.0, fout = 0.0;
                double xi = at(g, x, p);
                for (int d = 0; d < g->ndims; d++) {
                    long lo[3], hi[3], qm[3], qp[3];
                    sh(lo, p, d, 0);
                    sh(hi, p, d, 1);
                    sh(qm, p, d, -1);
                    sh(qp, p, d, 1);
                    double vlo = wat(g, d, V[d], lo), vhi = wat(g, d, V[d], hi);
                    double wm = g->iga ? 1.0 : at(g, x, qm);
                    double wp = g->iga ? 1.0 : at(g, x, qp);
                    double wi = g->iga ? 1.0 : xi;
                    fin += pos(vlo) * wm - neg(vhi) * wp;
                    fout += pos(vhi) * wi - neg(vlo) * wi;
                }
                double Gi = gat(g, G, p);
                long k = cidx(g, p);
                beta_up[k] = fin > 0.0 ? Gi * (mx - xi) / fin : 1.0;
                beta_dn[k] = fout > 0.0 ? Gi * (xi - mn) / fout : 1.0;
            }
    }

    for (int d = 0; d < g->ndims; d++) {
        long e[3] = {g->n[0], g->n[1], g->n[2]};
        e[d] += 1;
        ROWS_IN_PARALLEL
        for (long i0 = 0; i0 < e[0]; i0++) {
            long p[3] = {i0, 0, 0};
            for (p[1] = 0; p[1] < e[1]; p[1]++)
                for (p[2] = 0; p[2] < e[2]; p[2]++) {
                    long L[3], R[3];
                    sh(L, p, d, -1);
                    sh(R, p, d, 0);
                    double v = wat(g, d, V[d], p);
                    double up = 1.0, dn = 1.0;
                    /* positive V: leaves L, enters R */
                    if (at(g, beta_dn, L) < up) up = at(g, beta_dn, L);
                    if (at(g, beta_up, R) < up) up = at(g, beta_up, R);
                    /* negative V: leaves R, enters L */
                    if (at(g, beta_up, L) < dn) dn = at(g, beta_up, L);
                    if (at(g, beta_dn, R) < dn) dn = at(g, beta_dn, R);
                    Vlim[d][(p[0] * e[1] + p[1]) * e[2] + p[2]] =
                        pos(v) * up + neg(v) * dn;
                }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* one step and the step loop                                                */
/* ------------------------------------------------------------------------ */

typedef struct {
    double *x, *y;          /* pass input / output */
    double *V[3], *W[3];    /* raw and limited pseudo-velocities */
    double *cprev[3];       /* advector of the previous pass (own copy) */
    double *bup, *bdn;
} work_t;

static int work_alloc(const grid_t *g, work_t *w)
{
    memset(w, 0, sizeof *w);
    long N = cells(g);
    w->x = malloc(sizeof(double) * N);
    w->y = malloc(sizeof(double) * N);
    w->bup = malloc(sizeof(double) * N);
    w->bdn = malloc(sizeof(double) * N);
    if (!w->x || !w->y || !w->bup || !w->bdn) return -1;
    for (int d = 0; d < g->ndims; d++) {
        long M = walls(g, d);
        w->V[d] = malloc(sizeof(double) * M);
        w->W[d] = malloc(sizeof(double) * M);
        w->cprev[d] = malloc(sizeof(double) * M);
        if (!w->V[d] || !w->W[d] || !w->cprev[d]) return -1;
    }
    return 0;
}

static void work_free(work_t *w)
{
    free(w->x);
    free(w->y);
    free(w->bup);
    free(w->bdn);
    for (int d = 0; d < 3; d++) {
        free(w->V[d]);
        free(w->W[d]);
        free(w->cprev[d]);
    }
}

/* psi_out = one MPDATA step of psi_n: donor-cell pass with the advector c,
 * then n_iters-1 corrective passes, each advecting the previous pass's result
 * with the (optionally limited) pseudo-velocity computed from it; the
 * pseudo-velocity of a pass is the advector of the next. */
static void one_step(const grid_t *g, int n_iters, const double *psi_n,
                     const double *G, double *const c[3], work_t *w,
                     double *psi_out)
{
    long N = cells(g);
    donor_pass(g, psi_n, c, G, 0, w->y);
    for (int d = 0; d < g->ndims; d++)
        memcpy(w->cprev[d], c[d], sizeof(double) * walls(g, d));
    for (int it = 2; it <= n_iters; it++) {
        memcpy(w->x, w->y, sizeof(double) * N);
        antidiffusive_velocity(g, w->x, w->cprev, G, w->V);
        double **adv = w->V;
        if (g->fct) {
            fct_limit(g, psi_n, w->x, G, w->V, w->W, w->bup, w->bdn);
            adv = w->W;
        }
        donor_pass(g, w->x, adv, G, g->iga, w->y);
        for (int d = 0; d < g->ndims; d++)
            memcpy(w->cprev[d], adv[d], sizeof(double) * walls(g, d));
    }
    memcpy(psi_out, w->y, sizeof(double) * N);
}

static int make_grid(grid_t *g, int ndims, const long n[3], const int bc[3],
                     unsigned opts)
{
    if (ndims < 1 || ndims > 3) return -1;
    if (opts & ~(unsigned)(ORC_OPT_FCT | ORC_OPT_IGA | ORC_OPT_TOT | ORC_OPT_KAHAN | ORC_OPT_ABS |
                           ORC_OPT_DFL))
        return -1;
    /* abs and iga are the two alternative variable-sign options */
    if ((opts & ORC_OPT_ABS) && (opts & ORC_OPT_IGA)) return -1;
    g->ndims = ndims;
    for (int d = 0; d < 3; d++) {
        g->n[d] = d < ndims ? n[d] : 1;
        g->bc[d] = d < ndims ? bc[d] : ORC_BC_PERIODIC;
        if (g->n[d] < 1) return -1;
        if (g->bc[d] != ORC_BC_PERIODIC && g->bc[d] != ORC_BC_OPEN) return -1;
    }
    g->fct = (opts & ORC_OPT_FCT) != 0;
    g->iga = (opts & ORC_OPT_IGA) != 0;
    g->tot = (opts & ORC_OPT_TOT) != 0;
    g->kahan = (opts & ORC_OPT_KAHAN) != 0;
    g->abs = (opts & ORC_OPT_ABS) != 0;
    g->dfl = (opts & ORC_OPT_DFL) != 0;
    return 0;
}

int orc_step(int ndims, const long n[3], const int bc[3], int n_iters,
             unsigned opts, double *psi, const double *g_,
             const double *c0, const double *c1, const double *c2,
             long n_steps)
{
    grid_t g;
    if (make_grid(&g, ndims, n, bc, opts)) return -1;
    if (n_iters < 1 || n_steps < 0 || !psi) return -1;
    if (g.iga && n_iters > 2) return -1;
    double *c[3] = {(double *)c0, (double *)c1, (double *)c2};
    for (int d = 0; d < ndims; d++)
        if (!c[d]) return -1;
    work_t w;
    if (work_alloc(&g, &w)) {
        work_free(&w);
        return -1;
    }
    double *tmp = malloc(sizeof(double) * cells(&g));
    if (!tmp) {
        work_free(&w);
        return -1;
    }
    for (long s = 0; s < n_steps; s++) {
        memcpy(tmp, psi, sizeof(double) * cells(&g));
        one_step(&g, n_iters, tmp, g_, c, &w, psi);
    }
    free(tmp);
    work_free(&w);
    return 0;
}

/* Threads the stage loops use (1 unless built with -fopenmp). */
int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* diagnostics                                                               */
/* ------------------------------------------------------------------------ */

int orc_diag(int ndims, const long n[3], const double *psi, const double *G,
             double out[3], long *n_nonfinite)
{
    if (ndims < 1 || ndims > 3 || !psi || !out || !n_nonfinite) return -1;
    long N = 1;
    for (int d = 0; d < ndims; d++) N *= n[d];
    double s = 0.0, comp = 0.0;
    double mn = INFINITY, mx = -INFINITY;
    long bad = 0;
    for (long k = 0; k < N; k++) {
        double v = psi[k];
        if (!isfinite(v)) {
            bad++;
            continue;
        }
        double term = G ? G[k] * v : v;
        double t = s + term; /* Neumaier compensated summation */
        if (fabs(s) >= fabs(term))
            comp += (s - t) + term;
        else
            comp += (term - t) + s;
        s = t;
        if (v < mn) mn = v;
        if (v > mx) mx = v;
    }
    out[0] = s + comp;
    out[1] = mn;
    out[2] = mx;
    *n_nonfinite = bad;
    return 0;
}

int orc_courant_max(int ndims, const long n[3], const int bc[3],
                    const double *G, const double *c0, const double *c1,
                    const double *c2, double *out)
{
    grid_t g;
    if (make_grid(&g, ndims, n, bc, 0) || !out) return -1;
    const double *c[3] = {c0, c1, c2};
    for (int d = 0; d < ndims; d++)
        if (!c[d]) return -1;
    double best = 0.0;
    long p[3];
    for (p[0] = 0; p[0] < g.n[0]; p[0]++)
        for (p[1] = 0; p[1] < g.n[1]; p[1]++)
            for (p[2] = 0; p[2] < g.n[2]; p[2]++) {
                double s = 0.0;
                for (int d = 0; d < ndims; d++) {
                    long lo[3], hi[3];
                    sh(lo, p, d, 0);
                    sh(hi, p, d, 1);
                    double a = fabs(wat(&g, d, c[d], lo));
                    double b = fabs(wat(&g, d, c[d], hi));
                    s += a > b ? a : b;
                }
                s /= gat(&g, G, p);
                if (s > best) best = s;
            }
    *out = best;
    return 0;
}



/* ======================================================================== */
/* Reverse mode (adjoint) of the step -- an extension, not in the paper.     */
/*                                                                          */
/* Every forward stage above gets a transposed loop that runs in the        */
/* opposite order and accumulates adjoints into the cells / walls the       */
/* forward read (through the same boundary map).  Conventions at the        */
/* non-differentiable points:                                               */
/*   d[u]^+/du = 1 only for u > 0, d[u]^-/du = 1 only for u < 0,            */
/*   d|u|/du = [u > 0] - [u < 0];                                           */
/*   a max / min passes the derivative to the operand it returned, ties     */
/*   going to the earliest operand in the order the forward scans them;     */
/*   the zero-denominator branch of a psi-fraction and the "no flux"        */
/*   branch (coefficient 1) of the limiter have zero derivative.            */
/* G is a constant of the problem (no adjoint).                             */
/* ======================================================================== */

static int sgn_d(double u) { return (u > 0.0) - (u < 0.0); }

/* adjoint of frac(): returns d frac / d num and d frac / d den */
static void frac_adj(const grid_t *g, double num, double den, double m,
                     double *dn, double *dd)
{
    if (g->iga) {
        *dn = 1.0 / m;
        *dd = 0.0;
        return;
    }
    if (den == 0.0) {
        *dn = 0.0;
        *dd = 0.0;
        return;
    }
    *dn = 1.0 / den;
    *dd = -num / (den * den);
}

/* adjoint of one wall flux of the donor-cell pass */
static void donor_flux_adj(const grid_t *g, int d, const double *x,
                           const double *c, const long p[3], double fb,
                           double *xb, double *cb)
{
    long L[3], R[3];
    sh(L, p, d, -1);
    sh(R, p, d, 0);
    double u = wat(g, d, c, p);
    double du = (u > 0.0 ? at(g, x, L) : 0.0) + (u < 0.0 ? at(g, x, R) : 0.0);
    cb[widx(g, d, p)] += du * fb;
    xb[cidx(g, L)] += pos(u) * fb;
    xb[cidx(g, R)] += neg(u) * fb;
}

static void donor_pass_adj(const grid_t *g, const double *x, double *const c[3],
                           const double *G, int iga_flux, const double *yb,
                           double *xb, double *cb[3])
{
    long p[3];
    for (p[0] = 0; p[0] < g->n[0]; p[0]++)
        for (p[1] = 0; p[1] < g->n[1]; p[1]++)
            for (p[2] = 0; p[2] < g->n[2]; p[2]++) {
                long k = cidx(g, p);
                double ob = yb[k];
                xb[k] += ob;
                double accb = G ? -ob / at(g, G, p) : -ob;
                for (int d = 0; d < g->ndims; d++) {
                    long lo[3], hi[3];
                    sh(lo, p, d, 0);
                    sh(hi, p, d, 1);
                    if (iga_flux) {
                        cb[d][widx(g, d, hi)] += accb;
                        cb[d][widx(g, d, lo)] -= accb;
                    } else {
                        donor_flux_adj(g, d, x, c[d], hi, accb, xb, cb[d]);
                        donor_flux_adj(g, d, x, c[d], lo, -accb, xb, cb[d]);
                    }
                }
            }
}

/* adjoint of pseudo_velocity() at wall p of dimension d: vb = dJ/dV */
static void pseudo_velocity_adj(const grid_t *g, int d, const double *x,
                                double *const c[3], const double *G,
                                const long p[3], double vb, double *xb,
                                double *cb[3])
{
    if (vb == 0.0) return;
    long L[3], R[3];
    sh(L, p, d, -1);
    sh(R, p, d, 0);
    double u = wat(g, d, c[d], p);
    double Gb = 0.5 * (gat(g, G, L) + gat(g, G, R));
    double xL = at(g, x, L), xR = at(g, x, R);
    double ub = 0.0; /* adjoint of u */

    /* A term: (|u| - u^2/Gb) A */
    double nA = xR - xL, dA = xR + xL, fn, fd;
    double A = frac(g, nA, dA, 2.0);
    frac_adj(g, nA, dA, 2.0, &fn, &fd);
    double coef = fabs(u) - u * u / Gb;
    ub += (sgn_d(u) - 2.0 * u / Gb) * A * vb;
    double Ab = coef * vb;
    xb[cidx(g, R)] += (fn + fd) * Ab;
    xb[cidx(g, L)] += (-fn + fd) * Ab;

    double cbar[3] = {0.0, 0.0, 0.0}, cbar_b[3] = {0.0, 0.0, 0.0};
    for (int o = 0; o < g->ndims; o++) {
        if (o == d) continue;
        cbar[o] = cross_mean(g, o, c[o], L, R);
        long Rp[3], Lp[3], Rm[3], Lm[3];
        sh(Rp, R, o, 1);
        sh(Lp, L, o, 1);
        sh(Rm, R, o, -1);
        sh(Lm, L, o, -1);
        double a = at(g, x, Rp), b = at(g, x, Lp), e = at(g, x, Rm),
               f = at(g, x, Lm);
        double nB = a + b - e - f, dB = a + b + e + f;
        double B = frac(g, nB, dB, 4.0);
        frac_adj(g, nB, dB, 4.0, &fn, &fd);
        /* V -= 0.5 u cb B / Gb */
        ub += -0.5 * cbar[o] / Gb * B * vb;
        cbar_b[o] += -0.5 * u / Gb * B * vb;
        double Bb = -0.5 * u * cbar[o] / Gb * vb;
        xb[cidx(g, Rp)] += (fn + fd) * Bb;
        xb[cidx(g, Lp)] += (fn + fd) * Bb;
        xb[cidx(g, Rm)] += (-fn + fd) * Bb;
        xb[cidx(g, Lm)] += (-fn + fd) * Bb;
    }

    if (g->tot) {
        long R2[3], L2[3];
        sh(R2, R, d, 1);
        sh(L2, L, d, -1);
        double xR2 = at(g, x, R2), xL2 = at(g, x, L2);
        double nD = xR2 - xR - xL + xL2, dD = xR2 + xR + xL + xL2;
        double D = frac(g, nD, dD, 4.0);
        frac_adj(g, nD, dD, 4.0, &fn, &fd);
        double cD = (3.0 * u * fabs(u) / Gb - 2.0 * u * u * u / (Gb * Gb) - u) / 3.0;
        ub += (6.0 * fabs(u) / Gb - 6.0 * u * u / (Gb * Gb) - 1.0) / 3.0 * D * vb;
        double Db = cD * vb;
        xb[cidx(g, R2)] += (fn + fd) * Db;
        xb[cidx(g, R)] += (-fn + fd) * Db;
        xb[cidx(g, L)] += (-fn + fd) * Db;
        xb[cidx(g, L2)] += (fn + fd) * Db;

        for (int o = 0; o < g->ndims; o++) {
            if (o == d) continue;
            long Rp[3], Lp[3], Rm[3], Lm[3];
            sh(Rp, R, o, 1);
            sh(Lp, L, o, 1);
            sh(Rm, R, o, -1);
            sh(Lm, L, o, -1);
            double a = at(g, x, Rp), b = at(g, x, Lp), e = at(g, x, Rm),
                   f = at(g, x, Lm);
            double nE = a - b - e + f, dE = a + b + e + f;
            double E = frac(g, nE, dE, 4.0);
            frac_adj(g, nE, dE, 4.0, &fn, &fd);
            double cE = fabs(u) * cbar[o] / Gb - 2.0 * u * u * cbar[o] / (Gb * Gb);
            ub += (sgn_d(u) * cbar[o] / Gb - 4.0 * u * cbar[o] / (Gb * Gb)) * E * vb;
            cbar_b[o] += (fabs(u) / Gb - 2.0 * u * u / (Gb * Gb)) * E * vb;
            double Eb = cE * vb;
            xb[cidx(g, Rp)] += (fn + fd) * Eb;
            xb[cidx(g, Lp)] += (-fn + fd) * Eb;
            xb[cidx(g, Rm)] += (-fn + fd) * Eb;
            xb[cidx(g, Lm)] += (fn + fd) * Eb;
        }

        if (g->ndims == 3) {
            int o1 = (d == 0) ? 1 : 0;
            int o2 = (d == 2) ? 1 : 2;
            double num = 0.0, den = 0.0;
            const long *side[2] = {L, R};
            long pts[2][4][3];
            for (int s = 0; s < 2; s++) {
                sh2(pts[s][0], side[s], o1, 1, o2, 1);
                sh2(pts[s][1], side[s], o1, -1, o2, 1);
                sh2(pts[s][2], side[s], o1, 1, o2, -1);
                sh2(pts[s][3], side[s], o1, -1, o2, -1);
                double vpp = at(g, x, pts[s][0]), vmp = at(g, x, pts[s][1]),
                       vpm = at(g, x, pts[s][2]), vmm = at(g, x, pts[s][3]);
                num += vpp - vmp - vpm + vmm;
                den += vpp + vmp + vpm + vmm;
            }
            double T = frac(g, num, den, 8.0);
            frac_adj(g, num, den, 8.0, &fn, &fd);
            double k = -(2.0 / 3.0) / (Gb * Gb);
            ub += k * cbar[o1] * cbar[o2] * T * vb;
            cbar_b[o1] += k * u * cbar[o2] * T * vb;
            cbar_b[o2] += k * u * cbar[o1] * T * vb;
            double Tb = k * u * cbar[o1] * cbar[o2] * vb;
            static const double sgn4[4] = {1.0, -1.0, -1.0, 1.0};
            for (int s = 0; s < 2; s++)
                for (int q = 0; q < 4; q++)
                    xb[cidx(g, pts[s][q])] += (sgn4[q] * fn + fd) * Tb;
        }
    }

    cb[d][widx(g, d, p)] += ub;
    for (int o = 0; o < g->ndims; o++) {
        if (o == d || cbar_b[o] == 0.0) continue;
        long a[3], b[3], e[3], f[3];
        sh(a, L, o, 0);
        sh(b, L, o, 1);
        sh(e, R, o, 0);
        sh(f, R, o, 1);
        double q = 0.25 * cbar_b[o];
        cb[o][widx(g, o, a)] += q;
        cb[o][widx(g, o, b)] += q;
        cb[o][widx(g, o, e)] += q;
        cb[o][widx(g, o, f)] += q;
    }
}

/* adjoint of fct_limit(): Wb = dJ/dVlim (walls) -> Vb, xb, pnb */
static void fct_limit_adj(const grid_t *g, const double *psi_n, const double *x,
                          const double *G, double *const V[3], const double *bup,
                          const double *bdn, double *const Wb[3], double *Vb[3],
                          double *xb, double *pnb, double *bub, double *bdb)
{
    long N = cells(g);
    for (long k = 0; k < N; k++) bub[k] = bdb[k] = 0.0;
    long p[3];
    /* limited velocities: W = [V]^+ up + [V]^- dn */
    for (int d = 0; d < g->ndims; d++) {
        long e[3] = {g->n[0], g->n[1], g->n[2]};
        e[d] += 1;
        for (p[0] = 0; p[0] < e[0]; p[0]++)
            for (p[1] = 0; p[1] < e[1]; p[1]++)
                for (p[2] = 0; p[2] < e[2]; p[2]++) {
                    long w = (p[0] * e[1] + p[1]) * e[2] + p[2];
                    double wb = Wb[d][w];
                    if (wb == 0.0) continue;
                    long L[3], R[3];
                    sh(L, p, d, -1);
                    sh(R, p, d, 0);
                    double v = wat(g, d, V[d], p);
                    double up = 1.0, dn = 1.0;
                    int wu = 0, wd = 0;
                    if (at(g, bdn, L) < up) {
                        up = at(g, bdn, L);
                        wu = 1;
                    }
                    if (at(g, bup, R) < up) {
                        up = at(g, bup, R);
                        wu = 2;
                    }
                    if (at(g, bup, L) < dn) {
                        dn = at(g, bup, L);
                        wd = 1;
                    }
                    if (at(g, bdn, R) < dn) {
                        dn = at(g, bdn, R);
                        wd = 2;
                    }
                    Vb[d][widx(g, d, p)] +=
                        ((v > 0.0 ? up : 0.0) + (v < 0.0 ? dn : 0.0)) * wb;
                    double upb = pos(v) * wb, dnb = neg(v) * wb;
                    if (wu == 1) bdb[cidx(g, L)] += upb;
                    if (wu == 2) bub[cidx(g, R)] += upb;
                    if (wd == 1) bub[cidx(g, L)] += dnb;
                    if (wd == 2) bdb[cidx(g, R)] += dnb;
                }
    }

    /* limiter coefficients, bounds and in/out fluxes */
    for (p[0] = 0; p[0] < g->n[0]; p[0]++)
        for (p[1] = 0; p[1] < g->n[1]; p[1]++)
            for (p[2] = 0; p[2] < g->n[2]; p[2]++) {
                long k = cidx(g, p);
                double bu_b = bub[k], bd_b = bdb[k];
                if (bu_b == 0.0 && bd_b == 0.0) continue;
                /* bounds with the operand that attains them (forward scan
                 * order: cell then face neighbours, psi_n before x) */
                double mx = at(g, psi_n, p), mn = mx;
                long amx = k, amn = k;
                int smx = 0, smn = 0; /* 0: psi_n, 1: x */
                double v = at(g, x, p);
                if (v > mx) { mx = v; smx = 1; }
                if (v < mn) { mn = v; smn = 1; }
                for (int d = 0; d < g->ndims; d++)
                    for (int s = -1; s <= 1; s += 2) {
                        long q[3];
                        sh(q, p, d, s);
                        long kq = cidx(g, q);
                        double a = at(g, psi_n, q), b = at(g, x, q);
                        if (a > mx) { mx = a; amx = kq; smx = 0; }
                        if (a < mn) { mn = a; amn = kq; smn = 0; }
                        if (b > mx) { mx = b; amx = kq; smx = 1; }
                        if (b < mn) { mn = b; amn = kq; smn = 1; }
                    }
                double fin = 0.0, fout = 0.0;
                double xi = at(g, x, p);
                for (int d = 0; d < g->ndims; d++) {
                    long lo[3], hi[3], qm[3], qp[3];
                    sh(lo, p, d, 0);
                    sh(hi, p, d, 1);
                    sh(qm, p, d, -1);
                    sh(qp, p, d, 1);
                    double vlo = wat(g, d, V[d], lo), vhi = wat(g, d, V[d], hi);
                    double wm = g->iga ? 1.0 : at(g, x, qm);
                    double wp = g->iga ? 1.0 : at(g, x, qp);
                    double wi = g->iga ? 1.0 : xi;
                    fin += pos(vlo) * wm - neg(vhi) * wp;
                    fout += pos(vhi) * wi - neg(vlo) * wi;
                }
                double Gi = gat(g, G, p);
                double finb = 0.0, foutb = 0.0, mxb = 0.0, mnb = 0.0;
                if (fin > 0.0 && bu_b != 0.0) {
                    mxb += Gi / fin * bu_b;
                    xb[k] -= Gi / fin * bu_b;
                    finb -= Gi * (mx - xi) / (fin * fin) * bu_b;
                }
                if (fout > 0.0 && bd_b != 0.0) {
                    xb[k] += Gi / fout * bd_b;
                    mnb -= Gi / fout * bd_b;
                    foutb -= Gi * (xi - mn) / (fout * fout) * bd_b;
                }
                if (mxb != 0.0) {
                    if (smx) xb[amx] += mxb;
                    else pnb[amx] += mxb;
                }
                if (mnb != 0.0) {
                    if (smn) xb[amn] += mnb;
                    else pnb[amn] += mnb;
                }
                for (int d = 0; d < g->ndims; d++) {
                    long lo[3], hi[3], qm[3], qp[3];
                    sh(lo, p, d, 0);
                    sh(hi, p, d, 1);
                    sh(qm, p, d, -1);
                    sh(qp, p, d, 1);
                    double vlo = wat(g, d, V[d], lo), vhi = wat(g, d, V[d], hi);
                    double wm = g->iga ? 1.0 : at(g, x, qm);
                    double wp = g->iga ? 1.0 : at(g, x, qp);
                    double wi = g->iga ? 1.0 : xi;
                    long wlo = widx(g, d, lo), whi = widx(g, d, hi);
                    Vb[d][wlo] += (vlo > 0.0 ? wm : 0.0) * finb;
                    Vb[d][whi] -= (vhi < 0.0 ? wp : 0.0) * finb;
                    Vb[d][whi] += (vhi > 0.0 ? wi : 0.0) * foutb;
                    Vb[d][wlo] -= (vlo < 0.0 ? wi : 0.0) * foutb;
                    if (!g->iga) {
                        xb[cidx(g, qm)] += pos(vlo) * finb;
                        xb[cidx(g, qp)] -= neg(vhi) * finb;
                        xb[k] += (pos(vhi) - neg(vlo)) * foutb;
                    }
                }
            }
}

/* forward record of one step: per pass its input field, the advector its
 * pseudo-velocity used, the raw and limited pseudo-velocities and the
 * limiter coefficients */
typedef struct {
    double *x;
    double *cin[3];
    double *V[3], *W[3];
    double *bup, *bdn;
} pass_rec_t;

static void free_recs(pass_rec_t *r, int n)
{
    for (int p = 0; p < n; p++) {
        free(r[p].x);
        free(r[p].bup);
        free(r[p].bdn);
        for (int d = 0; d < 3; d++) {
            free(r[p].cin[d]);
            free(r[p].V[d]);
            free(r[p].W[d]);
        }
    }
}

static int alloc_recs(const grid_t *g, pass_rec_t *r, int n)
{
    memset(r, 0, sizeof(pass_rec_t) * n);
    long N = cells(g);
    for (int p = 0; p < n; p++) {
        r[p].x = malloc(sizeof(double) * N);
        r[p].bup = malloc(sizeof(double) * N);
        r[p].bdn = malloc(sizeof(double) * N);
        if (!r[p].x || !r[p].bup || !r[p].bdn) return -1;
        for (int d = 0; d < g->ndims; d++) {
            long M = walls(g, d);
            r[p].cin[d] = malloc(sizeof(double) * M);
            r[p].V[d] = malloc(sizeof(double) * M);
            r[p].W[d] = malloc(sizeof(double) * M);
            if (!r[p].cin[d] || !r[p].V[d] || !r[p].W[d]) return -1;
        }
    }
    return 0;
}

/* recompute one step from psi_n, keeping what the reverse sweep needs;
 * rec[0] is the donor pass (its cin is the input advector), rec[p] pass p+1 */
static void record_step(const grid_t *g, int n_iters, const double *psi_n,
                        const double *G, double *const c[3], pass_rec_t *rec,
                        double *y)
{
    long N = cells(g);
    memcpy(rec[0].x, psi_n, sizeof(double) * N);
    for (int d = 0; d < g->ndims; d++)
        memcpy(rec[0].cin[d], c[d], sizeof(double) * walls(g, d));
    donor_pass(g, psi_n, c, G, 0, y);
    for (int it = 2; it <= n_iters; it++) {
        pass_rec_t *r = &rec[it - 1];
        pass_rec_t *prev = &rec[it - 2];
        memcpy(r->x, y, sizeof(double) * N);
        for (int d = 0; d < g->ndims; d++)
            memcpy(r->cin[d], it == 2 ? prev->cin[d] : prev->W[d],
                   sizeof(double) * walls(g, d));
        antidiffusive_velocity(g, r->x, r->cin, G, r->V);
        if (g->fct) {
            fct_limit(g, psi_n, r->x, G, r->V, r->W, r->bup, r->bdn);
        } else {
            for (int d = 0; d < g->ndims; d++)
                memcpy(r->W[d], r->V[d], sizeof(double) * walls(g, d));
        }
        donor_pass(g, r->x, r->W, G, g->iga, y);
    }
}

/* reverse of one step: yb = dJ/dpsi_{n+1} -> pnb = dJ/dpsi_n (overwritten),
 * cgrad += dJ/dc (input advector) */
static int adjoint_step(const grid_t *g, int n_iters, const double *psi_n,
                        const double *G, double *const c[3], const double *yb_in,
                        double *pnb, double *cgrad[3])
{
    long N = cells(g);
    pass_rec_t rec[8];
    double *y = malloc(sizeof(double) * N);
    double *yb = malloc(sizeof(double) * N);
    double *xb = malloc(sizeof(double) * N);
    double *bub = malloc(sizeof(double) * N);
    double *bdb = malloc(sizeof(double) * N);
    double *Ab[3] = {0, 0, 0}, *Vb[3] = {0, 0, 0}, *Cb[3] = {0, 0, 0};
    int rc = -1;
    if (alloc_recs(g, rec, n_iters) || !y || !yb || !xb || !bub || !bdb) goto done;
    for (int d = 0; d < g->ndims; d++) {
        Ab[d] = calloc(walls(g, d), sizeof(double));
        Vb[d] = calloc(walls(g, d), sizeof(double));
        Cb[d] = calloc(walls(g, d), sizeof(double));
        if (!Ab[d] || !Vb[d] || !Cb[d]) goto done;
    }
    record_step(g, n_iters, psi_n, G, c, rec, y);
    memcpy(yb, yb_in, sizeof(double) * N);
    for (long k = 0; k < N; k++) pnb[k] = 0.0;

    /* Ab holds dJ/d(advector produced by the pass being reversed) */
    for (int it = n_iters; it >= 2; it--) {
        pass_rec_t *r = &rec[it - 1];
        for (long k = 0; k < N; k++) xb[k] = 0.0;
        /* corrective donor-cell pass (advector W, or flux W under iga) */
        donor_pass_adj(g, r->x, r->W, G, g->iga, yb, xb, Ab);
        /* limiter */
        for (int d = 0; d < g->ndims; d++)
            memset(Vb[d], 0, sizeof(double) * walls(g, d));
        if (g->fct) {
            fct_limit_adj(g, psi_n, r->x, G, r->V, r->bup, r->bdn, Ab, Vb, xb,
                          pnb, bub, bdb);
        } else {
            for (int d = 0; d < g->ndims; d++)
                memcpy(Vb[d], Ab[d], sizeof(double) * walls(g, d));
        }
        /* pseudo-velocity: adjoint flows to x and to the previous advector */
        for (int d = 0; d < g->ndims; d++)
            memset(Ab[d], 0, sizeof(double) * walls(g, d));
        for (int d = 0; d < g->ndims; d++) {
            long e[3] = {g->n[0], g->n[1], g->n[2]};
            e[d] += 1;
            long p[3];
            for (p[0] = 0; p[0] < e[0]; p[0]++)
                for (p[1] = 0; p[1] < e[1]; p[1]++)
                    for (p[2] = 0; p[2] < e[2]; p[2]++)
                        pseudo_velocity_adj(g, d, r->x, r->cin, G, p,
                                            Vb[d][(p[0] * e[1] + p[1]) * e[2] + p[2]],
                                            xb, Ab);
        }
        /* the advector of pass 2 is the input advector */
        if (it == 2)
            for (int d = 0; d < g->ndims; d++) {
                for (long w = 0; w < walls(g, d); w++) Cb[d][w] += Ab[d][w];
                memset(Ab[d], 0, sizeof(double) * walls(g, d));
            }
        memcpy(yb, xb, sizeof(double) * N);
    }
    /* donor-cell pass of the input field with the input advector */
    for (long k = 0; k < N; k++) xb[k] = 0.0;
    donor_pass_adj(g, psi_n, c, G, 0, yb, xb, Cb);
    for (long k = 0; k < N; k++) pnb[k] += xb[k];
    for (int d = 0; d < g->ndims; d++)
        for (long w = 0; w < walls(g, d); w++) cgrad[d][w] += Cb[d][w];
    rc = 0;
done:
    free_recs(rec, n_iters);
    free(y);
    free(yb);
    free(xb);
    free(bub);
    free(bdb);
    for (int d = 0; d < 3; d++) {
        free(Ab[d]);
        free(Vb[d]);
        free(Cb[d]);
    }
    return rc;
}

int orc_adjoint(int ndims, const long n[3], const int bc[3], int n_iters,
                unsigned opts, const double *psi0, const double *G,
                const double *c0, const double *c1, const double *c2,
                long n_steps, long ckpt_every, const double *lambda_T,
                double *grad_psi0, double *grad_c0, double *grad_c1,
                double *grad_c2)
{
    grid_t g;
    if (make_grid(&g, ndims, n, bc, opts)) return -1;
    if (n_iters < 1 || n_iters > 8 || n_steps < 1 || ckpt_every < 1) return -1;
    if (g.iga && n_iters > 2) return -1;
    if (g.abs || g.dfl) return -1;   /* reverse mode: not for the abs and dfl options */
    if (!psi0 || !lambda_T || !grad_psi0) return -1;
    double *c[3] = {(double *)c0, (double *)c1, (double *)c2};
    double *gc[3] = {grad_c0, grad_c1, grad_c2};
    for (int d = 0; d < ndims; d++)
        if (!c[d] || !gc[d]) return -1;
    long N = cells(&g);
    long nck = (n_steps + ckpt_every - 1) / ckpt_every;
    double *ck = malloc(sizeof(double) * N * nck);           /* checkpoints */
    double *seg = malloc(sizeof(double) * N * (ckpt_every + 1)); /* segment states */
    double *lam = malloc(sizeof(double) * N);
    double *lam2 = malloc(sizeof(double) * N);
    work_t w;
    int rc = -1;
    int have_w = work_alloc(&g, &w) == 0;
    if (!ck || !seg || !lam || !lam2 || !have_w) goto out;

    /* forward sweep keeping a checkpoint at the start of each segment */
    memcpy(seg, psi0, sizeof(double) * N);
    for (long s = 0; s < n_steps; s++) {
        if (s % ckpt_every == 0) memcpy(ck + (s / ckpt_every) * N, seg, sizeof(double) * N);
        memcpy(seg + N, seg, sizeof(double) * N);
        one_step(&g, n_iters, seg + N, G, c, &w, seg);
    }
    for (int d = 0; d < ndims; d++) memset(gc[d], 0, sizeof(double) * walls(&g, d));
    memcpy(lam, lambda_T, sizeof(double) * N);

    /* reverse sweep, segment by segment, recomputing the states inside */
    for (long sg = nck - 1; sg >= 0; sg--) {
        long s0 = sg * ckpt_every;
        long s1 = s0 + ckpt_every < n_steps ? s0 + ckpt_every : n_steps;
        memcpy(seg, ck + sg * N, sizeof(double) * N);
        for (long s = s0; s < s1 - 1; s++)
            one_step(&g, n_iters, seg + (s - s0) * N, G, c, &w, seg + (s - s0 + 1) * N);
        for (long s = s1 - 1; s >= s0; s--) {
            if (adjoint_step(&g, n_iters, seg + (s - s0) * N, G, c, lam, lam2, gc)) goto out;
            memcpy(lam, lam2, sizeof(double) * N);
        }
    }
    memcpy(grad_psi0, lam, sizeof(double) * N);
    /* periodic: wall n_d is wall 0; its gradient is reported in entry 0 */
    for (int d = 0; d < ndims; d++) {
        if (g.bc[d] != ORC_BC_PERIODIC) continue;
        long e[3] = {g.n[0], g.n[1], g.n[2]};
        e[d] += 1;
        long p[3];
        for (p[0] = 0; p[0] < e[0]; p[0]++)
            for (p[1] = 0; p[1] < e[1]; p[1]++)
                for (p[2] = 0; p[2] < e[2]; p[2]++)
                    if (p[d] == g.n[d]) gc[d][(p[0] * e[1] + p[1]) * e[2] + p[2]] = 0.0;
    }
    rc = 0;
out:
    free(ck);
    free(seg);
    free(lam);
    free(lam2);
    if (have_w) work_free(&w);
    return rc;
}
