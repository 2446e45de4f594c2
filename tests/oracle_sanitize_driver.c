/* Driver for the sanitizer run of the oracle (test infrastructure): calls
 * every oracle entry point over the grid shapes, boundary types and option
 * sets the tests use, on exactly sized heap arrays, so that AddressSanitizer
 * sees any read or write outside them and UndefinedBehaviorSanitizer any
 * undefined arithmetic.  Exit status 0 when every call returned as
 * expected. */
#include <stdio.h>
#include <stdlib.h>

#include "mpdata_oracle.h"

static unsigned long long rng = 88172645463325252ull;

static double uni(double lo, double hi)
{
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return lo + (hi - lo) * (double)(rng >> 11) / 9007199254740992.0;
}

static double *arr(long m, double lo, double hi)
{
    double *a = malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    if (!a) exit(3);
    for (long i = 0; i < m; i++) a[i] = uni(lo, hi);
    return a;
}

static int fails = 0;

static void expect(int rc, int want, const char *what)
{
    if (rc != want) {
        fprintf(stderr, "%s: returned %d, expected %d\n", what, rc, want);
        fails++;
    }
}

static void run_case(int nd, const long n[3], const int bc[3], int n_iters, unsigned opts,
                     int with_g, int adjoint)
{
    long cells = 1;
    for (int d = 0; d < nd; d++) cells *= n[d];
    long walls[3] = {0, 0, 0};
    for (int d = 0; d < nd; d++) walls[d] = cells / n[d] * (n[d] + 1);
    const int vs = (opts & (ORC_OPT_IGA | ORC_OPT_ABS)) != 0;
    double *psi = arr(cells, vs ? -1.0 : 0.0, 1.0);
    double *g = with_g ? arr(cells, 0.7, 1.3) : NULL;
    double *c[3] = {NULL, NULL, NULL};
    for (int d = 0; d < nd; d++) c[d] = arr(walls[d], -0.4 / nd, 0.4 / nd);
    int want = ((opts & ORC_OPT_IGA) && (opts & ORC_OPT_ABS)) ? -1 : 0;
    expect(orc_step(nd, n, bc, n_iters, opts, psi, g, c[0], c[1], c[2], 3), want, "orc_step");
    double out[3];
    long bad = 0;
    expect(orc_diag(nd, n, psi, g, out, &bad), 0, "orc_diag");
    double cm = 0.0;
    expect(orc_courant_max(nd, n, bc, g, c[0], c[1], c[2], &cm), 0, "orc_courant_max");
    if (adjoint) {
        double *lam = arr(cells, -1.0, 1.0), *gp = arr(cells, 0.0, 0.0);
        double *gc[3] = {NULL, NULL, NULL};
        for (int d = 0; d < nd; d++) gc[d] = arr(walls[d], 0.0, 0.0);
        int wa = (opts & (ORC_OPT_ABS | ORC_OPT_DFL)) ? -1 : 0;
        expect(orc_adjoint(nd, n, bc, n_iters, opts, psi, g, c[0], c[1], c[2], 4, 2, lam, gp,
                           gc[0], gc[1], gc[2]),
               wa, "orc_adjoint");
        free(lam);
        free(gp);
        for (int d = 0; d < nd; d++) free(gc[d]);
    }
    free(psi);
    free(g);
    for (int d = 0; d < nd; d++) free(c[d]);
}

int main(void)
{
    const long shapes[][4] = {{1, 7, 1, 1},   {1, 3, 1, 1},  {2, 5, 4, 1},
                              {2, 3, 3, 1},   {2, 1, 6, 1},  {3, 4, 3, 5},
                              {3, 3, 3, 3}};
    const unsigned opts[] = {0,
                             ORC_OPT_FCT,
                             ORC_OPT_TOT,
                             ORC_OPT_IGA,
                             ORC_OPT_IGA | ORC_OPT_TOT | ORC_OPT_FCT,
                             ORC_OPT_ABS | ORC_OPT_FCT,
                             ORC_OPT_ABS | ORC_OPT_IGA,
                             ORC_OPT_DFL | ORC_OPT_FCT,
                             ORC_OPT_DFL | ORC_OPT_IGA | ORC_OPT_FCT,
                             ORC_OPT_KAHAN | ORC_OPT_FCT | ORC_OPT_TOT};
    for (size_t s = 0; s < sizeof shapes / sizeof shapes[0]; s++) {
        const int nd = (int)shapes[s][0];
        const long n[3] = {shapes[s][1], shapes[s][2], shapes[s][3]};
        for (int b = 0; b < 2; b++) {
            int bc[3] = {b, b, b};
            int periodic_ok = 1;
            for (int d = 0; d < nd; d++)
                if (n[d] < 3) periodic_ok = 0;
            if (b == ORC_BC_PERIODIC && !periodic_ok) continue;
            for (size_t o = 0; o < sizeof opts / sizeof opts[0]; o++)
                for (int with_g = 0; with_g < 2; with_g++)
                    for (int ni = 1; ni <= 3; ni++) {
                        if ((opts[o] & ORC_OPT_IGA) && ni > 2) continue;
                        run_case(nd, n, bc, ni, opts[o], with_g, ni >= 2);
                    }
        }
    }
    if (fails) {
        fprintf(stderr, "%d unexpected return codes\n", fails);
        return 1;
    }
    printf("oracle sanitizer run: all calls returned as expected\n");
    return 0;
}
