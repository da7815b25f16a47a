/* Drives the CSPH-TVD oracle on small 1D grids (periodic, wall and outflow
 * ends, mixed, a forced source; 4 cells to a few segments of particles) so
 * that a build with AddressSanitizer and UndefinedBehaviorSanitizer checks
 * every ghost-particle index and array access of its extended arrays.  A 2D
 * grid must be refused (OR_EINVAL) without touching the state.  Exit status 0 when
 * every run behaves; the sanitizers abort on any invalid access. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "../../oracle/csph_oracle.c"

static int run_case(int64_t nx, const int32_t bc[4], double fx)
{
    /* tau0 = 0.5: the sources are explicit, and on 4 cells dt of eq. (16) is 0.1 */
    or_gas g = {1.4, 1.0, 1.0, 1.0, 1.0, 0.5, -1.0, -1.0, 0.1, 0.5, 2.0, 0.1, 1.0, 2.0, fx, 0.0};
    or_grid gr = {nx, 1, 1.0 / (double)nx, {bc[0], bc[1], bc[2], bc[3]}, 0.01, 0.1,
                  0.0, 0.0, 0.0, 0.0, 0.0};
    or_num nm = {0.4, 1, 0.5};
    double* W = malloc(sizeof(double) * 5 * nx);
    double* U = malloc(sizeof(double) * 5 * nx);
    for (int64_t j = 0; j < nx; j++) {
        const double x = (j + 0.5) / (double)nx;
        W[j] = 1.0 + 0.05 * sin(6.283185307179586 * x);
        W[nx + j] = 0.05 * cos(6.283185307179586 * x);
        W[2 * nx + j] = 0.0;
        W[3 * nx + j] = 1.0 + 0.05 * cos(6.283185307179586 * 2.0 * x);
        W[4 * nx + j] = 1.005 * W[j];
    }
    or_prim_to_cons(&g, nx, W, U);
    double t = 0.0, budget[2] = {0.0, 0.0}, dt_last = 0.0;
    int64_t steps = 0;
    int st = cs_run(&g, &gr, &nm, U, 25, 0.0, &t, &steps, budget, &dt_last);
    /* one step with the displacements read back */
    double* V = malloc(sizeof(double) * 5 * nx);
    double* xi = malloc(sizeof(double) * nx);
    double src[2];
    int st2 = st == OR_OK ? cs_step(&g, &gr, &nm, U, V, t, 1e-4, src, xi) : st;
    free(W);
    free(U);
    free(V);
    free(xi);
    if (st != OR_OK || steps != 25 || st2 != OR_OK) {
        fprintf(stderr, "case nx=%lld failed: %d %d\n", (long long)nx, st, st2);
        return 1;
    }
    return 0;
}

static int refused(int64_t nx, int64_t ny, const int32_t bc[4])
{
    or_gas g = {1.4, 1.0, 1.0, 1.0, 1.0, 0.05, -1.0, -1.0, 0.1, 0.5, 2.0, 0.1, 1.0, 2.0, 0.0, 0.0};
    or_grid gr = {nx, ny, 1.0 / (double)nx, {bc[0], bc[1], bc[2], bc[3]}, 0.01, 0.1,
                  0.0, 0.0, 0.0, 0.0, 0.0};
    or_num nm = {0.4, 1, 0.5};
    double* U = calloc((size_t)(5 * nx * ny), sizeof(double));
    double* V = calloc((size_t)(5 * nx * ny), sizeof(double));
    double src[2];
    int st = cs_step(&g, &gr, &nm, U, V, 0.0, 1e-3, src, NULL);
    free(U);
    free(V);
    return st == OR_EINVAL ? 0 : 1;
}

int main(void)
{
    const int32_t kinds[6][4] = {{OR_BC_PERIODIC, OR_BC_PERIODIC, 0, 0},
                                 {OR_BC_WALL, OR_BC_WALL, 0, 0},
                                 {OR_BC_OUTFLOW, OR_BC_OUTFLOW, 0, 0},
                                 {OR_BC_WALL, OR_BC_OUTFLOW, 0, 0},
                                 {OR_BC_OUTFLOW, OR_BC_WALL, 0, 0},
                                 {OR_BC_SOURCE, OR_BC_OUTFLOW, 0, 0}};
    const int64_t sizes[5] = {4, 5, 37, 59, 120};
    int bad = 0;
    for (int b = 0; b < 6; b++)
        for (int s = 0; s < 5; s++) bad += run_case(sizes[s], kinds[b], b == 1 ? -2.0 : 0.5);
    const int32_t per[4] = {OR_BC_PERIODIC, OR_BC_PERIODIC, OR_BC_PERIODIC, OR_BC_PERIODIC};
    bad += refused(16, 16, per);
    printf("csph driver: %d failures\n", bad);
    return bad ? 1 : 0;
}
