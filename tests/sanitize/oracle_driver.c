/* Drives the oracle through its entry points on small grids (1D and 2D;
 * periodic, wall, outflow and forced-source ends; both fluxes; the stiff
 * branch) so that a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer can check every
 * ghost-cell index and array access.  Exit status 0 when every run returns
 * OR_OK; the sanitizers abort on any invalid access. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "../../oracle/muscl_oracle.c"

static int run_case(int64_t nx, int64_t ny, const int32_t bc[4], int riemann, double tau0)
{
    or_gas g = {1.4, 1.0, 1.0, 1.0, 1.0, tau0, -1.0, -1.0, 0.1, 0.5, 2.0, 0.1, 1.0, 2.0, 0.0, 0.0};
    /* a source segment and an active wedge whenever the x-low end is a source */
    or_grid gr = {nx, ny, 1.0 / (double)nx, {bc[0], bc[1], bc[2], bc[3]}, 0.01, 0.1,
                  0.5, 0.2, 0.0, 0.5, bc[0] == OR_BC_SOURCE && ny > 1 ? 0.3 : 0.0};
    or_num nm = {0.4, riemann, 0.5};
    const int64_t n = nx * ny;
    double* W = malloc(sizeof(double) * 5 * n);
    double* U = malloc(sizeof(double) * 5 * n);
    for (int64_t k = 0; k < ny; k++)
        for (int64_t j = 0; j < nx; j++) {
            const int64_t i = k * nx + j;
            const double x = (j + 0.5) / (double)nx, y = (k + 0.5) / (double)ny;
            W[i] = 1.0 + 0.2 * sin(6.283185307179586 * x) * cos(6.283185307179586 * y);
            W[n + i] = 0.3 * cos(6.283185307179586 * x);
            W[2 * n + i] = ny > 1 ? 0.2 * sin(6.283185307179586 * y) : 0.0;
            W[3 * n + i] = 1.0 + 0.1 * cos(6.283185307179586 * (x + y));
            W[4 * n + i] = 1.005 * W[i];
        }
    or_prim_to_cons(&g, n, W, U);
    double t = 0.0, budget[2] = {0.0, 0.0}, dt_last = 0.0;
    int64_t steps = 0;
    int st = or_run(&g, &gr, &nm, U, 25, 0.0, &t, &steps, budget, &dt_last);
    free(W);
    free(U);
    if (st != OR_OK || steps != 25) {
        fprintf(stderr, "case nx=%lld ny=%lld failed: %d\n", (long long)nx, (long long)ny, st);
        return 1;
    }
    return 0;
}

int main(void)
{
    const int32_t kinds[4][4] = {{OR_BC_PERIODIC, OR_BC_PERIODIC, OR_BC_PERIODIC, OR_BC_PERIODIC},
                                 {OR_BC_WALL, OR_BC_WALL, OR_BC_OUTFLOW, OR_BC_OUTFLOW},
                                 {OR_BC_OUTFLOW, OR_BC_WALL, OR_BC_WALL, OR_BC_OUTFLOW},
                                 {OR_BC_SOURCE, OR_BC_OUTFLOW, OR_BC_WALL, OR_BC_PERIODIC}};
    int bad = 0;
    for (int b = 0; b < 4; b++)
        for (int riemann = 0; riemann < 2; riemann++) {
            bad += run_case(37, 1, kinds[b], riemann, 0.05);
            bad += run_case(4, 1, kinds[b], riemann, 0.05);
            bad += run_case(23, 17, kinds[b], riemann, 0.05);
            bad += run_case(4, 5, kinds[b], riemann, 1e-4);   /* stiff branch */
        }
    printf("oracle driver: %d failures\n", bad);
    return bad ? 1 : 0;
}
