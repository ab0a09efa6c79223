/* CPU self test of the oracle's C line operator (oracle/lines.c) under
 * AddressSanitizer and UndefinedBehaviorSanitizer: every direction of small
 * closure and periodic blocks, tridiagonal and pentadiagonal rows, explicit
 * stencils, lines as short as the closure allows.  The sanitizers abort on
 * any out-of-bounds access, leak or undefined behaviour. */
#include <stdio.h>
#include <stdlib.h>

int orc_block_dir(int nx, int ny, int nz, int ng, int dir, int periodic, int d, double h, int nl,
                  const double *alpha, int M, const double *a, int nc, int mc, const double *cbar,
                  const double *in, double *out, int nthreads);

int main(void) {
    /* tridiagonal (alpha = 1/3, Pade-like) and pentadiagonal coefficient sets; values need not be a
       real scheme for a memory check, only well conditioned */
    const double alpha3[3] = {0.3, 1.0, 0.3};
    const double alpha5[5] = {0.05, 0.4, 1.0, 0.4, 0.05};
    const double alpha1[1] = {1.0};
    double a[11], cbar[22];
    for (int i = 0; i < 11; ++i) a[i] = 0.01 * (i - 5);
    for (int i = 0; i < 22; ++i) cbar[i] = 0.02 * ((i % 11) - 5);
    int fails = 0;
    const int shapes[][3] = {{3, 4, 5}, {7, 3, 9}, {12, 10, 3}, {5, 5, 5}};
    for (int sh = 0; sh < 4; ++sh)
        for (int nl = 0; nl <= 2; ++nl)
            for (int periodic = 0; periodic <= 1; ++periodic)
                for (int dir = 0; dir < 3; ++dir) {
                    const int nx = shapes[sh][0], ny = shapes[sh][1], nz = shapes[sh][2], ng = 5;
                    const int n[3] = {nx, ny, nz};
                    const int M = 3, nc = nl, mc = 5;
                    if (!periodic && n[dir] < 2 * nc + 1) continue;
                    if (periodic && n[dir] < 2 * nl + 1) continue;
                    const long nin = (long)(nx + 2 * ng) * (ny + 2 * ng) * (nz + 2 * ng);
                    double *in = (double *)malloc(sizeof(double) * nin);
                    double *out = (double *)malloc(sizeof(double) * nx * ny * nz);
                    for (long i = 0; i < nin; ++i) in[i] = (double)((i * 7919) % 101) / 101.0;
                    const double *al = nl == 0 ? alpha1 : nl == 1 ? alpha3 : alpha5;
                    const double *ac = a + 5 - M;
                    const int rc = orc_block_dir(nx, ny, nz, ng, dir, periodic, 1, 0.1, nl, al, M, ac, nc, mc,
                                                 cbar, in, out, 2);
                    if (rc) {
                        printf("orc_block_dir failed: shape %d nl %d periodic %d dir %d rc %d\n", sh, nl, periodic,
                               dir, rc);
                        ++fails;
                    }
                    free(in);
                    free(out);
                }
    printf("%s (%d failures)\n", fails ? "FAIL" : "OK", fails);
    return fails ? 1 : 0;
}
