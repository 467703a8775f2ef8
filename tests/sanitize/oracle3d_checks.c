/* Drives the FP64 D3Q14 oracle on the smallest and ragged periodic boxes, with
 * and without initial heat flux, for the AddressSanitizer /
 * UndefinedBehaviorSanitizer build of the CPU tests.  Exit status 0 when every
 * call returns and the results are finite. */
#include "../../oracle/phonon_oracle_d3q14.c"

#include <stdio.h>
#include <stdlib.h>

static int finite_all(const double* v, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

int main(void)
{
    const int boxes[][3] = {{1, 1, 1}, {2, 1, 1}, {1, 5, 3}, {3, 2, 2}, {9, 4, 3}, {65, 2, 2}};
    const double taus[][2] = {{0.6, 5.0}, {0.55, INFINITY}, {2.3, 0.2}};
    int bad = 0, ran = 0;
    for (size_t b = 0; b < sizeof boxes / sizeof boxes[0]; ++b)
        for (size_t t = 0; t < sizeof taus / sizeof taus[0]; ++t) {
            ora3_case c;
            memset(&c, 0, sizeof c);
            c.nx = boxes[b][0];
            c.ny = boxes[b][1];
            c.nz = boxes[b][2];
            c.tau_n = taus[t][0];
            c.tau_r = taus[t][1];
            c.cv = 0.7;
            c.t0 = 1.0;
            if (ora3_check(&c) != 0) continue;
            const size_t n = (size_t)c.nx * c.ny * c.nz;
            double* f[4];
            for (int k = 0; k < 4; ++k) f[k] = malloc(n * sizeof(double));
            double* e = malloc(14 * n * sizeof(double));
            double* w = malloc(14 * n * sizeof(double));
            for (size_t i = 0; i < n; ++i) {
                f[0][i] = 1.0 + 0.01 * sin(0.3 * (double)i);
                f[1][i] = 1e-3 * cos(0.1 * (double)i);
                f[2][i] = 1e-3 * sin(0.2 * (double)i);
                f[3][i] = -1e-3 * cos(0.05 * (double)i);
            }
            const int flux = (int)((b + t) & 1);
            ora3_init(&c, f[0], flux ? f[1] : NULL, flux ? f[2] : NULL, flux ? f[3] : NULL, e);
            ora3_run(&c, e, w, 5);
            ora3_moments(&c, e, f[0], f[1], f[2], f[3]);
            double tot[4];
            ora3_totals(&c, e, tot);
            for (int k = 0; k < 4; ++k) bad |= !finite_all(f[k], n);
            bad |= !finite_all(tot, 4);
            double node[14], post[14];
            for (int i = 0; i < 14; ++i) node[i] = e[(size_t)i * n];
            ora3_collide_node(&c, node, post);
            bad |= !finite_all(post, 14);
            for (int k = 0; k < 4; ++k) free(f[k]);
            free(e);
            free(w);
            ++ran;
        }
    printf("oracle3d sanitizer checks: %d cases, %s\n", ran, bad ? "NON-FINITE RESULT" : "ok");
    return bad;
}
