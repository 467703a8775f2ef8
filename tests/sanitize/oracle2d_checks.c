/* Drives the FP64 D2Q8 oracle through every boundary kind, the smallest and
 * ragged grids, initial heat flux, wall-flux changes, moments and totals, for
 * the AddressSanitizer / UndefinedBehaviorSanitizer build of the CPU tests.
 * Exit status 0 when every call returns and the results are finite. */
#include "../../oracle/phonon_oracle.c"

#include <stdio.h>
#include <stdlib.h>

static int finite_all(const double* v, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

static int run_case(ora_case c, int with_flux, long steps)
{
    if (ora_check(&c) != 0) return 0;   /* rejected combinations are fine */
    const size_t n = (size_t)c.nx * c.ny;
    double* T = malloc(n * sizeof *T);
    double* qx = malloc(n * sizeof *qx);
    double* qy = malloc(n * sizeof *qy);
    double* e = malloc(8 * n * sizeof *e);
    double* w = malloc(8 * n * sizeof *w);
    double out[3];
    int bad = 0;
    for (size_t i = 0; i < n; ++i) {
        T[i] = c.t0 + 0.01 * sin(0.37 * (double)i);
        qx[i] = 1e-3 * cos(0.11 * (double)i);
        qy[i] = -1e-3 * sin(0.23 * (double)i);
    }
    ora_init(&c, T, with_flux ? qx : NULL, with_flux ? qy : NULL, e);
    ora_run(&c, e, w, steps);
    for (int k = 0; k < 4; ++k) c.q_wall[k] = -c.q_wall[k];
    ora_run(&c, e, w, steps);
    ora_moments(&c, e, T, qx, qy);
    ora_totals(&c, e, out);
    if (!finite_all(T, n) || !finite_all(qx, n) || !finite_all(qy, n) || !finite_all(out, 3)) bad = 1;
    double node[8], post[8];
    for (int i = 0; i < 8; ++i) node[i] = e[i * n];
    ora_collide_node(&c, node, post);
    if (!finite_all(post, 8)) bad = 1;
    free(T); free(qx); free(qy); free(e); free(w);
    return bad;
}

int main(void)
{
    const int sizes[][2] = {{2, 2}, {2, 5}, {3, 2}, {5, 3}, {17, 9}, {64, 2}, {65, 3}};
    const int kinds[][2] = {{ORA_PERIODIC, ORA_PERIODIC}, {ORA_ISOTHERMAL, ORA_PERIODIC},
                            {ORA_PERIODIC, ORA_DIFFUSE}, {ORA_GRADIENT, ORA_DIFFUSE},
                            {ORA_HEATFLUX, ORA_PERIODIC}, {ORA_PERIODIC, ORA_HEATFLUX},
                            {ORA_ISOTHERMAL, ORA_ISOTHERMAL}, {ORA_ISOTHERMAL, ORA_DIFFUSE}};
    const double taus[][2] = {{0.6, 0.8}, {0.51, INFINITY}, {2.3, 0.2}};
    int bad = 0, ran = 0;
    ora_set_threads(3);
    for (size_t s = 0; s < sizeof sizes / sizeof sizes[0]; ++s)
        for (size_t k = 0; k < sizeof kinds / sizeof kinds[0]; ++k)
            for (size_t t = 0; t < sizeof taus / sizeof taus[0]; ++t) {
                ora_case c;
                memset(&c, 0, sizeof c);
                c.nx = sizes[s][0];
                c.ny = sizes[s][1];
                c.tau_n = taus[t][0];
                c.tau_r = taus[t][1];
                c.cv = 1.3;
                c.bc_x = kinds[k][0];
                c.bc_y = kinds[k][1];
                c.t0 = 1.0;
                c.grad_x = c.bc_x == ORA_GRADIENT ? 1e-3 : 0.0;
                for (int w = 0; w < 4; ++w) {
                    c.t_wall[w] = 1.0 + 0.01 * (w - 1.5);
                    c.q_wall[w] = 1e-3 * (w + 1);
                }
                if (kinds[k][0] == ORA_ISOTHERMAL && kinds[k][1] == ORA_ISOTHERMAL) c.wall_kind[3] = ORA_HEATFLUX;
                bad |= run_case(c, (int)((s + k) & 1), 7);
                ++ran;
            }
    printf("oracle2d sanitizer checks: %d cases, %s\n", ran, bad ? "NON-FINITE RESULT" : "ok");
    return bad;
}
