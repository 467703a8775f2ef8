/*
 * phonon_oracle_d3q14.c -- plain FP64 reference time-stepper for the
 * three-dimensional (D3Q14) phonon lattice Boltzmann equation on a fully
 * periodic grid.
 *
 * TEST INFRASTRUCTURE ONLY.  Like the D2Q8 stepper beside it, this file is an
 * oracle: only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark load it, and it shares no source, header, table or helper with
 * the product library.
 *
 * The paper derives the scheme on the D2Q8 lattice and states that the same
 * derivation carries over to D3Q14 (Sec. 2.2) without giving its weights.
 * Here the scheme keeps every formula of Sec. 2.2-2.4 -- the update of Eq. 13,
 * the equilibrium of Eq. 15, the source of Eq. 16, the heat flux of Eqs.
 * 19/54, c = sqrt(3/5) v_g (Eq. 48) and tau = tau_C/dt + 1/2 (Eq. 49) -- and
 * only the velocity set and the weights change:
 *
 *   velocities (c = 1): 6 axis movers (+-1,0,0), (0,+-1,0), (0,0,+-1) and
 *   8 corner movers (+-1,+-1,+-1); no rest population (Sec. 2.2 drops it for
 *   phonons on D2Q8 as well).
 *
 *   weights: the Chapman-Enskog recovery of Eq. 47 uses only the moment
 *   identities Eqs. 22-25 of the equilibrium and Eqs. 26-28 of the source.
 *   With the forms of Eqs. 15-16 they hold if and only if
 *       sum_i omega_i = 1,   sum_i omega_i c_ia c_ib = (5/9) delta_ab,
 *       sum_i a_i c_ia c_ib = (3/5) delta_ab,
 *       sum_i a_i c_ia c_ib c_ig c_id = (1/5) (d_ab d_gd + d_ag d_bd + d_ad d_bg)
 *   (odd moments vanish by symmetry).  On the 6 + 8 velocities these read
 *       6 w_a + 8 w_c = 1,  2 w_a + 8 w_c = 5/9   ->  w_a = 1/9,  w_c = 1/24,
 *       2 a_a + 8 a_c = 3/5 (the xx and xxxx moments),  8 a_c = 1/5 (xxyy)
 *                                                  ->  a_a = 1/5,  a_c = 1/40,
 *   the unique solution.  (On D2Q8 the same four conditions give Eqs. 17-18.)
 *
 * State kept: the pre-collision distributions e_i(x, t) at the start of a step,
 * FP64.  One step: moments (Eqs. 53-54), equilibrium and source (Eqs. 15-16),
 * relaxation (Eq. 13 right-hand side), periodic advection (Eq. 13 left-hand
 * side).  Lattice units dx = dt = c = 1.
 *
 * Layout: e[i][z][y][x], x fastest; direction order below.  OpenMP
 * parallelises over planes only; there is no blocking or fusion.
 */
#include <math.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int nx, ny, nz;
    double tau_n, tau_r;   /* tau_N/dt, tau_R/dt (tau_r may be +inf) */
    double cv;             /* volumetric heat capacity C_V */
    double t0;             /* reference temperature for the totals */
} ora3_case;

#define Q3 14

/* Velocities: 0..5 the axis movers +x -x +y -y +z -z, 6..13 the corner movers. */
static const int C3X[Q3] = {1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
static const int C3Y[Q3] = {0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1};
static const int C3Z[Q3] = {0, 0, 0, 0, 1, -1, 1, 1, 1, 1, -1, -1, -1, -1};

/* Weights of the equilibrium (omega_i) and of the flux terms (a_i), derived in
 * the header comment from Eqs. 22-28. */
static double omega3(int i) { return i < 6 ? 1.0 / 9.0 : 1.0 / 24.0; }
static double a3(int i) { return i < 6 ? 1.0 / 5.0 : 1.0 / 40.0; }

#define IDX3(c, i, x, y, z) \
    ((((size_t)(i) * (size_t)(c)->nz + (size_t)(z)) * (size_t)(c)->ny + (size_t)(y)) * (size_t)(c)->nx + (size_t)(x))

int ora3_check(const ora3_case* c)
{
    if (!c || c->nx < 1 || c->ny < 1 || c->nz < 1) return -1;
    if (!(c->tau_n > 0.0) || !(c->tau_r > 0.0) || !(c->cv > 0.0)) return -1;
    return 0;
}

/* Eq. 49 with 1/tau_C = 1/tau_N + 1/tau_R (Sec. 2.1). */
static double ora3_tau(const ora3_case* c)
{
    return 1.0 / (1.0 / c->tau_n + 1.0 / c->tau_r) + 0.5;
}

/* Eq. 54: q = 2 tau_r / (2 tau_r + 1) * sum_i c_i e_i. */
static double ora3_qfactor(const ora3_case* c)
{
    if (isinf(c->tau_r)) return 1.0;
    return 2.0 * c->tau_r / (2.0 * c->tau_r + 1.0);
}

/* One node's relaxation, Eq. 13 right-hand side with Eqs. 15-16 (c = dt = 1). */
void ora3_collide_node(const ora3_case* c, const double* e_in, double* e_out)
{
    const double tau = ora3_tau(c);
    double e = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
    for (int i = 0; i < Q3; ++i) {
        e += e_in[i];                       /* Eq. 53 */
        jx += C3X[i] * e_in[i];
        jy += C3Y[i] * e_in[i];
        jz += C3Z[i] * e_in[i];
    }
    const double T = e / c->cv;
    const double qf = ora3_qfactor(c);      /* Eq. 54 */
    const double qx = qf * jx, qy = qf * jy, qz = qf * jz;
    for (int i = 0; i < Q3; ++i) {
        const double ciq = C3X[i] * qx + C3Y[i] * qy + C3Z[i] * qz;
        const double eeq = omega3(i) * c->cv * T + 5.0 * a3(i) * ciq / 3.0;          /* Eq. 15 */
        const double S = isinf(c->tau_r) ? 0.0
                       : -(1.0 - 1.0 / (2.0 * tau)) * 5.0 * a3(i) * ciq / (3.0 * c->tau_r);  /* Eq. 16 */
        e_out[i] = e_in[i] + (eeq - e_in[i]) / tau + S;                               /* Eq. 13 */
    }
}

/* Equilibrium initial state (n = 0) of Eq. 15 for temperature T and heat flux
 * q: the flux term carries q / beta so that Eq. 54 returns q at n = 0.  T,
 * qx, qy, qz: nz*ny*nx arrays (x fastest); a NULL flux component is zero. */
void ora3_init(const ora3_case* c, const double* T, const double* qx, const double* qy,
               const double* qz, double* e)
{
    const double qf = ora3_qfactor(c);
    const size_t n = (size_t)c->nx * c->ny * c->nz;
    for (size_t k = 0; k < n; ++k) {
        const double jx = qx ? qx[k] / qf : 0.0;
        const double jy = qy ? qy[k] / qf : 0.0;
        const double jz = qz ? qz[k] / qf : 0.0;
        for (int i = 0; i < Q3; ++i)
            e[(size_t)i * n + k] = omega3(i) * c->cv * T[k]
                                 + 5.0 * a3(i) * (C3X[i] * jx + C3Y[i] * jy + C3Z[i] * jz) / 3.0;
    }
}

static int wrap(int v, int n) { return ((v % n) + n) % n; }

/* nsteps steps: relaxation of every node into work, then periodic advection
 * e_i(x + c_i) <- work_i(x). */
void ora3_run(const ora3_case* c, double* e, double* work, long nsteps)
{
    const int nx = c->nx, ny = c->ny, nz = c->nz;
    for (long s = 0; s < nsteps; ++s) {
#pragma omp parallel for schedule(static)
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    double in[Q3], out[Q3];
                    for (int i = 0; i < Q3; ++i) in[i] = e[IDX3(c, i, x, y, z)];
                    ora3_collide_node(c, in, out);
                    for (int i = 0; i < Q3; ++i) work[IDX3(c, i, x, y, z)] = out[i];
                }
#pragma omp parallel for schedule(static)
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x)
                    for (int i = 0; i < Q3; ++i) {
                        const int xd = wrap(x + C3X[i], nx), yd = wrap(y + C3Y[i], ny),
                                  zd = wrap(z + C3Z[i], nz);
                        e[IDX3(c, i, xd, yd, zd)] = work[IDX3(c, i, x, y, z)];
                    }
    }
}

/* T and q of the kept state (Eqs. 53-54). */
void ora3_moments(const ora3_case* c, const double* e, double* T, double* qx, double* qy,
                  double* qz)
{
    const double qf = ora3_qfactor(c);
    const size_t n = (size_t)c->nx * c->ny * c->nz;
    for (size_t k = 0; k < n; ++k) {
        double s = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
        for (int i = 0; i < Q3; ++i) {
            const double v = e[(size_t)i * n + k];
            s += v;
            jx += C3X[i] * v;
            jy += C3Y[i] * v;
            jz += C3Z[i] * v;
        }
        if (T) T[k] = s / c->cv;
        if (qx) qx[k] = qf * jx;
        if (qy) qy[k] = qf * jy;
        if (qz) qz[k] = qf * jz;
    }
}

/* out[0] = sum over nodes of (C_V T - C_V t0), out[1..3] = sum of q. */
void ora3_totals(const ora3_case* c, const double* e, double out[4])
{
    const double qf = ora3_qfactor(c);
    const size_t n = (size_t)c->nx * c->ny * c->nz;
    double s = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
    for (size_t k = 0; k < n; ++k)
        for (int i = 0; i < Q3; ++i) {
            const double v = e[(size_t)i * n + k];
            s += v;
            jx += C3X[i] * v;
            jy += C3Y[i] * v;
            jz += C3Z[i] * v;
        }
    out[0] = s - c->cv * c->t0 * (double)n;
    out[1] = qf * jx;
    out[2] = qf * jy;
    out[3] = qf * jz;
}
