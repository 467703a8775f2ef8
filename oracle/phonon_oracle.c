/*
 * phonon_oracle.c -- plain FP64 reference time-stepper for the D2Q8 phonon
 * lattice Boltzmann equation under Callaway's dual relaxation model
 * (Guo & Wang, "Lattice Boltzmann scheme for hydrodynamic equation of phonon
 * transport", Sec. 2.2-2.5).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle the HIP path is checked
 * against.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark load it; the product library never links or calls it, and it
 * shares no source, header, table or helper with the product.
 *
 * It is deliberately slow and literal:
 *   - state kept: the absolute energy-density distributions e_i(x, t) at the
 *     start of a time step (after advection and boundary treatment), FP64;
 *   - one step, in the paper's order: moments (Eqs. 53-54) -> equilibrium
 *     (Eq. 15) and source (Eq. 16) -> relaxation (Eq. 13 right-hand side) ->
 *     advection (Eq. 13 left-hand side) -> boundary treatment of the unknown
 *     populations after advection (Sec. 2.5: Eqs. 55, 57, 58, 59-60);
 *   - lattice units: dx = dt = c = 1 (so the group speed is sqrt(5/3), Eq. 48),
 *     tau = tau_C/dt + 1/2 (Eq. 49) with 1/tau_C = 1/tau_N + 1/tau_R (Sec. 2.1),
 *     tau_r = tau_R/dt (Sec. 2.4).
 *
 * Layout: e[i][y][x], i = 0..7 for the paper's directions 1..8, x fastest.
 * OpenMP parallelises over rows only; there is no blocking or fusion.
 */
#include <math.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Boundary kinds (Sec. 2.5). */
enum { ORA_PERIODIC = 0, ORA_ISOTHERMAL = 1, ORA_DIFFUSE = 2, ORA_GRADIENT = 3, ORA_HEATFLUX = 4 };

typedef struct {
    int nx, ny;
    double tau_n, tau_r;   /* tau_N/dt, tau_R/dt */
    double cv;             /* volumetric heat capacity C_V */
    int bc_x, bc_y;
    double t0;             /* reference temperature (at x = 0 for the gradient seam) */
    double grad_x;         /* gradient seam: temperature drop per node along +x */
    double t_wall[4];      /* isothermal walls: x=0, x=nx-1, y=0, y=ny-1 */
    double q_wall[4];      /* heat-flux walls: heat flux q_0 into the domain (Eq. 56), same order */
    int wall_kind[4];      /* kind of each wall, same order; 0 = the kind of its axis */
} ora_case;

/* D2Q8 velocities, Eq. 14 with c = 1, in the paper's numbering 1..8
 * (1:+x 2:+y 3:-x 4:-y 5:(+,+) 6:(-,+) 7:(-,-) 8:(+,-)); the +x set {1,5,8}
 * and -x set {3,6,7} are the ones Eqs. 59-60 name. */
static const int CX[8] = {1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[8] = {0, 1, 0, -1, 1, 1, -1, -1};

/* Weights of Eq. 17 (omega_i) and Eq. 18 (a_i). */
static double omega_w(int i) { return i < 4 ? 2.0 / 9.0 : 1.0 / 36.0; }
static double a_w(int i) { return i < 4 ? 1.0 / 5.0 : 1.0 / 20.0; }

#define IDX(c, i, x, y) (((size_t)(i) * (size_t)(c)->ny + (size_t)(y)) * (size_t)(c)->nx + (size_t)(x))

static int is_wall_kind(int k) { return k == ORA_ISOTHERMAL || k == ORA_DIFFUSE || k == ORA_HEATFLUX; }

/* Kind of wall w (0: x = 0, 1: x = nx-1, 2: y = 0, 3: y = ny-1). */
static int kind_of(const ora_case* c, int w)
{
    int k = c->wall_kind[w];
    return k ? k : (w < 2 ? c->bc_x : c->bc_y);
}

/* Validity of a case: sizes, relaxation times, and the boundary sets whose
 * treatment the paper defines.  The gradient seam is along x only, with
 * periodic, diffuse or heat-flux walls across it.  Corners (walls on both
 * axes) are not defined by the paper; they are accepted only when both x
 * walls are isothermal, which then own the corner nodes (the Sec. 3.1.2
 * square).  A per-wall kind may differ from its axis kind only on a walled
 * axis. */
int ora_check(const ora_case* c)
{
    if (!c || c->nx < 2 || c->ny < 2) return -1;
    if (!(c->tau_n > 0.0) || !(c->tau_r > 0.0) || !(c->cv > 0.0)) return -1;
    if (c->bc_x < 0 || c->bc_x > 4 || c->bc_y < 0 || c->bc_y > 4 || c->bc_y == ORA_GRADIENT) return -1;
    for (int w = 0; w < 4; ++w)
        if (c->wall_kind[w] && (!is_wall_kind(c->wall_kind[w]) || !is_wall_kind(w < 2 ? c->bc_x : c->bc_y)))
            return -1;
    int wx = is_wall_kind(c->bc_x), wy = is_wall_kind(c->bc_y);
    if (wx && wy && !(kind_of(c, 0) == ORA_ISOTHERMAL && kind_of(c, 1) == ORA_ISOTHERMAL)) return -2;
    if (c->bc_x == ORA_GRADIENT && (kind_of(c, 2) == ORA_ISOTHERMAL || kind_of(c, 3) == ORA_ISOTHERMAL))
        return -2;
    return 0;
}

/* Non-dimensional relaxation time of the single relaxation step, Eq. 49 with
 * the overall relaxation time of Sec. 2.1 (tau_r may be +inf). */
static double ora_tau(const ora_case* c)
{
    double inv_tc = 1.0 / c->tau_n + 1.0 / c->tau_r;
    return 1.0 / inv_tc + 0.5;
}

/* Prefactor of Eq. 54: q = 2 tau_r / (2 tau_r + 1) * sum_i c_i e_i. */
static double ora_qfactor(const ora_case* c)
{
    if (isinf(c->tau_r)) return 1.0;
    return 2.0 * c->tau_r / (2.0 * c->tau_r + 1.0);
}

/* Reference temperature of column x: t0, or the gradient ramp. */
static double ora_tref(const ora_case* c, int x)
{
    return c->bc_x == ORA_GRADIENT ? c->t0 - c->grad_x * (double)x : c->t0;
}

/* One node's relaxation: Eq. 13 right-hand side with Eqs. 15-16 (c = dt = 1).
 * e_in: 8 populations at the start of the step; e_out: post-collision. */
void ora_collide_node(const ora_case* c, const double* e_in, double* e_out)
{
    const double tau = ora_tau(c);
    /* Eq. 53: e = sum_i e_i = C_V T */
    double e = 0.0, jx = 0.0, jy = 0.0;
    for (int i = 0; i < 8; ++i) {
        e += e_in[i];
        jx += CX[i] * e_in[i];
        jy += CY[i] * e_in[i];
    }
    const double T = e / c->cv;
    /* Eq. 54 */
    const double qx = ora_qfactor(c) * jx;
    const double qy = ora_qfactor(c) * jy;
    for (int i = 0; i < 8; ++i) {
        const double ciq = CX[i] * qx + CY[i] * qy;
        /* Eq. 15 */
        const double eeq = omega_w(i) * c->cv * T + 5.0 * a_w(i) * ciq / 3.0;
        /* Eq. 16 (dt = 1); zero when tau_R is infinite */
        const double S = isinf(c->tau_r) ? 0.0
                       : -(1.0 - 1.0 / (2.0 * tau)) * 5.0 * a_w(i) * ciq / (3.0 * c->tau_r);
        /* Eq. 13 */
        e_out[i] = e_in[i] + (eeq - e_in[i]) / tau + S;
    }
}

/* Initial state (n = 0): the equilibrium of Eq. 15 for the given temperature
 * and heat flux.  The heat flux enters through sum_i c_i e_i = q / qfactor so
 * that Eq. 54 read back at n = 0 returns the given q.  Isothermal wall nodes
 * hold the wall equilibrium of Eq. 55 from the start.  T, qx, qy: ny*nx row
 * major; qx/qy may be NULL (zero flux). */
void ora_init(const ora_case* c, const double* T, const double* qx, const double* qy, double* e)
{
    const double qf = ora_qfactor(c);
    for (int y = 0; y < c->ny; ++y)
        for (int x = 0; x < c->nx; ++x) {
            size_t n = (size_t)y * c->nx + x;
            double jx = qx ? qx[n] / qf : 0.0, jy = qy ? qy[n] / qf : 0.0;
            for (int i = 0; i < 8; ++i)
                e[IDX(c, i, x, y)] = omega_w(i) * c->cv * T[n]
                                   + 5.0 * a_w(i) * (CX[i] * jx + CY[i] * jy) / 3.0;
        }
    /* Eq. 55 on isothermal wall nodes (y walls first: x walls own corners) */
    for (int w = 3; w >= 0; --w) {
        if (kind_of(c, w) != ORA_ISOTHERMAL) continue;
        const int n = w < 2 ? c->ny : c->nx;
        for (int k = 0; k < n; ++k) {
            const int x = w < 2 ? (w == 0 ? 0 : c->nx - 1) : k;
            const int y = w < 2 ? k : (w == 2 ? 0 : c->ny - 1);
            for (int i = 0; i < 8; ++i) e[IDX(c, i, x, y)] = omega_w(i) * c->cv * c->t_wall[w];
        }
    }
}

/* Diffuse reflection (Eq. 58) at one wall node: the populations leaving the
 * wall (c_i . n < 0) share the incident energy (c_i . n > 0) in proportion to
 * omega_i.  (nxo, nyo) is the outward unit normal. */
static void diffuse_node(const ora_case* c, double* e, int x, int y, int nxo, int nyo)
{
    double incident = 0.0, wsum = 0.0;
    for (int i = 0; i < 8; ++i) {
        int cn = CX[i] * nxo + CY[i] * nyo;
        if (cn > 0) incident += e[IDX(c, i, x, y)];
        if (cn < 0) wsum += omega_w(i);
    }
    for (int i = 0; i < 8; ++i)
        if (CX[i] * nxo + CY[i] * nyo < 0)
            e[IDX(c, i, x, y)] = omega_w(i) / wsum * incident;
}

/* Heat-flux boundary (Eq. 57) at one wall node: as Eq. 58, with the incident
 * sum raised by q_0 / c times (2 tau_r + 1) / (2 tau_r), so that Eq. 56 holds
 * for the populations after the treatment (c = 1; the factor is 1 when tau_r
 * is infinite). */
static void heatflux_node(const ora_case* c, double* e, int x, int y, int nxo, int nyo, double q0)
{
    double incident = 0.0, wsum = 0.0;
    for (int i = 0; i < 8; ++i) {
        int cn = CX[i] * nxo + CY[i] * nyo;
        if (cn > 0) incident += e[IDX(c, i, x, y)];
        if (cn < 0) wsum += omega_w(i);
    }
    const double inv_factor = isinf(c->tau_r) ? 1.0 : (2.0 * c->tau_r + 1.0) / (2.0 * c->tau_r);
    const double total = incident + q0 * inv_factor;
    for (int i = 0; i < 8; ++i)
        if (CX[i] * nxo + CY[i] * nyo < 0)
            e[IDX(c, i, x, y)] = omega_w(i) / wsum * total;
}

/* Boundary treatment of wall w after advection, by its kind: Eq. 55, 57 or 58. */
static void treat_wall(const ora_case* c, double* e, int w)
{
    const int kind = kind_of(c, w);
    const int n = w < 2 ? c->ny : c->nx;
    const int nxo = w == 0 ? -1 : (w == 1 ? 1 : 0), nyo = w == 2 ? -1 : (w == 3 ? 1 : 0);
    for (int k = 0; k < n; ++k) {
        const int x = w < 2 ? (w == 0 ? 0 : c->nx - 1) : k;
        const int y = w < 2 ? k : (w == 2 ? 0 : c->ny - 1);
        if (kind == ORA_ISOTHERMAL)
            for (int i = 0; i < 8; ++i) e[IDX(c, i, x, y)] = omega_w(i) * c->cv * c->t_wall[w];
        else if (kind == ORA_DIFFUSE)
            diffuse_node(c, e, x, y, nxo, nyo);
        else if (kind == ORA_HEATFLUX)
            heatflux_node(c, e, x, y, nxo, nyo, c->q_wall[w]);
    }
}

/* Advance n steps.  e: state at the start of a step (in/out), work: scratch
 * of the same size (8*ny*nx doubles). */
void ora_run(const ora_case* c, double* e, double* work, long nsteps)
{
    const int nx = c->nx, ny = c->ny;
    const int px = (c->bc_x == ORA_PERIODIC || c->bc_x == ORA_GRADIENT);
    const int py = (c->bc_y == ORA_PERIODIC);
    /* seam jump of Eqs. 59-60: T_h - T_c over one period of nx nodes */
    const double dT_seam = c->grad_x * (double)nx;
    for (long s = 0; s < nsteps; ++s) {
        /* relaxation, node by node (Eqs. 13, 15, 16, 53, 54) */
#pragma omp parallel for schedule(static)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                double in[8], out[8];
                for (int i = 0; i < 8; ++i) in[i] = e[IDX(c, i, x, y)];
                ora_collide_node(c, in, out);
                for (int i = 0; i < 8; ++i) work[IDX(c, i, x, y)] = out[i];
            }
        /* advection: e_i(x + c_i, t + 1) = e*_i(x, t) (Eq. 13 left-hand side),
         * written as a gather from x - c_i.  Sources outside a walled axis are
         * left for the boundary treatment. */
#pragma omp parallel for schedule(static)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x)
                for (int i = 0; i < 8; ++i) {
                    int sx = x - CX[i], sy = y - CY[i];
                    int outside = 0;
                    double jump = 0.0;
                    if (sx < 0 || sx >= nx) {
                        if (!px) outside = 1;
                        else {
                            /* Eq. 59: +x movers entering at x=0 from the right end carry
                             * omega_i C_V (T_h - T_c); Eq. 60: -x movers entering at
                             * x = nx-1 from the left end carry omega_i C_V (T_c - T_h). */
                            if (c->bc_x == ORA_GRADIENT)
                                jump = (sx < 0 ? 1.0 : -1.0) * omega_w(i) * c->cv * dT_seam;
                            sx = (sx + nx) % nx;
                        }
                    }
                    if (sy < 0 || sy >= ny) {
                        if (!py) outside = 1;
                        else sy = (sy + ny) % ny;
                    }
                    /* unknown population: give it a defined value; the boundary
                     * treatment below overwrites every one of these */
                    e[IDX(c, i, x, y)] = outside ? 0.0 : work[IDX(c, i, sx, sy)] + jump;
                }
        /* boundary treatment after advection (Sec. 2.5); the y walls first,
         * so that (isothermal) x walls own the corner nodes */
        if (!py) {
            treat_wall(c, e, 2);
            treat_wall(c, e, 3);
        }
        if (!px) {
            treat_wall(c, e, 0);
            treat_wall(c, e, 1);
        }
    }
}

/* Macroscopic fields of a state (Eqs. 53-54): T, q_x, q_y, each ny*nx. */
void ora_moments(const ora_case* c, const double* e, double* T, double* qx, double* qy)
{
    const double qf = ora_qfactor(c);
#pragma omp parallel for schedule(static)
    for (int y = 0; y < c->ny; ++y)
        for (int x = 0; x < c->nx; ++x) {
            double s = 0.0, jx = 0.0, jy = 0.0;
            for (int i = 0; i < 8; ++i) {
                double v = e[IDX(c, i, x, y)];
                s += v;
                jx += CX[i] * v;
                jy += CY[i] * v;
            }
            size_t n = (size_t)y * c->nx + x;
            T[n] = s / c->cv;
            qx[n] = qf * jx;
            qy[n] = qf * jy;
        }
}

/* Deviation totals of a state in FP64: sum of (e - C_V T_ref), sum q_x, sum q_y. */
void ora_totals(const ora_case* c, const double* e, double out[3])
{
    const double qf = ora_qfactor(c);
    double se = 0.0, sx = 0.0, sy = 0.0;
    for (int y = 0; y < c->ny; ++y)
        for (int x = 0; x < c->nx; ++x) {
            double s = 0.0, jx = 0.0, jy = 0.0;
            for (int i = 0; i < 8; ++i) {
                double v = e[IDX(c, i, x, y)];
                s += v;
                jx += CX[i] * v;
                jy += CY[i] * v;
            }
            se += s - c->cv * ora_tref(c, x);
            sx += qf * jx;
            sy += qf * jy;
        }
    out[0] = se;
    out[1] = sx;
    out[2] = sy;
}

int ora_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void ora_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
