"""Pins of the oracle's boundary treatments against the paper's closed forms.

Each test runs the FP64 C stepper on one of the paper's validation settings
(or a workload of this project) and compares it with an analytic result of
Sec. 3 or with an exact consequence of the scheme.  Tolerances are set from
the observed agreement with margin, and each one says which discretisation
effect it allows for.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import closed_forms as cf, ref


@pytest.fixture(autouse=True, scope="module")
def _threads():
    ref.set_threads(min(8, max(1, ref.max_threads())))


# ---------------------------------------------------------------- isothermal walls

def test_walls_profile_after_5000_steps():
    """128 x 64, isothermal walls at T0 +/- 0.5, periodic y, tau_N = 0.6,
    tau_R = 0.8, uniform T0 start: after 5000 steps the profile is the linear
    Fourier profile to within 1e-2 (only the n = 2 mode of the separation of
    variables solution remains, damped to 4e-3), closer still to that
    transient series, and exactly uniform in y."""
    case = W.wall_case()
    o = ref.Oracle(case)
    o.run(case.steps)
    T, qx, qy = o.moments()
    d = case.nx - 1
    X = np.arange(case.nx) / d
    theta = (T[0] - case.t_wall[1]) / (case.t_wall[0] - case.t_wall[1])
    assert np.abs(T - T[0]).max() == 0.0
    assert np.abs(qy).max() < 1e-15
    assert np.abs(theta - (1 - X)).max() < 1e-2
    series = cf.fourier_1d_theta(X, case.steps, d, cf.diffusivity(case.tau_r), 0.5)
    assert np.abs(theta - series).max() < 5e-3


def test_walls_steady_state_eq70_eq71():
    """Steady cross-plane conduction between isothermal walls matches the
    temperature-jump solution Eq. 70 in the interior and the flux Eq. 71
    within 2% (Kn_R = 8e-3, where the paper reports good agreement)."""
    case = W.wall_case(ny=4)
    o = ref.Oracle(case)
    o.run(60000)
    T, qx, _ = o.moments()
    d = case.nx - 1
    X = np.arange(case.nx) / d
    kn_r = cf.knudsen(case.tau_r, d)
    theta = (T[0] - case.t_wall[1]) / (case.t_wall[0] - case.t_wall[1])
    assert np.abs(theta[1:-1] - cf.cross_plane_theta_eq70(X[1:-1], kn_r)).max() < 6e-3
    Q = qx[0, 1:-1].mean() / (cf.VG * (case.t_wall[0] - case.t_wall[1]))
    assert Q == pytest.approx(cf.cross_plane_q_eq71(kn_r), rel=0.02)
    # steady flux is uniform across the film (energy balance Eq. 6)
    assert np.ptp(qx[0, 1:-1]) < 1e-6 * abs(qx[0, 1:-1].mean())


def test_isothermal_wall_nodes_hold_equilibrium():
    """Eq. 55: wall nodes carry omega_i C_V T_s at every step."""
    case = W.wall_case(nx=16, ny=4, steps=7)
    o = ref.Oracle(case, W.random_field(16, 4, 0.1, 1.0, 5))
    o.run(7)
    om = np.array([2 / 9] * 4 + [1 / 36] * 4)
    pops = o.populations()
    assert np.allclose(pops[:, :, 0], (om * case.t_wall[0])[:, None], atol=1e-15)
    assert np.allclose(pops[:, :, -1], (om * case.t_wall[1])[:, None], atol=1e-15)


@pytest.mark.parametrize("nodes", [201, 101, 51, 21])
def test_diffusive_transient_eq61_eq62(nodes):
    """Sec. 3.1.1: film at T_c = 299 K, left wall raised to T_h = 301 K,
    Kn_R = 1.29e-3, Kn_N = 1.29e3, grid nodes x 3.  At t* = 1e6 the error norms
    of Eqs. 63-64 against Eqs. 61-62 are small and shrink with the grid."""
    kn_r, kn_n = 1.29e-3, 1.29e3
    N = nodes - 1
    tn, tr = cf.lattice_relaxation_times(N, kn_n, kn_r)
    case = W.Case("d1", nodes, 3, tn, tr, bc_x="isothermal", bc_y="periodic", t0=299.0,
                  t_wall=(301.0, 299.0, 0.0, 0.0))
    o = ref.Oracle(case)
    o.run(int(round(1e6 * tr)))
    T, qx, _ = o.moments()
    X = np.arange(nodes) / N
    ts = o.steps / tr
    theta = (T[0] - 299.0) / 2.0
    Q = qx[0] * N / (cf.VG ** 2 * tr / 3.0 * 2.0)
    tha = cf.fourier_1d_theta_eq61(X, ts, kn_r)
    Qa = cf.fourier_1d_q_eq62(X, ts, kn_r)
    e1_t = np.abs(theta - tha).sum() / np.abs(tha).sum()
    e1_q = np.abs(Q - Qa).sum() / np.abs(Qa).sum()
    # observed: E1(Theta) = 1.5e-3, 3.9e-3, 8.7e-3, 2.2e-2 and E1(Q) = 0.013,
    # 0.028, 0.057, 0.14 for 201 ... 21 nodes (first order, Fig. 4)
    bound_t = {201: 3e-3, 101: 8e-3, 51: 1.7e-2, 21: 4.5e-2}[nodes]
    bound_q = {201: 2.6e-2, 101: 5.5e-2, 51: 0.11, 21: 0.28}[nodes]
    assert e1_t < bound_t
    assert e1_q < bound_q


def test_diffusive_transient_first_order():
    """Error norms of Eqs. 63-64 fall about linearly with the grid spacing
    (Sec. 3.1.1, Fig. 4: approximately first order).  Coarse grids only."""
    kn_r, kn_n = 1.29e-3, 1.29e3
    errs = []
    for nodes in (101, 51, 21):
        N = nodes - 1
        tn, tr = cf.lattice_relaxation_times(N, kn_n, kn_r)
        case = W.Case("d1", nodes, 3, tn, tr, bc_x="isothermal", bc_y="periodic", t0=299.0,
                      t_wall=(301.0, 299.0, 0.0, 0.0))
        o = ref.Oracle(case)
        o.run(int(round(1e6 * tr)))
        T, _, _ = o.moments()
        X = np.arange(nodes) / N
        tha = cf.fourier_1d_theta_eq61(X, o.steps / tr, kn_r)
        errs.append((N, np.abs((T[0] - 299.0) / 2.0 - tha).sum() / np.abs(tha).sum()))
    errs = np.array(errs)
    order = np.polyfit(np.log(1.0 / errs[:, 0]), np.log(errs[:, 1]), 1)[0]
    assert 0.8 < order < 1.5


# ---------------------------------------------------------------- gradient seam

@pytest.mark.parametrize("tau_n,tau_r", [(0.7, 3.0), (0.55, 50.0), (2.0, 0.3)])
def test_gradient_seam_exact_flux(tau_n, tau_r):
    """Eqs. 59-60 with period nx and jump grad * nx, periodic in y, starting
    from the ramp: the deviation stays uniform and the heat flux at step n is
    exactly (5/9) C_V G tau_r (1 - rho^n), which tends to Fourier's law
    q = lambda G with lambda = C_V v_g^2 tau_R / 3."""
    G = 1e-3
    case = W.Case("g", 16, 6, tau_n, tau_r, bc_x="gradient", bc_y="periodic", grad_x=G, t0=1.0,
                  cv=1.3)
    o = ref.Oracle(case)
    rho = cf.scheme_constants(tau_n, tau_r)["rho"]
    ramp = np.tile(case.t_ref(), (case.ny, 1))
    for n in (1, 2, 5, 40, 200):
        o.run(n - o.steps)
        T, qx, qy = o.moments()
        want = 5.0 / 9.0 * 1.3 * G * tau_r * (1 - rho ** n)
        assert np.abs(qx - want).max() < 1e-14
        assert np.abs(qy).max() < 1e-15
        assert np.abs(T - ramp).max() < 1e-13
    assert want == pytest.approx(1.3 * cf.VG ** 2 * tau_r / 3.0 * G, rel=1e-6 if abs(rho) < 0.95 else 1)


# ---------------------------------------------------------------- diffuse walls

def test_diffuse_walls_zero_normal_flux_and_fixed_point():
    """Eq. 58 is Eq. 57 with q_0 = 0: after the boundary treatment the normal
    heat flux of Eq. 56 vanishes at every wall node, at every step, for any
    field; a uniform equilibrium is a fixed point."""
    for bc_x, bc_y, nx, ny in (("periodic", "diffuse", 24, 17), ("diffuse", "periodic", 17, 24)):
        case = W.Case("c", nx, ny, 0.6, 7.0, bc_x=bc_x, bc_y=bc_y, t0=1.0)
        o = ref.Oracle(case, W.random_field(nx, ny, 0.05, 1.0, 21), *W.random_flux(nx, ny, 0.01, 22))
        for _ in range(5):
            o.run(7)
            _, qx, qy = o.moments()
            if bc_y == "diffuse":
                assert np.abs(qy[[0, -1], :]).max() < 1e-15
            else:
                assert np.abs(qx[:, [0, -1]]).max() < 1e-15
        u = ref.Oracle(case)
        e0 = u.populations().copy()
        u.run(50)
        assert np.abs(u.populations() - e0).max() < 1e-15


def test_diffuse_walls_energy():
    """Energy through the wet-node wall: the wall row loses its own outgoing
    populations and regains what arrives from the first interior row, so the
    total is exact when the deviation is odd about the mid-plane (the two walls'
    defects cancel) and otherwise off by a
    first-order discretisation defect that halves with each grid doubling."""
    ny = 33
    y = np.arange(ny) / (ny - 1)
    odd = 1 + 0.01 * np.cos(np.pi * y) + 0.003 * np.cos(3 * np.pi * y) + 0.002 * (y - 0.5)
    case = W.Case("c", 4, ny, 0.6, 7.0, bc_x="periodic", bc_y="diffuse", t0=1.0)
    o = ref.Oracle(case, np.tile(odd[:, None], (1, 4)))
    a = o.totals()[0]
    o.run(2000)
    # rounding drift only: total energy is ~132 in absolute terms
    assert o.totals()[0] == pytest.approx(a, abs=1e-10)
    defects = []
    for ny in (17, 33, 65):
        y = np.arange(ny) / (ny - 1)
        prof = 1 + 0.01 * np.sin(np.pi * y / 2)
        case = W.Case("c", 4, ny, 0.6, 7.0, bc_x="periodic", bc_y="diffuse", t0=1.0)
        o = ref.Oracle(case, np.tile(prof[:, None], (1, 4)))
        a = o.totals()[0]
        worst = 0.0
        for _ in range(20):
            o.run(int(0.05 * (ny - 1) ** 2))
            worst = max(worst, abs(o.totals()[0] - a))
        defects.append(worst / (0.01 * 4 * ny))
    # observed 9.6e-3, 4.1e-3, 2.1e-3
    assert defects[0] < 1.2e-2
    assert defects[1] / defects[0] < 0.6 and defects[2] / defects[1] < 0.6


@pytest.mark.parametrize("kn_r", [1.0, 10.0])
def test_poiseuille_eq68_eq69(kn_r):
    """Sec. 3.2 on its own grid (3 x 301, Kn_N = 0.01): the steady heat-flux
    profile follows Eq. 68 (centre within 0.5%, relative L2 within 5%; the
    gap sits in the first nodes off each wall) and the conductivity Eq. 69
    within 2%.  The profile is exactly uniform along x."""
    G = 1e-4
    tn, tr = cf.lattice_relaxation_times(300, 0.01, kn_r)
    case = W.Case("p", 3, 301, tn, tr, bc_x="gradient", bc_y="diffuse", grad_x=G, t0=1.0)
    o = ref.Oracle(case)
    prev = None
    for _ in range(400):
        o.run(500)
        _, qx, _ = o.moments()
        if prev is not None and np.abs(qx - prev).max() < 1e-13 * np.abs(qx).max():
            break
        prev = qx.copy()
    assert np.abs(qx - qx[:, :1]).max() < 1e-15
    Q = qx[:, 1] / cf.poiseuille_q_scale(tr, G)
    Y = np.arange(301) / 300.0
    kn_c = cf.overall_knudsen(0.01, kn_r)
    Qa = cf.poiseuille_q_eq68(Y, kn_c, kn_r)
    assert Q[150] == pytest.approx(Qa[150], rel=5e-3)
    assert np.linalg.norm(Q - Qa) / np.linalg.norm(Qa) < 0.05
    assert Q.mean() == pytest.approx(cf.poiseuille_conductivity_eq69(kn_c, kn_r), rel=0.02)


# ---------------------------------------------------------------- closed forms themselves

def test_closed_forms_self_consistent():
    """The transcribed formulas agree with the statements around them: Eq. 69
    integrates Eq. 68; Eq. 68 solves the steady Eq. 7 across the film
    (Q = 1 + Kn_eff^2 Q'') with the slip condition Eq. 11; Eq. 70 is
    antisymmetric with the Eq. 71 flux by Fourier's law; Eq. 62 is -dEq.61/dX."""
    kn_c, kn_r = 4e-3, 4.0
    k = math.sqrt(kn_c * kn_r / 5)
    Y = np.linspace(0, 1, 200001)
    Q = cf.poiseuille_q_eq68(Y, kn_c, kn_r)
    assert np.trapezoid(Q, Y) == pytest.approx(cf.poiseuille_conductivity_eq69(kn_c, kn_r), rel=1e-9)
    h = Y[1] - Y[0]
    Qpp = (Q[2:] - 2 * Q[1:-1] + Q[:-2]) / h ** 2
    assert np.abs(1 + k * k * Qpp - Q[1:-1]).max() < 1e-5
    Qp0 = (Q[1] - Q[0]) / h
    assert Q[0] == pytest.approx(8 / 15 * kn_c * Qp0, rel=1e-3)
    th = cf.cross_plane_theta_eq70(np.array([0.0, 1.0]), 0.3)
    assert th[0] + th[1] == pytest.approx(1.0, abs=1e-15)
    slope = th[1] - th[0]
    assert -slope * 0.3 / 3.0 == pytest.approx(cf.cross_plane_q_eq71(0.3), rel=1e-12)
    X = np.linspace(0.05, 0.95, 19)
    dX = 1e-6
    dth = (cf.fourier_1d_theta_eq61(X + dX, 2e5, 1.29e-3) - cf.fourier_1d_theta_eq61(X - dX, 2e5, 1.29e-3)) / (2 * dX)
    assert np.allclose(-dth, cf.fourier_1d_q_eq62(X, 2e5, 1.29e-3), atol=1e-6)
    # uniform-start series reduces to Eq. 61 at theta0 = 0
    alpha_t = 1.29e-3 ** 2 * 2e5 / 3.0
    assert np.allclose(cf.fourier_1d_theta(X, alpha_t, 1.0, 1.0, 0.0), cf.fourier_1d_theta_eq61(X, 2e5, 1.29e-3),
                       atol=1e-12)


# ---------------------------------------------------------------- Sec. 3.1.2 square

def test_square_closed_forms_eq65_67():
    """Eqs. 65-67 as transcribed: Theta harmonic, Q = -grad Theta, Theta = 0 on
    the three isothermal sides, Q_y = -1 (heat flux Q0 into the square) on the
    top side."""
    X = np.linspace(0.05, 0.95, 19)
    XX, YY = np.meshgrid(X, X)
    h = 1e-4
    th, qx, qy = cf.square_eq65_67(XX, YY)
    f = lambda dx, dy: cf.square_eq65_67(XX + dx, YY + dy)[0]
    lap = (f(h, 0) + f(-h, 0) + f(0, h) + f(0, -h) - 4.0 * th) / h ** 2
    assert np.abs(lap).max() < 1e-4
    assert np.abs(qx + (f(h, 0) - f(-h, 0)) / (2 * h)).max() < 1e-6
    assert np.abs(qy + (f(0, h) - f(0, -h)) / (2 * h)).max() < 1e-6
    e = np.linspace(0.0, 1.0, 7)
    assert np.abs(cf.square_eq65_67(np.zeros(7), e)[0]).max() < 1e-15
    assert np.abs(cf.square_eq65_67(np.ones(7), e)[0]).max() < 1e-12
    assert np.abs(cf.square_eq65_67(e, np.zeros(7))[0]).max() < 1e-15
    xt = np.linspace(0.1, 0.9, 9)
    assert np.allclose(cf.square_eq65_67(xt, np.ones(9), n_terms=20000)[2], -1.0, atol=2e-4)


def test_square_heatflux_top_eq65():
    """Sec. 3.1.2 (Kn_R = 2e-3, Kn_N = 2e3; heat flux on the top side, the other
    three sides isothermal, corners owned by the isothermal x walls), run to
    steady state (14 time constants of the slowest mode) on 21 and 41 nodes
    per side: the temperature approaches Eq. 65 (relative L2 0.19 -> 0.077,
    more than halving per grid doubling; the wall temperature jump and the
    corner singularities where the flux meets the cold sides are grid-scale
    effects), and the top wall carries exactly q0 (Eq. 56)."""
    q0 = 1e-3
    errs = []
    for nodes in (21, 41):
        d = nodes - 1
        tn, tr = cf.lattice_relaxation_times(d, 2e3, 2e-3)
        case = W.square_case(nodes, tn, tr, q0=q0)
        o = ref.Oracle(case)
        lam = cf.diffusivity(tr)                  # conductivity with C_V = 1
        o.run(int(14 * d * d / (1.25 * math.pi ** 2 * lam)))
        T, _, qy = o.moments()
        assert np.allclose(qy[-1, 1:-1], -q0, rtol=1e-12)
        X = np.arange(nodes) / d
        XX, YY = np.meshgrid(X, X)
        th = cf.square_eq65_67(XX, YY)[0]
        got = (T - case.t0) / (q0 * d / lam)      # Theta / Q0 = (T - T_c) lambda / (q0 L)
        errs.append(float(np.linalg.norm(got - th) / np.linalg.norm(th)))
    assert errs[1] < 0.08 and errs[1] < 0.5 * errs[0], errs
