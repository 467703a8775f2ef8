"""Pins of the oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each checks a consequence of
the scheme that a plausible mistake (wrong weight, sign, index, transposed
velocity, missing source factor, wrong seam) would break.
"""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import bloch, closed_forms as cf, ref
from measure import front_radius

CX = np.array([1, 0, -1, 0, 1, -1, -1, 1])
CY = np.array([0, 1, 0, -1, 1, 1, -1, -1])

REGIMES = [(0.6, 0.8), (0.55, 50.0), (0.7, 3.0), (2.3, 0.2), (0.51, math.inf), (1.0, 1000.0)]


def _case(nx, ny, tau_n, tau_r, **kw):
    return W.Case("t", nx, ny, tau_n, tau_r, **kw)


def _collision_matrix_from_oracle(tau_n, tau_r):
    case = _case(4, 4, tau_n, tau_r)
    return np.stack([ref.collide_node(case, np.eye(8)[j]) for j in range(8)], axis=1)


# ---------------------------------------------------------------- single node

@pytest.mark.parametrize("tau_n,tau_r", REGIMES)
def test_collision_moments(tau_n, tau_r):
    """Moments of one relaxation step follow from Eqs. 22-28 and Eq. 54:
    energy kept (Eqs. 22, 26); first moment scaled by rho (Eqs. 23, 27, 54);
    second moment relaxed toward (5/9) C_V T delta at rate 1/tau (Eqs. 24, 28);
    third moment c_x c_y^2 relaxed toward q_x / 3 at rate 1/tau plus the
    source's share (Eqs. 25, 16)."""
    p = cf.scheme_constants(tau_n, tau_r)
    tau, rho, beta = p["tau"], p["rho"], p["beta"]
    kappa = 1.0 / tau - (0.0 if math.isinf(tau_r) else (1.0 - 0.5 / tau) / tau_r)
    rng = np.random.default_rng(7)
    case = _case(4, 4, tau_n, tau_r, cv=1.7)
    for _ in range(20):
        e = rng.uniform(-1, 1, 8) + 0.3
        s = ref.collide_node(case, e)
        E = e.sum()
        jx, jy = CX @ e, CY @ e
        assert s.sum() == pytest.approx(E, abs=1e-14)
        assert CX @ s == pytest.approx(rho * jx, abs=1e-14)
        assert CY @ s == pytest.approx(rho * jy, abs=1e-14)
        for ca, cb in ((CX, CX), (CY, CY)):
            m2, m2s = (ca * cb) @ e, (ca * cb) @ s
            assert m2s == pytest.approx((1 - 1 / tau) * m2 + (5.0 / 9.0) * E / tau, abs=1e-14)
        assert (CX * CY) @ s == pytest.approx((1 - 1 / tau) * ((CX * CY) @ e), abs=1e-14)
        m3, m3s = (CX * CY * CY) @ e, (CX * CY * CY) @ s
        assert m3s == pytest.approx((1 - 1 / tau) * m3 + kappa * beta * jx / 3.0, abs=1e-14)


@pytest.mark.parametrize("tau_n,tau_r", REGIMES)
def test_collision_eigenvalues(tau_n, tau_r):
    """The relaxation matrix has eigenvalues 1 (energy), rho twice (heat flux)
    and 1 - 1/tau five times (non-conserved moments)."""
    p = cf.scheme_constants(tau_n, tau_r)
    M = _collision_matrix_from_oracle(tau_n, tau_r)
    lam = np.sort_complex(np.linalg.eigvals(M))
    want = np.sort_complex(np.array([1.0, p["rho"], p["rho"]] + [1 - 1 / p["tau"]] * 5,
                                    dtype=complex))
    assert np.allclose(lam, want, atol=1e-10)


def test_weights_from_equilibrium_fixed_point():
    """A uniform equilibrium with zero flux is a fixed point: with Eq. 17's
    weights summing to 1 over eight directions, e_i = omega_i C_V T relaxes to
    itself, and its second moment is (5/9) C_V T (Eq. 24)."""
    golden = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
    case = _case(4, 4, 0.6, 0.8, cv=2.0)
    # isolate omega_i from the fixed point: relax a state that carries energy only
    # in direction i and read the energy handed to every direction
    M = _collision_matrix_from_oracle(0.6, 0.8)
    tau = cf.scheme_constants(0.6, 0.8)["tau"]
    # column j of (M - (1-1/tau) I) * tau, minus the flux part, gives omega
    om = np.array([(M[i, 0] + M[i, 2]) / 2.0 * tau for i in range(8)])
    om[0] -= (1 - 1 / tau) * tau / 2.0
    om[2] -= (1 - 1 / tau) * tau / 2.0
    assert np.allclose(om[:4], 2.0 / 9.0, atol=1e-13)
    assert np.allclose(om[4:], 1.0 / 36.0, atol=1e-13)
    assert om.sum() == pytest.approx(golden["weights_sum"]["value"], abs=1e-13)
    e = np.array([2 / 9] * 4 + [1 / 36] * 4) * 2.0 * 1.3
    assert np.allclose(ref.collide_node(case, e), e, atol=1e-15)


# ---------------------------------------------------------------- advection

def test_advection_direction_and_numbering():
    """With tau_N = tau_R huge the relaxation is the identity to 1e-12, so one
    step moves a lone population e_i by c_i (Eq. 13 left-hand side with
    Eq. 14's velocities in the paper's numbering)."""
    nx, ny = 9, 7
    case = _case(nx, ny, 1e12, 1e12, t0=0.0)
    for i in range(8):
        o = ref.Oracle(case, np.zeros((ny, nx)))
        pops = o.populations()
        pops[...] = 0.0
        pops[i, 3, 4] = 1.0
        o.run(1)
        pops = o.populations()
        y1, x1 = 3 + CY[i], 4 + CX[i]
        assert pops[i, y1, x1] == pytest.approx(1.0, abs=1e-11)
        pops[i, y1, x1] = 0.0
        assert np.abs(pops).max() < 1e-11


# ---------------------------------------------------------------- periodic

@pytest.mark.parametrize("tau_n,tau_r", REGIMES)
def test_stepper_matches_bloch(tau_n, tau_r):
    """The C stepper equals the Fourier-mode matrix power (an independent route:
    no stepping, no indexing) on a non-square periodic grid from a random
    non-equilibrium state."""
    nx, ny, n = 24, 16, 57
    case = _case(nx, ny, tau_n, tau_r)
    T0 = W.random_field(nx, ny, 0.01, 1.0, 1)
    qx, qy = W.random_flux(nx, ny, 1e-3, 2)
    o = ref.Oracle(case, T0, qx, qy)
    rng = np.random.default_rng(3)
    o.populations()[...] += 1e-3 * rng.standard_normal((8, ny, nx))
    e0 = o.populations().copy()
    o.run(n)
    eb = bloch.evolve_populations(e0, n, tau_n, tau_r)
    assert np.abs(o.populations() - eb).max() < 1e-13


@pytest.mark.parametrize("tau_n,tau_r", REGIMES)
def test_periodic_invariants(tau_n, tau_r):
    """Total energy is constant and the total heat flux is multiplied by
    rho = (2 tau_r - 1)/(2 tau_r + 1) per step, for any tau_N; with tau_R
    infinite it is constant (normal scattering conserves quasi-momentum)."""
    nx, ny, n = 20, 12, 40
    case = _case(nx, ny, tau_n, tau_r)
    T0 = W.random_field(nx, ny, 0.05, 1.0, 11)
    qx, qy = W.random_flux(nx, ny, 0.01, 12)
    o = ref.Oracle(case, T0, qx, qy)
    a = o.totals()
    o.run(n)
    b = o.totals()
    rho = cf.scheme_constants(tau_n, tau_r)["rho"]
    assert b[0] == pytest.approx(a[0], abs=1e-12)
    assert b[1] == pytest.approx(a[1] * rho ** n, abs=1e-12)
    assert b[2] == pytest.approx(a[2] * rho ** n, abs=1e-12)


@pytest.mark.parametrize("tau_n,tau_r", REGIMES)
def test_initial_flux_reads_back_through_eq54(tau_n, tau_r):
    """Initial state with a given heat flux (read as the Eq. 15 equilibrium
    with first moment q / beta, the paper being silent): Eq. 54 on the raw
    populations at n = 0 returns the given q and Eq. 53 the given T, node by
    node; the uniform part of the flux then decays by exactly rho per step
    from the *given* flux (the decay factor fixed by Eqs. 13, 15, 16, 54), so
    a state that stored q instead of q / beta (off by beta) or dropped the
    flux share fails.  The temperature is checked against its deviation."""
    nx, ny, n = 18, 11, 7
    p = cf.scheme_constants(tau_n, tau_r)
    beta, rho = p["beta"], p["rho"]
    cv = 1.3
    case = _case(nx, ny, tau_n, tau_r, cv=cv)
    T0 = W.random_field(nx, ny, 0.05, 1.0, 21)
    qx, qy = W.random_flux(nx, ny, 0.01, 22)
    qx = qx + 0.004                      # a uniform part, which no advection moves
    qy = qy - 0.003
    o = ref.Oracle(case, T0, qx, qy)
    e = o.populations()
    E = e.sum(axis=0)
    jx = np.tensordot(CX, e, axes=1)
    jy = np.tensordot(CY, e, axes=1)
    assert np.abs(E / cv - T0).max() <= 1e-13
    assert np.abs(beta * jx - qx).max() <= 1e-15
    assert np.abs(beta * jy - qy).max() <= 1e-15
    # the populations are the Eq. 15 equilibrium itself: its second moments
    # are (5/9) C_V T delta_ab (Eq. 24), the mixed one vanishes
    assert np.abs((CX * CX) @ e.reshape(8, -1) - 5.0 / 9.0 * E.ravel()).max() <= 1e-13
    assert np.abs((CX * CY) @ e.reshape(8, -1)).max() <= 1e-15
    o.run(n)
    tot = o.totals()
    assert tot[1] == pytest.approx(rho ** n * qx.sum(), rel=1e-12, abs=1e-14)
    assert tot[2] == pytest.approx(rho ** n * qy.sum(), rel=1e-12, abs=1e-14)
    # a uniform start stays uniform: every node's flux is rho^n times the given one
    u = ref.Oracle(case, np.full((ny, nx), 1.2), np.full((ny, nx), 0.004), np.full((ny, nx), -0.003))
    u.run(n)
    _, ux, uy = u.moments()
    assert np.abs(ux - rho ** n * 0.004).max() <= 1e-15
    assert np.abs(uy + rho ** n * 0.003).max() <= 1e-15


@pytest.mark.parametrize("tau_n,tau_r", [(0.55, 50.0), (0.6, 5.0), (0.8, 0.8), (0.51, 1000.0)])
def test_bloch_dispersion_is_eq52(tau_n, tau_r):
    """Slow Bloch eigenvalues reproduce the temperature equation Eq. 52 (the
    scheme's Chapman-Enskog limit) for long waves, in every direction.  Only
    hydrodynamic roots (|s| well below one per step) are the expansion's
    limit; a root near -1/tau_R with tau_R ~ 1 step is a kinetic mode."""
    tau_c = cf.scheme_constants(tau_n, tau_r)["tau_c"]
    for k in (0.01, 0.02, 0.04):
        want = [w for w in cf.telegraph_rates(k, tau_r, tau_c) if abs(w) < 0.1]
        assert want
        for theta in (0.0, 0.4, math.pi / 4):
            s = np.log(bloch.slow_eigenvalues(k, theta, tau_n, tau_r, count=3))
            for w in want:
                err = np.min(np.abs(s - w)) / abs(w)
                assert err < 5e-3, (k, theta, s, want)


def test_second_sound_phase_speed():
    """Long waves with dominant normal scattering travel at v_g / sqrt(3)
    (Sec. 3.4), i.e. sqrt(5)/3 nodes per step."""
    golden = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
    v = golden["second_sound_speed"]["value_over_vg"] * cf.VG
    assert v == pytest.approx(math.sqrt(5.0) / 3.0, rel=1e-12)
    s = np.log(bloch.slow_eigenvalues(0.005, 0.3, 0.5001, math.inf, count=3))
    speed = np.max(np.abs(s.imag)) / 0.005
    assert speed == pytest.approx(v, rel=1e-4)
    assert np.max(s.real) == pytest.approx(0.0, abs=1e-4)


def test_second_sound_front_speed_1d():
    """With normal scattering dominant (tau_R / tau_N ~ 2e5, as in the second
    sound case of Sec. 3.4) a plane heat pulse travels at v_g / sqrt(3):
    measured on the exact periodic solution, within 0.5%."""
    nx, ny = 2048, 4
    T0 = np.tile(W.gaussian_field(nx, 1, nx // 2, 0, 0.01, 20.0, 1.0), (ny, 1))
    ts = np.arange(150, 1001, 85)
    radii = []
    for t in ts:
        T, _, _ = bloch.evolve_temperature_field(T0, int(t), 0.55, 1e5)
        radii.append(front_radius(T[0, nx // 2:] - 1.0))
    slope = np.polyfit(ts, radii, 1)[0]
    assert slope == pytest.approx(cf.second_sound_speed(), rel=5e-3)


def test_second_sound_front_speed_2d():
    """The ring front of a 2D Gaussian pulse (sigma = 20) moves at v_g / sqrt(3)
    within 3% when resistive scattering is weak (tau_R = 1e5)."""
    n = 1024
    T0 = W.gaussian_field(n, n, n // 2, n // 2, 0.01, 20.0, 1.0)
    ts = np.arange(150, 391, 40)
    radii = []
    for t in ts:
        T, _, _ = bloch.evolve_temperature_field(T0, int(t), 0.55, 1e5)
        radii.append(front_radius(T[n // 2, n // 2:] - 1.0))
    slope = np.polyfit(ts, radii, 1)[0]
    assert slope == pytest.approx(cf.second_sound_speed(), rel=0.03)


# ---------------------------------------------------------------- mapping

def test_tau_max_values(golden_dir):
    """tau = 0.5 + sqrt(3/5) N Kn_C reproduces the four maxima printed in
    Sec. 3.4 only when N counts lattice spacings (nodes - 1)."""
    g = json.load(open(os.path.join(golden_dir, "tau_max.json")))
    for c in g["cases"]:
        kn_c = cf.overall_knudsen(c["kn_n"], c["kn_r"])
        tau = cf.tau_from_knudsen(c["nodes"] - 1, kn_c)
        assert round(tau, 4) == pytest.approx(c["tau_max"], abs=1e-12), c["name"]
        tn, tr = cf.lattice_relaxation_times(c["nodes"] - 1, c["kn_n"], c["kn_r"])
        assert cf.scheme_constants(tn, tr)["tau"] == pytest.approx(tau, rel=1e-12)
        # counting nodes instead of spacings misses at least one printed value
    miss = [abs(round(cf.tau_from_knudsen(c["nodes"], cf.overall_knudsen(c["kn_n"], c["kn_r"])), 4)
                - c["tau_max"]) > 1e-9 for c in g["cases"]]
    assert any(miss)


def test_separable_route_equals_full_fft_and_stepper():
    """The separable spectral route (used at 8192^2) gives the same rows as the
    full 2D FFT route and as the C stepper on a small lattice."""
    nx, ny, n = 96, 80, 150
    fx = np.exp(-(np.arange(nx) - 40) ** 2 / (2 * 6.0 ** 2))
    fy = np.exp(-(np.arange(ny) - 47) ** 2 / (2 * 5.0 ** 2))
    T0 = 1.0 + 0.01 * np.outer(fy, fx)
    S = bloch.SeparableSolution(fx, fy, 0.01, n, 0.55, 50.0)
    rows = [0, 13, 47, 79]
    Ts, qxs, qys = S.rows(rows)
    Tf, qxf, qyf = bloch.evolve_temperature_field(T0, n, 0.55, 50.0)
    assert np.abs(Ts - Tf[rows]).max() < 1e-15
    assert np.abs(qxs - qxf[rows]).max() < 1e-15 and np.abs(qys - qyf[rows]).max() < 1e-15
    o = ref.Oracle(W.Case("s", nx, ny, 0.55, 50.0), T0)
    o.run(n)
    To, qxo, qyo = o.moments()
    assert np.abs(Ts - To[rows]).max() < 1e-14
    assert np.abs(qxs - qxo[rows]).max() < 1e-14


def test_mode_solution_equals_stepper():
    """The few-mode exact solution (used at 16384^2) equals the C stepper on a
    small lattice with the same kind of seeded modes."""
    nx, ny, n = 64, 48, 90
    modes = W.draw_modes(n_modes=5, kmax=3, amp_total=1e-3, seed=3)
    T0 = W.modes_field(modes, nx, ny, 1.0)
    sol = bloch.ModeSolution(modes, nx, ny, n, 0.6, 5.0)
    o = ref.Oracle(W.Case("m", nx, ny, 0.6, 5.0), T0)
    o.run(n)
    To, qxo, qyo = o.moments()
    Tm, qxm, qym = sol.rows(range(ny))
    # the stepper carries T ~ 1 in absolute FP64: a few ulps of 1.0 of rounding
    assert np.abs(Tm - To).max() < 2e-14 and np.abs(qxm - qxo).max() < 1e-15
    ys, xs = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    Ta, _, qya = sol.at(xs, ys)
    assert np.abs(Ta - To).max() < 2e-14 and np.abs(qya - qyo).max() < 1e-15
