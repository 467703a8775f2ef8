"""Analytic results of the paper used to pin the oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Everything is in lattice units (dx = dt = c = 1, so v_g = sqrt(5/3) by Eq. 48)
unless a function says it takes the paper's non-dimensional groups.
"""
from __future__ import annotations

import math
from typing import Tuple

import numpy as np

VG = math.sqrt(5.0 / 3.0)          # Eq. 48: c = sqrt(3/5) v_g with c = 1


# --------------------------------------------------------------------------
# parameter mapping (Eqs. 48-49, Sec. 3.4 closing discussion)
# --------------------------------------------------------------------------

def overall_knudsen(kn_n: float, kn_r: float) -> float:
    """1/Kn_C = 1/Kn_R + 1/Kn_N (Sec. 3 introduction)."""
    return 1.0 / (1.0 / kn_n + 1.0 / kn_r)


def tau_from_knudsen(n_cells: int, kn_c: float) -> float:
    """tau = 0.5 + sqrt(3/5) N_x Kn_C (from Eqs. 48-49; Sec. 3.4 discussion).

    n_cells is the number of lattice spacings across the length d."""
    return 0.5 + math.sqrt(3.0 / 5.0) * n_cells * kn_c


def lattice_relaxation_times(n_cells: int, kn_n: float, kn_r: float) -> Tuple[float, float]:
    """(tau_N/dt, tau_R/dt) for Knudsen numbers Kn = v_g tau / d on a length of
    n_cells spacings: tau/dt = Kn * n_cells * sqrt(3/5) (Eq. 48, dx = c dt)."""
    f = n_cells * math.sqrt(3.0 / 5.0)
    return kn_n * f, kn_r * f


def knudsen(tau_lattice: float, d_cells: float) -> float:
    """Kn = v_g tau / d in lattice units."""
    return VG * tau_lattice / d_cells


def scheme_constants(tau_n: float, tau_r: float) -> dict:
    """tau (Eq. 49), the Eq. 54 factor beta, and the per-step heat-flux decay
    rho = (2 tau_r - 1)/(2 tau_r + 1) that follows from Eqs. 13, 15, 16, 54
    (total heat flux on a periodic grid is multiplied by rho each step)."""
    inv_tc = 1.0 / tau_n + (0.0 if math.isinf(tau_r) else 1.0 / tau_r)
    tau_c = 1.0 / inv_tc
    if math.isinf(tau_r):
        beta, rho = 1.0, 1.0
    else:
        beta = 2.0 * tau_r / (2.0 * tau_r + 1.0)
        rho = (2.0 * tau_r - 1.0) / (2.0 * tau_r + 1.0)
    return dict(tau_c=tau_c, tau=tau_c + 0.5, beta=beta, rho=rho)


# --------------------------------------------------------------------------
# Sec. 3.1.1: 1D transient conduction between isothermal walls
# --------------------------------------------------------------------------

def fourier_1d_theta_eq61(X, t_star, kn_r, n_terms: int = 2000):
    """Eq. 61 as printed: film initially at T_c, left wall at T_h from t = 0."""
    X = np.asarray(X, dtype=np.float64)
    n = np.arange(1, n_terms + 1)[:, None]
    s = np.sum(np.sin(n * np.pi * X[None, :]) / n
               * np.exp(-kn_r ** 2 * n ** 2 * np.pi ** 2 * t_star / 3.0), axis=0)
    return 1.0 - X - 2.0 / np.pi * s


def fourier_1d_q_eq62(X, t_star, kn_r, n_terms: int = 2000):
    """Eq. 62 as printed (Q = q_x d / (lambda (T_h - T_c)))."""
    X = np.asarray(X, dtype=np.float64)
    n = np.arange(1, n_terms + 1)[:, None]
    s = np.sum(np.cos(n * np.pi * X[None, :])
               * np.exp(-kn_r ** 2 * n ** 2 * np.pi ** 2 * t_star / 3.0), axis=0)
    return 1.0 + 2.0 * s


def fourier_1d_theta(X, t, d, alpha, theta0: float, n_terms: int = 2000):
    """Same separation-of-variables solution as Eq. 61 for a film at uniform
    initial Theta = theta0: Theta = 1 - X + sum_n b_n sin(n pi X) exp(-n^2 pi^2
    alpha t / d^2), b_n = 2 int_0^1 (theta0 - 1 + X) sin(n pi X) dX.  With
    theta0 = 0 this is Eq. 61 (alpha t / d^2 = Kn_R^2 t* / 3)."""
    X = np.asarray(X, dtype=np.float64)
    n = np.arange(1, n_terms + 1)[:, None].astype(np.float64)
    sgn = (-1.0) ** n
    b = 2.0 * ((theta0 - 1.0) * (1.0 - sgn) / (n * np.pi) - sgn / (n * np.pi))
    return 1.0 - X + np.sum(b * np.sin(n * np.pi * X[None, :])
                            * np.exp(-n ** 2 * np.pi ** 2 * alpha * t / d ** 2), axis=0)


def diffusivity(tau_r: float) -> float:
    """Thermal diffusivity lambda / C_V = v_g^2 tau_R / 3 (Eq. 9 Fourier limit)."""
    return VG ** 2 * tau_r / 3.0


# --------------------------------------------------------------------------
# Sec. 3.2: in-plane transport, phonon Poiseuille flow
# --------------------------------------------------------------------------

def poiseuille_q_eq68(Y, kn_c: float, kn_r: float):
    """Eq. 68: Q_x(Y) with Kn_eff = sqrt(Kn_C Kn_R / 5)."""
    Y = np.asarray(Y, dtype=np.float64)
    k = math.sqrt(kn_c * kn_r / 5.0)
    e1 = math.exp(-1.0 / k)
    den = 1.0 + e1 + (8.0 / 15.0) * (kn_c / k) * (1.0 - e1)
    return 1.0 - (np.exp((Y - 1.0) / k) + np.exp(-Y / k)) / den


def poiseuille_conductivity_eq69(kn_c: float, kn_r: float) -> float:
    """Eq. 69: lambda_eff / lambda."""
    k = math.sqrt(kn_c * kn_r / 5.0)
    e1 = math.exp(-1.0 / k)
    den = 1.0 + e1 + (8.0 / 15.0) * (kn_c / k) * (1.0 - e1)
    return 1.0 - 2.0 * k * (1.0 - e1) / den


def poiseuille_q_scale(tau_r: float, grad: float, cv: float = 1.0) -> float:
    """Denominator of Q_x: -(1/3) C_V v_g^2 tau_R dT/dx with dT/dx = -grad."""
    return cv * VG ** 2 * tau_r * grad / 3.0


# --------------------------------------------------------------------------
# Sec. 3.3: cross-plane transport with temperature jump
# --------------------------------------------------------------------------

def cross_plane_theta_eq70(X, kn_r: float):
    X = np.asarray(X, dtype=np.float64)
    return -X / (1.0 + 4.0 / 3.0 * kn_r) + (1.0 + 2.0 / 3.0 * kn_r) / (1.0 + 4.0 / 3.0 * kn_r)


def cross_plane_q_eq71(kn_r: float) -> float:
    """Q = q_x / (C_V v_g (T_h - T_c))."""
    return kn_r / (3.0 * (1.0 + 4.0 / 3.0 * kn_r))


# --------------------------------------------------------------------------
# Eq. 52: temperature equation -> dispersion of plane waves
# --------------------------------------------------------------------------

def telegraph_rates(k: float, tau_r: float, tau_c: float) -> np.ndarray:
    """Growth rates s (per time step) of T ~ exp(s t + i k x) under Eq. 52:
    s^2 + s (1/tau_R + (4/15) tau_C v_g^2 k^2) + (1/3) v_g^2 k^2 = 0."""
    b = (0.0 if math.isinf(tau_r) else 1.0 / tau_r) + 4.0 / 15.0 * tau_c * VG ** 2 * k * k
    c0 = VG ** 2 * k * k / 3.0
    return np.roots([1.0, b, c0])


def second_sound_speed() -> float:
    """v_g / sqrt(3) (Sec. 3.4), = sqrt(5)/3 lattice nodes per step."""
    return VG / math.sqrt(3.0)


# --------------------------------------------------------------------------
# Sec. 3.4, Appendix B: heat pulse through a plate, hydrodynamic model
# (Eqs. 72-80) solved by the Laplace transform
# --------------------------------------------------------------------------

def heat_pulse_transforms(X, s, kn_n: float, kn_r: float, t_pulse: float = 100.0):
    """Laplace transforms (Theta_bar, Q_bar) at positions X (0..1) and complex
    s (broadcast against each other), Eqs. B9-B13 with the boundary data of
    Eq. B7 (pulse of t_pulse in units of tau_N).

    Eq. B10 with B12 is rewritten with decaying exponentials only,
    C1 e^{AX} = -C2 e^{-A(2-X)}, so large |A| cannot overflow; A is the root
    of Eq. B9 with positive real part."""
    X = np.asarray(X, dtype=np.float64)
    s = np.asarray(s, dtype=np.complex128)
    kn_c = overall_knudsen(kn_n, kn_r)
    A = np.sqrt((kn_r / kn_n * s + 1.0) / (kn_n * kn_r / (3.0 * s) + 4.0 / 15.0 * kn_c * kn_r))   # Eq. B9
    A = np.where(A.real < 0, -A, A)
    C2 = (1.0 - np.exp(-t_pulse * s)) / (s * (1.0 - np.exp(-2.0 * A)))                            # Eq. B11
    e1, e2 = np.exp(-A * X), np.exp(-A * (2.0 - X))
    Q = C2 * (e1 - e2)                                            # Eq. B10 with C1 = -C2 e^{-2A} (B12)
    Theta = kn_n / s * C2 * A * (e1 + e2)                         # Eq. B13
    return Theta, Q


def heat_pulse_solution(X, t_star: float, kn_n: float, kn_r: float, t_pulse: float = 100.0,
                        gamma_t: float = 3.0, n_terms: int = 200000, chunk: int = 20000):
    """Theta(X, t*) and Q(X, t*) of the hydrodynamic model (Eqs. 77-80) by the
    Riemann-sum inverse Laplace transform of Eqs. B14-B15 with gamma t* =
    gamma_t (3 in the paper), summed over n_terms terms.  Theta = (T - T0) C_V
    v_g / q0, Q = q_x / q0, t* = t / tau_N, X = x / d (Eq. 76)."""
    X = np.atleast_1d(np.asarray(X, dtype=np.float64))
    t = float(t_star)
    gam = gamma_t / t
    th0, q0 = heat_pulse_transforms(X, np.array([gam + 0j]), kn_n, kn_r, t_pulse)
    sum_t = 0.5 * th0.real.copy()
    sum_q = 0.5 * q0.real.copy()
    for start in range(1, n_terms + 1, chunk):
        n = np.arange(start, min(start + chunk, n_terms + 1), dtype=np.float64)
        s = gam + 1j * np.pi * n / t
        th, q = heat_pulse_transforms(X[None, :], s[:, None], kn_n, kn_r, t_pulse)
        sign = np.where(n % 2 == 1, -1.0, 1.0)[:, None]
        sum_t += (th * sign).real.sum(axis=0)
        sum_q += (q * sign).real.sum(axis=0)
    f = math.exp(gam * t) / t
    return f * sum_t, f * sum_q


def heat_pulse_diffusive_limit(X, t_star: float, kn_n: float, kn_r: float, t_pulse: float = 100.0):
    """Theta(X, t*) of Eqs. 77-78 in the limit Kn_R << Kn_N with Kn_C Kn_R
    negligible: Theta_t* = D Theta_XX, D = Kn_N Kn_R / 3, inflow Kn_N Q(0) with
    Q(0) the pulse of Eq. 80, X = 1 insulated.  For a constant inflow F from
    t* = 0 the solution is F t + (F/D)[(1 - X)^2/2 - 1/6]
    - (2F/D) sum_n cos(n pi X) exp(-D n^2 pi^2 t) / (n pi)^2; the pulse is that
    minus the same delayed by t_pulse."""
    X = np.asarray(X, dtype=np.float64)
    D, F = kn_n * kn_r / 3.0, kn_n
    n = np.arange(1, 20001, dtype=np.float64)

    def step(t):
        if t <= 0.0:
            return np.zeros_like(X)
        series = (np.cos(np.pi * np.multiply.outer(X, n)) * (np.exp(-D * (n * np.pi) ** 2 * t) / (n * np.pi) ** 2)).sum(axis=-1)
        return F * t + F / D * ((1.0 - X) ** 2 / 2.0 - 1.0 / 6.0) - 2.0 * F / D * series

    return step(float(t_star)) - step(float(t_star) - t_pulse)


# --------------------------------------------------------------------------
# Sec. 3.1.2: square with a heat flux on the top side, Fourier solution
# --------------------------------------------------------------------------

def square_eq65_67(X, Y, n_terms: int = 4000):
    """(Theta, Q_x, Q_y) / Q0 of Eqs. 65-67 (Fourier's law in the unit square,
    Theta = 0 on X = 0, X = 1, Y = 0, heat flux Q0 into the square through
    Y = 1).  The hyperbolic ratios are written with decaying exponentials
    (sinh(n pi Y) / cosh(n pi) and cosh(n pi Y) / cosh(n pi)), which is the
    same series without overflow."""
    X = np.asarray(X, dtype=np.float64)[..., None]
    Y = np.asarray(Y, dtype=np.float64)[..., None]
    n = np.arange(1, n_terms + 1, dtype=np.float64)
    k = n * np.pi
    odd = 1.0 - np.cos(k)                                   # 2 for odd n, 0 for even n
    den = 1.0 + np.exp(-2.0 * k)
    sh = (np.exp(k * (Y - 1.0)) - np.exp(-k * (Y + 1.0))) / den
    ch = (np.exp(k * (Y - 1.0)) + np.exp(-k * (Y + 1.0))) / den
    theta = (2.0 / k ** 2 * odd * np.sin(k * X) * sh).sum(axis=-1)          # Eq. 65
    qx = -(2.0 / k * odd * np.cos(k * X) * sh).sum(axis=-1)                # Eq. 66
    qy = -(2.0 / k * odd * np.sin(k * X) * ch).sum(axis=-1)                # Eq. 67
    return theta, qx, qy
