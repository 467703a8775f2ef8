"""Exact evolution of the D2Q8 phonon lattice Boltzmann scheme on periodic grids.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

On a fully periodic grid the scheme of Sec. 2.2 is linear and shift
invariant, so each discrete Fourier mode evolves on its own.  For a mode with
wave vector k the state vector of the 8 populations advances by

    e_hat(k, n+1) = D(k) C e_hat(k, n),   D(k) = diag(exp(-i k . c_i)),

where C is the single-node relaxation matrix assembled from Eq. 13 with the
equilibrium of Eq. 15, the source of Eq. 16 and the moments of Eqs. 53-54, and
D(k) is the advection e_i(x + c_i) <- e*_i(x) of Eq. 13's left-hand side in
Fourier space (field convention f(x) = sum_k f_hat(k) exp(i k . x)).  The state
after n steps is therefore the matrix power (D C)^n applied to the initial
spectrum: no time-stepping, and no code shared with the C stepper.  Powers are
taken by binary exponentiation on stacks of 8x8 complex matrices.
"""
from __future__ import annotations

import math
from typing import Dict, Iterable, Optional, Sequence, Tuple

import numpy as np

# Eq. 14 velocities (c = 1), paper numbering 1..8 as rows 0..7
C = np.array([[1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]],
             dtype=np.float64)
OMEGA = np.array([2 / 9] * 4 + [1 / 36] * 4)      # Eq. 17
A_W = np.array([1 / 5] * 4 + [1 / 20] * 4)        # Eq. 18


def relaxation_params(tau_n: float, tau_r: float) -> Dict[str, float]:
    """tau (Eq. 49 with 1/tau_C = 1/tau_N + 1/tau_R) and the Eq. 54 factor."""
    inv_tc = 1.0 / tau_n + (0.0 if math.isinf(tau_r) else 1.0 / tau_r)
    tau = 1.0 / inv_tc + 0.5
    beta = 1.0 if math.isinf(tau_r) else 2.0 * tau_r / (2.0 * tau_r + 1.0)
    return dict(tau=tau, beta=beta, tau_c=1.0 / inv_tc)


def collision_matrix(tau_n: float, tau_r: float, cv: float = 1.0) -> np.ndarray:
    """8x8 real matrix of one node's relaxation e -> e* (Eq. 13 right-hand side).

    Rows of the moment map: C_V T = 1^T e (Eq. 53), q = beta C^T e (Eq. 54).
    e^eq = omega C_V T + (5/3) diag(a) C q   (Eq. 15, c = 1)
    S    = -(1 - 1/(2 tau)) (5/3) diag(a) C q / tau_r   (Eq. 16, dt = 1)
    e*   = e + (e^eq - e) / tau + S."""
    p = relaxation_params(tau_n, tau_r)
    tau, beta = p["tau"], p["beta"]
    ones = np.ones(8)
    to_q = beta * C.T                                   # 2x8: q from e
    eq = np.outer(OMEGA, ones) + (5.0 / 3.0) * np.diag(A_W) @ C @ to_q
    src = np.zeros((8, 8)) if math.isinf(tau_r) else \
        -(1.0 - 1.0 / (2.0 * tau)) * (5.0 / 3.0) * np.diag(A_W) @ C @ to_q / tau_r
    return np.eye(8) + (eq - np.eye(8)) / tau + src


def step_matrices(kx: np.ndarray, ky: np.ndarray, tau_n: float, tau_r: float) -> np.ndarray:
    """Stack of one-step matrices D(k) C for wave vectors (kx, ky); shape (N, 8, 8)."""
    kx = np.asarray(kx, dtype=np.float64).ravel()
    ky = np.asarray(ky, dtype=np.float64).ravel()
    phase = np.exp(-1j * (np.outer(kx, C[:, 0]) + np.outer(ky, C[:, 1])))   # (N, 8)
    return phase[:, :, None] * collision_matrix(tau_n, tau_r)[None, :, :]


def power_apply(M: np.ndarray, v: np.ndarray, n: int) -> np.ndarray:
    """M^n v for stacks M (N,8,8), v (N,8), by binary exponentiation."""
    v = v.astype(np.complex128, copy=True)
    P = M.astype(np.complex128, copy=True)
    n = int(n)
    while n > 0:
        if n & 1:
            v = np.einsum("nij,nj->ni", P, v)
        n >>= 1
        if n:
            P = P @ P
    return v


def _wave_numbers(nx: int, ny: int) -> Tuple[np.ndarray, np.ndarray]:
    kx = 2.0 * np.pi * np.fft.fftfreq(nx)
    ky = 2.0 * np.pi * np.fft.fftfreq(ny)
    KY, KX = np.meshgrid(ky, kx, indexing="ij")        # (ny, nx), matches fft2 layout
    return KX, KY


def evolve_populations(e0: np.ndarray, n: int, tau_n: float, tau_r: float) -> np.ndarray:
    """Exact state after n steps from any initial populations e0 (8, ny, nx)."""
    _, ny, nx = e0.shape
    KX, KY = _wave_numbers(nx, ny)
    eh = np.fft.fft2(e0, axes=(1, 2)).reshape(8, -1).T          # (N, 8)
    M = step_matrices(KX, KY, tau_n, tau_r)
    eh = power_apply(M, eh, n)
    return np.real(np.fft.ifft2(eh.T.reshape(8, ny, nx), axes=(1, 2)))


def moments_of(e: np.ndarray, tau_r: float, cv: float = 1.0):
    """(T, q_x, q_y) of populations (8, ny, nx): Eqs. 53-54."""
    beta = relaxation_params(1.0, tau_r)["beta"]
    T = e.sum(axis=0) / cv
    qx = beta * np.tensordot(C[:, 0], e, axes=1)
    qy = beta * np.tensordot(C[:, 1], e, axes=1)
    return T, qx, qy


def evolve_temperature_field(T0: np.ndarray, n: int, tau_n: float, tau_r: float,
                             t0: float = 1.0, cv: float = 1.0, rel_cut: float = 1e-15
                             ) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Exact (T, q_x, q_y) after n steps from the equilibrium of T0 with zero
    flux (e_i = omega_i C_V T0, Eq. 15), on a periodic grid.

    Modes whose initial amplitude is below rel_cut times the largest are not
    evolved (the Bloch matrices have spectral radius <= 1 in the tested
    regimes, so the dropped part stays below that level)."""
    ny, nx = T0.shape
    dT = np.asarray(T0, dtype=np.float64) - t0
    Th = np.fft.fft2(dT)
    mag = np.abs(Th)
    keep = mag > rel_cut * mag.max() if mag.max() > 0 else np.zeros_like(mag, bool)
    KX, KY = _wave_numbers(nx, ny)
    eh0 = (cv * Th[keep])[:, None] * OMEGA[None, :]
    M = step_matrices(KX[keep], KY[keep], tau_n, tau_r)
    eh = power_apply(M, eh0, n)
    beta = relaxation_params(tau_n, tau_r)["beta"]
    out = []
    for row in (np.ones(8) / cv, beta * C[:, 0], beta * C[:, 1]):
        F = np.zeros((ny, nx), dtype=np.complex128)
        F[keep] = eh @ row
        out.append(np.real(np.fft.ifft2(F)))
    return out[0] + t0, out[1], out[2]


class ModeSolution:
    """Exact solution for an initial field t0 + sum_m amp_m cos(2 pi (kx_m x / nx
    + ky_m y / ny) + phase_m) with zero flux, evaluable at any node set."""

    def __init__(self, modes: Sequence, nx: int, ny: int, n: int, tau_n: float,
                 tau_r: float, t0: float = 1.0, cv: float = 1.0):
        self.nx, self.ny, self.t0, self.cv = nx, ny, t0, cv
        self.kx = np.array([2 * np.pi * m.kx / nx for m in modes])
        self.ky = np.array([2 * np.pi * m.ky / ny for m in modes])
        # cos(theta + phase) = Re[exp(i phase) exp(i theta)]: the +k half carries
        # amp exp(i phase) / 2 and the -k half is its complex conjugate.
        amp = np.array([m.amp * np.exp(1j * m.phase) / 2.0 for m in modes])
        eh0 = (cv * amp)[:, None] * OMEGA[None, :]
        M = step_matrices(self.kx, self.ky, tau_n, tau_r)
        self.eh = power_apply(M, eh0, n)                       # (M, 8)
        beta = relaxation_params(tau_n, tau_r)["beta"]
        self.coef = np.stack([self.eh @ (np.ones(8) / cv),
                              self.eh @ (beta * C[:, 0]),
                              self.eh @ (beta * C[:, 1])])     # (3, M)

    def at(self, xs: np.ndarray, ys: np.ndarray):
        """(T, q_x, q_y) at nodes (xs, ys) (any matching shapes)."""
        xs = np.asarray(xs, dtype=np.float64)
        ys = np.asarray(ys, dtype=np.float64)
        ph = np.exp(1j * (np.multiply.outer(xs, self.kx) + np.multiply.outer(ys, self.ky)))
        vals = 2.0 * np.real(ph @ self.coef.T)                # (..., 3)
        return vals[..., 0] + self.t0, vals[..., 1], vals[..., 2]

    def rows(self, ys: Iterable[int]):
        """(T, q_x, q_y) on whole rows ys, shape (len(ys), nx); separable evaluation."""
        ys = np.asarray(list(ys), dtype=np.float64)
        x = np.arange(self.nx, dtype=np.float64)
        ex = np.exp(1j * np.multiply.outer(self.kx, x))        # (M, nx)
        ey = np.exp(1j * np.multiply.outer(ys, self.ky))       # (R, M)
        out = [2.0 * np.real((ey * c[None, :]) @ ex) for c in self.coef]
        return out[0] + self.t0, out[1], out[2]


def slow_eigenvalues(k: float, theta: float, tau_n: float, tau_r: float, count: int = 3
                     ) -> np.ndarray:
    """The `count` eigenvalues of D(k) C of largest modulus for a wave vector of
    length k at angle theta (per-step growth factors of the slow modes)."""
    M = step_matrices(np.array([k * math.cos(theta)]), np.array([k * math.sin(theta)]),
                      tau_n, tau_r)[0]
    lam = np.linalg.eigvals(M)
    return lam[np.argsort(-np.abs(lam))][:count]


class SeparableSolution:
    """Exact solution from T0 = t0 + amp * fy(y) fx(x) (periodic, zero flux),
    evaluated on chosen rows.

    The spectrum of a separable field is the outer product of two 1D FFTs; only
    wave numbers whose 1D amplitude exceeds rel_cut times the largest are kept
    (a box of modes), each advanced by its matrix power.  Rows are then
    synthesised by two dense products, so a 8192^2 lattice needs no 2D FFT."""

    def __init__(self, fx: np.ndarray, fy: np.ndarray, amp: float, n: int, tau_n: float, tau_r: float,
                 t0: float = 1.0, cv: float = 1.0, rel_cut: float = 1e-15):
        self.nx, self.ny, self.t0 = fx.size, fy.size, t0
        Fx, Fy = np.fft.fft(fx), np.fft.fft(fy)
        ix = np.nonzero(np.abs(Fx) > rel_cut * np.abs(Fx).max())[0]
        iy = np.nonzero(np.abs(Fy) > rel_cut * np.abs(Fy).max())[0]
        self.kx = 2.0 * np.pi * np.fft.fftfreq(self.nx)[ix]
        self.ky = 2.0 * np.pi * np.fft.fftfreq(self.ny)[iy]
        KY, KX = np.meshgrid(self.ky, self.kx, indexing="ij")           # (my, mx)
        spec = amp * np.outer(Fy[iy], Fx[ix])                           # T_hat - t0 part
        eh0 = (cv * spec.ravel())[:, None] * OMEGA[None, :]
        M = step_matrices(KX, KY, tau_n, tau_r)
        eh = power_apply(M, eh0, n)
        beta = relaxation_params(tau_n, tau_r)["beta"]
        shape = (self.ky.size, self.kx.size)
        self.E = (eh @ (np.ones(8) / cv)).reshape(shape)
        self.Qx = (eh @ (beta * C[:, 0])).reshape(shape)
        self.Qy = (eh @ (beta * C[:, 1])).reshape(shape)
        self.n_modes = self.E.size

    def rows(self, ys):
        """(T, q_x, q_y) on rows ys, each (len(ys), nx)."""
        ys = np.asarray(list(ys), dtype=np.float64)
        A = np.exp(1j * np.multiply.outer(ys, self.ky))                 # (R, my)
        B = np.exp(1j * np.multiply.outer(self.kx, np.arange(self.nx)))  # (mx, nx)
        norm = 1.0 / (self.nx * self.ny)
        out = [np.real(A @ F @ B) * norm for F in (self.E, self.Qx, self.Qy)]
        return out[0] + self.t0, out[1], out[2]
