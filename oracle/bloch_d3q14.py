"""Exact evolution of the D3Q14 phonon lattice Boltzmann scheme on periodic grids.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The same construction as ``bloch`` for D2Q8: on a fully periodic grid the
scheme (Eq. 13 with Eqs. 15-16 and the moments of Eqs. 53-54) is linear and
shift invariant, so a Fourier mode of wave vector k advances by the 14x14
matrix D(k) C, D(k) = diag(exp(-i k . c_i)), C the single-node relaxation.

The weights are not typed in here: ``weights()`` solves the moment conditions
that the Chapman-Enskog recovery of Eq. 47 needs (Eqs. 22-25 for the
equilibrium, hence Eqs. 26-28 for the source, Sec. 2.3) over this velocity set,
as a least-squares problem that must come out exactly consistent.  The C
stepper carries the closed-form values of the same solution, so agreement
between the two checks both.
"""
from __future__ import annotations

import itertools
import math
from typing import Sequence, Tuple

import numpy as np

from .bloch import power_apply, relaxation_params

# 6 axis movers then 8 corner movers (c = 1), the stepper's order
C3 = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]]
              + [[sx, sy, sz] for sz in (1, -1) for sy in (1, -1) for sx in (1, -1)],
              dtype=np.float64)
IS_AXIS = np.abs(C3).sum(axis=1) == 1


def _solve_class_weights(rows, rhs) -> Tuple[float, float]:
    """Weights (axis, corner) from linear conditions on the two velocity classes."""
    A = np.array(rows, dtype=np.float64)
    b = np.array(rhs, dtype=np.float64)
    w, res, rank, _ = np.linalg.lstsq(A, b, rcond=None)
    assert rank == 2 and np.allclose(A @ w, b, rtol=0, atol=1e-14), "moment conditions inconsistent"
    return float(w[0]), float(w[1])


def weights() -> Tuple[np.ndarray, np.ndarray]:
    """(omega_i, a_i) for the 14 velocities, from the moment conditions.

    omega: sum omega = 1 (Eq. 22), sum omega c_x c_x = 5/9, sum omega c_x c_y = 0
    (Eq. 24).  a (with the 5/3 factor of Eq. 15): sum a c_x c_x = 3/5 (Eq. 23),
    sum a c_x^4 = 3/5 and sum a c_x^2 c_y^2 = 1/5 (Eq. 25: (5/3) sum a c c c c
    = (1/3)(dd + dd + dd)).  Each condition is written as the sum over the
    class members of the monomial, per class."""
    def per_class(f):
        v = np.array([f(c) for c in C3])
        return [v[IS_AXIS].sum(), v[~IS_AXIS].sum()]

    one = per_class(lambda c: 1.0)
    xx = per_class(lambda c: c[0] * c[0])
    xy = per_class(lambda c: c[0] * c[1])
    xxxx = per_class(lambda c: c[0] ** 4)
    xxyy = per_class(lambda c: c[0] ** 2 * c[1] ** 2)
    zzzz = per_class(lambda c: c[2] ** 4)
    yyzz = per_class(lambda c: c[1] ** 2 * c[2] ** 2)
    wa, wc = _solve_class_weights([one, xx, xy], [1.0, 5.0 / 9.0, 0.0])
    aa, ac = _solve_class_weights([xx, xxxx, xxyy, zzzz, yyzz], [0.6, 0.6, 0.2, 0.6, 0.2])
    omega = np.where(IS_AXIS, wa, wc)
    a = np.where(IS_AXIS, aa, ac)
    return omega, a


OMEGA3, A3 = weights()


def collision_matrix(tau_n: float, tau_r: float, cv: float = 1.0) -> np.ndarray:
    """14x14 real matrix of one node's relaxation e -> e* (Eq. 13 right-hand side)."""
    p = relaxation_params(tau_n, tau_r)
    tau, beta = p["tau"], p["beta"]
    to_q = beta * C3.T                                              # 3x14
    eq = np.outer(OMEGA3, np.ones(14)) + (5.0 / 3.0) * np.diag(A3) @ C3 @ to_q
    src = np.zeros((14, 14)) if math.isinf(tau_r) else \
        -(1.0 - 1.0 / (2.0 * tau)) * (5.0 / 3.0) * np.diag(A3) @ C3 @ to_q / tau_r
    return np.eye(14) + (eq - np.eye(14)) / tau + src


def step_matrices(k: np.ndarray, tau_n: float, tau_r: float) -> np.ndarray:
    """Stack of one-step matrices D(k) C for wave vectors k (N, 3); shape (N, 14, 14)."""
    k = np.asarray(k, dtype=np.float64).reshape(-1, 3)
    phase = np.exp(-1j * (k @ C3.T))                                # (N, 14)
    return phase[:, :, None] * collision_matrix(tau_n, tau_r)[None, :, :]


def evolve_populations(e0: np.ndarray, n: int, tau_n: float, tau_r: float) -> np.ndarray:
    """Exact state after n steps from any initial populations e0 (14, nz, ny, nx)."""
    _, nz, ny, nx = e0.shape
    kz, ky, kx = np.meshgrid(2 * np.pi * np.fft.fftfreq(nz), 2 * np.pi * np.fft.fftfreq(ny),
                             2 * np.pi * np.fft.fftfreq(nx), indexing="ij")
    K = np.stack([kx.ravel(), ky.ravel(), kz.ravel()], axis=1)
    eh = np.fft.fftn(e0, axes=(1, 2, 3)).reshape(14, -1).T
    eh = power_apply(step_matrices(K, tau_n, tau_r), eh, n)
    return np.real(np.fft.ifftn(eh.T.reshape(14, nz, ny, nx), axes=(1, 2, 3)))


def moments_of(e: np.ndarray, tau_r: float, cv: float = 1.0):
    """(T, q_x, q_y, q_z) of populations (14, ...): Eqs. 53-54."""
    beta = relaxation_params(1.0, tau_r)["beta"]
    return (e.sum(axis=0) / cv,) + tuple(beta * np.tensordot(C3[:, a], e, axes=1) for a in range(3))


def equilibrium(T: np.ndarray, q: Sequence[np.ndarray], tau_r: float, cv: float = 1.0) -> np.ndarray:
    """Populations (14, ...) of Eq. 15 whose Eq. 54 flux is q."""
    beta = relaxation_params(1.0, tau_r)["beta"]
    T = np.asarray(T, dtype=np.float64)
    cq = sum(np.multiply.outer(C3[:, a], np.asarray(q[a], dtype=np.float64) / beta) for a in range(3))
    return np.multiply.outer(OMEGA3, cv * T) + (5.0 / 3.0) * A3.reshape((14,) + (1,) * T.ndim) * cq


class ModeSolution:
    """Exact solution for T0 = t0 + sum_m amp_m cos(2 pi (kx x/nx + ky y/ny + kz z/nz)
    + phase_m) with zero initial flux, evaluable at any node set.  Each mode is
    an object with integer fields kx, ky, kz and float fields amp, phase."""

    def __init__(self, modes: Sequence, nx: int, ny: int, nz: int, n: int, tau_n: float,
                 tau_r: float, t0: float = 1.0, cv: float = 1.0):
        self.t0 = t0
        self.k = np.array([[2 * np.pi * m.kx / nx, 2 * np.pi * m.ky / ny, 2 * np.pi * m.kz / nz]
                           for m in modes])
        amp = np.array([m.amp * np.exp(1j * m.phase) / 2.0 for m in modes])
        eh0 = (cv * amp)[:, None] * OMEGA3[None, :]
        eh = power_apply(step_matrices(self.k, tau_n, tau_r), eh0, n)      # (M, 14)
        beta = relaxation_params(tau_n, tau_r)["beta"]
        self.coef = np.stack([eh @ (np.ones(14) / cv)] + [eh @ (beta * C3[:, a]) for a in range(3)])

    def at(self, xs, ys, zs):
        """(T, q_x, q_y, q_z) at nodes (xs, ys, zs) (matching shapes)."""
        pos = np.stack([np.asarray(v, dtype=np.float64) for v in (xs, ys, zs)], axis=-1)
        ph = np.exp(1j * (pos @ self.k.T))                                  # (..., M)
        vals = 2.0 * np.real(ph @ self.coef.T)                              # (..., 4)
        return vals[..., 0] + self.t0, vals[..., 1], vals[..., 2], vals[..., 3]


def slow_eigenvalues(k: np.ndarray, tau_n: float, tau_r: float, count: int = 3) -> np.ndarray:
    """The `count` eigenvalues of D(k) C of largest modulus for wave vector k (3,)."""
    lam = np.linalg.eigvals(step_matrices(np.asarray(k, dtype=np.float64), tau_n, tau_r)[0])
    return lam[np.argsort(-np.abs(lam))][:count]


def cube_symmetries():
    """The 48 signed axis permutations (P, s): v -> s * v[P]."""
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            yield perm, np.array(signs)
