"""Seeded synthetic inputs for the phonon lattice Boltzmann workloads (D2Q8, and
periodic D3Q14 boxes).

This module holds no arithmetic of the lattice Boltzmann scheme.  It only
describes grid shapes, relaxation-time pairs, boundary kinds and wall values,
and builds initial temperature fields from fixed seeds.  The HIP path (its
tests and ``bench.py``) and the oracle tests both take their inputs from here,
so the two sides never exchange data with each other.

All quantities are in lattice units: node spacing, time step and lattice speed
are 1, and the volumetric heat capacity is ``cv`` (1 unless a case says
otherwise).  ``tau_n`` and ``tau_r`` are the normal and resistive relaxation
times divided by the time step (the paper's tau_r = tau_R / dt convention,
Sec. 2.4).  Boundary kinds are plain strings so that neither side's enums leak
into the other:

* ``"periodic"``   plain wrap-around,
* ``"isothermal"`` wall nodes held at a temperature (Sec. 2.5, Eq. 55),
* ``"diffuse"``    adiabatic diffuse reflection (Sec. 2.5, Eq. 58),
* ``"gradient"``   periodic temperature-gradient seam (Sec. 2.5, Eqs. 59-60),
  x axis only, with reference ramp ``T_ref(x) = t0 - grad_x * x`` and a jump
  of ``grad_x * nx`` across the seam.

Wall temperatures are listed as ``t_wall = (x=0, x=nx-1, y=0, y=ny-1)``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

SEED = 1847

BC_KINDS = ("periodic", "isothermal", "diffuse", "gradient")


@dataclasses.dataclass
class Case:
    """One lattice instance: geometry, relaxation times, boundaries, init."""

    name: str
    nx: int
    ny: int
    tau_n: float
    tau_r: float
    bc_x: str = "periodic"
    bc_y: str = "periodic"
    t0: float = 1.0
    cv: float = 1.0
    t_wall: Tuple[float, float, float, float] = (0.0, 0.0, 0.0, 0.0)
    q_wall: Tuple[float, float, float, float] = (0.0, 0.0, 0.0, 0.0)
    wall_bc: Tuple = (0, 0, 0, 0)   # per-wall kind overriding the axis kind (0 = the axis kind)
    grad_x: float = 0.0
    steps: int = 0
    init: str = "uniform"          # "uniform" | "gaussian" | "modes" | "field"
    init_args: dict = dataclasses.field(default_factory=dict)

    def t_ref(self) -> np.ndarray:
        """Reference temperature per column: t0, or the gradient ramp."""
        x = np.arange(self.nx, dtype=np.float64)
        if self.bc_x == "gradient":
            return self.t0 - self.grad_x * x
        return np.full(self.nx, self.t0)


# --------------------------------------------------------------------------
# initial temperature fields
# --------------------------------------------------------------------------

def gaussian_field(nx: int, ny: int, cx: float, cy: float, amp: float,
                   sigma: float, t0: float, rows: Optional[Sequence[int]] = None
                   ) -> np.ndarray:
    """t0 + amp * exp(-r^2 / (2 sigma^2)) around (cx, cy); shape (ny, nx)."""
    x = np.arange(nx, dtype=np.float64)
    y = np.arange(ny, dtype=np.float64) if rows is None else np.asarray(rows, dtype=np.float64)
    gx = np.exp(-((x - cx) ** 2) / (2.0 * sigma * sigma))
    gy = np.exp(-((y - cy) ** 2) / (2.0 * sigma * sigma))
    return t0 + amp * np.outer(gy, gx)


@dataclasses.dataclass
class Mode:
    """One real Fourier mode amp * cos(2 pi (kx x / nx + ky y / ny) + phase)."""
    kx: int
    ky: int
    amp: float
    phase: float


def draw_modes(n_modes: int = 16, kmax: int = 16, amp_total: float = 1e-3,
               seed: int = SEED) -> List[Mode]:
    """Distinct integer wave numbers in [-kmax, kmax]^2 minus (0,0), no +/- pairs.

    Amplitude amp_total / n_modes each, phases uniform in [0, 2 pi)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    modes: List[Mode] = []
    seen = set()
    while len(modes) < n_modes:
        kx, ky = (int(v) for v in rng.integers(-kmax, kmax + 1, size=2))
        if (kx, ky) == (0, 0) or (kx, ky) in seen or (-kx, -ky) in seen:
            continue
        seen.add((kx, ky))
        modes.append(Mode(kx, ky, amp_total / n_modes, float(rng.uniform(0.0, 2.0 * math.pi))))
    return modes


def modes_field(modes: Sequence[Mode], nx: int, ny: int, t0: float,
                rows: Optional[Sequence[int]] = None) -> np.ndarray:
    """t0 + sum of modes on the grid (or on the listed rows); shape (len(rows), nx).

    Built as a sum of separable outer products so a 16384^2 field costs
    16 outer products, not 16 full transcendental passes."""
    x = np.arange(nx, dtype=np.float64)
    y = np.arange(ny, dtype=np.float64) if rows is None else np.asarray(rows, dtype=np.float64)
    out = np.full((y.size, nx), t0, dtype=np.float64)
    for m in modes:
        ex = np.exp(1j * (2.0 * math.pi * m.kx * x / nx + m.phase))
        ey = np.exp(1j * (2.0 * math.pi * m.ky * y / ny))
        out += m.amp * np.real(np.outer(ey, ex))
    return out


def modes_field_torch(modes: Sequence[Mode], nx: int, ny: int, t0: float, device,
                      dtype=None):
    """Same field as :func:`modes_field`, built with torch on ``device``.

    Used to place a 16384^2 initial field in device memory without a 2 GB
    host round trip; it evaluates the identical separable formula."""
    import torch
    dtype = dtype or torch.float64
    x = torch.arange(nx, dtype=torch.float64, device=device)
    y = torch.arange(ny, dtype=torch.float64, device=device)
    out = torch.full((ny, nx), t0, dtype=torch.float64, device=device)
    for m in modes:
        ax = 2.0 * math.pi * m.kx * x / nx + m.phase
        ay = 2.0 * math.pi * m.ky * y / ny
        # cos(a + b) = cos a cos b - sin a sin b, as two rank-1 updates
        out.addr_(torch.cos(ay), torch.cos(ax), alpha=m.amp)
        out.addr_(torch.sin(ay), torch.sin(ax), alpha=-m.amp)
    return out.to(dtype)


def initial_field(case: Case, rows: Optional[Sequence[int]] = None) -> np.ndarray:
    """Initial temperature field of a case, shape (ny, nx) (or listed rows)."""
    nrow = case.ny if rows is None else len(rows)
    if case.init == "uniform":
        return np.tile(case.t_ref(), (nrow, 1))
    if case.init == "gaussian":
        a = case.init_args
        return gaussian_field(case.nx, case.ny, a["cx"], a["cy"], a["amp"], a["sigma"],
                              case.t0, rows)
    if case.init == "modes":
        return modes_field(case.init_args["modes"], case.nx, case.ny, case.t0, rows)
    if case.init == "field":
        f = np.asarray(case.init_args["T"], dtype=np.float64)
        return f if rows is None else f[np.asarray(rows)]
    raise ValueError(f"unknown init {case.init!r}")


def random_field(nx: int, ny: int, amp: float, t0: float, seed: int) -> np.ndarray:
    """Uniform random field t0 + amp * U[-1, 1) (rough; for parity tests only)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return t0 + amp * rng.uniform(-1.0, 1.0, size=(ny, nx))


def random_flux(nx: int, ny: int, amp: float, seed: int) -> Tuple[np.ndarray, np.ndarray]:
    rng = np.random.Generator(np.random.PCG64(seed))
    return (amp * rng.uniform(-1.0, 1.0, size=(ny, nx)),
            amp * rng.uniform(-1.0, 1.0, size=(ny, nx)))


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

def wall_case(nx: int = 128, ny: int = 64, tau_n: float = 0.6, tau_r: float = 0.8,
              t0: float = 1.0, dT: float = 0.5, steps: int = 5000) -> Case:
    """Isothermal walls at x = 0 (t0 + dT) and x = nx-1 (t0 - dT), periodic in y,
    uniform t0 init.  Default: the 128 x 64 case, 5000 steps."""
    return Case("walls", nx, ny, tau_n, tau_r, bc_x="isothermal", bc_y="periodic",
                t0=t0, t_wall=(t0 + dT, t0 - dT, 0.0, 0.0), steps=steps)


POISEUILLE_RATIOS = (10.0, 100.0, 1000.0)
POISEUILLE_TAU_N = (0.51, 0.6, 0.7, 0.8)


def poiseuille_case(tau_n: float, ratio: float, nx: int = 1024, ny: int = 256,
                    grad_x: float = 1e-3, t0: float = 1.0, steps: int = 0) -> Case:
    """Channel: gradient seam in x (G = grad_x per node), diffuse walls at
    y = 0 and y = ny-1, start from the ramp (zero deviation)."""
    return Case(f"poiseuille_tn{tau_n}_r{ratio:g}", nx, ny, tau_n, tau_n * ratio,
                bc_x="gradient", bc_y="diffuse", t0=t0, grad_x=grad_x, steps=steps)


# Sec. 3.4 heat pulse: Kn_N and the three Kn_R values, pulse length 100 tau_N
HEAT_PULSE_KN_N = 1.29e-3
HEAT_PULSE_KN_R = (1.29e3, 1.29, 1.29e-3)


def heat_pulse_case(tau_n: float, tau_r: float, nodes: int = 401, ny: int = 3,
                    q0: float = 1e-3, t0: float = 1.0) -> Case:
    """Plate of nodes - 1 spacings along x, heat-flux wall at x = 0 carrying q0
    into the plate (switched off by the caller after the pulse), adiabatic
    (heat-flux wall with zero flux) at x = nodes - 1, periodic in y (1D), at
    T0 everywhere with no heat flux."""
    return Case(f"heat_pulse_{nodes}_{tau_r:g}", nodes, ny, tau_n, tau_r, bc_x="heatflux",
                bc_y="periodic", t0=t0, q_wall=(q0, 0.0, 0.0, 0.0))


def square_case(nodes: int, tau_n: float, tau_r: float, q0: float = 1e-3, t_c: float = 1.0) -> Case:
    """Sec. 3.1.2 square: heat flux q0 into the domain through the top wall
    (y = nodes - 1), the other three walls isothermal at t_c, uniform start."""
    return Case(f"square_{nodes}", nodes, nodes, tau_n, tau_r, bc_x="isothermal", bc_y="isothermal",
                t0=t_c, t_wall=(t_c, t_c, t_c, t_c), q_wall=(0.0, 0.0, 0.0, q0),
                wall_bc=(0, 0, 0, "heatflux"))


def poiseuille_cases(**kw) -> List[Case]:
    return [poiseuille_case(tn, r, **kw) for r in POISEUILLE_RATIOS for tn in POISEUILLE_TAU_N]


def second_sound_case(n: int = 8192, tau_n: float = 0.55, tau_r: float = 50.0,
                      amp: float = 0.01, sigma: float = 20.0, steps: int = 4000) -> Case:
    """Periodic n x n, Gaussian pulse amp * exp(-r^2 / (2 sigma^2)) on T0 = 1 at
    node (n/2, n/2)."""
    return Case(f"second_sound_{n}", n, n, tau_n, tau_r, t0=1.0, steps=steps,
                init="gaussian",
                init_args=dict(cx=n // 2, cy=n // 2, amp=amp, sigma=sigma))


def smooth_modes_case(n: int = 16384, tau_n: float = 0.6, tau_r: float = 5.0,
                      steps: int = 1000, seed: int = SEED, n_modes: int = 16,
                      kmax: int = 16, amp_total: float = 1e-3) -> Case:
    """Periodic n x n, T0 = 1 plus n_modes seeded Fourier modes of total
    amplitude amp_total (integer wave numbers up to kmax per axis)."""
    return Case(f"smooth_modes_{n}", n, n, tau_n, tau_r, t0=1.0, steps=steps,
                init="modes", init_args=dict(modes=draw_modes(n_modes, kmax, amp_total, seed)))


def knudsen_sweep(n_inst: int = 256, seed: int = SEED, side_lo: int = 64,
                  side_hi: int = 512, tau_n_lo: float = 0.51, tau_n_hi: float = 1.0,
                  tau_r_lo: float = 0.6, tau_r_hi: float = 1000.0, grad_x: float = 1e-3,
                  steps: int = 10000) -> List[Case]:
    """Independent channel instances of uneven size and (tau_n, tau_r):
    nx, ny uniform integers in [side_lo, side_hi], tau_n uniform, tau_r
    log-uniform; boundaries as the Poiseuille channel."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nx = rng.integers(side_lo, side_hi + 1, size=n_inst)
    ny = rng.integers(side_lo, side_hi + 1, size=n_inst)
    tn = rng.uniform(tau_n_lo, tau_n_hi, size=n_inst)
    tr = np.exp(rng.uniform(math.log(tau_r_lo), math.log(tau_r_hi), size=n_inst))
    return [Case(f"sweep_{k}", int(nx[k]), int(ny[k]), float(tn[k]), float(tr[k]),
                 bc_x="gradient", bc_y="diffuse", t0=1.0, grad_x=grad_x, steps=steps)
            for k in range(n_inst)]


# --------------------------------------------------------------------------
# three-dimensional (D3Q14) lattices: fully periodic boxes
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Mode3:
    """One real Fourier mode amp * cos(2 pi (kx x/nx + ky y/ny + kz z/nz) + phase)."""
    kx: int
    ky: int
    kz: int
    amp: float
    phase: float


@dataclasses.dataclass
class Case3D:
    """One periodic nx x ny x nz box: relaxation times and initial field.
    Fields are (nz, ny, nx) arrays, x fastest."""

    name: str
    nx: int
    ny: int
    nz: int
    tau_n: float
    tau_r: float
    t0: float = 1.0
    cv: float = 1.0
    steps: int = 0
    init: str = "uniform"          # "uniform" | "modes" | "gaussian" | "field"
    init_args: dict = dataclasses.field(default_factory=dict)

    @property
    def nodes(self) -> int:
        return self.nx * self.ny * self.nz


def draw_modes_3d(n_modes: int = 16, kmax: int = 8, amp_total: float = 1e-3,
                  seed: int = SEED) -> List[Mode3]:
    """Distinct integer wave vectors in [-kmax, kmax]^3 minus 0, no +/- pairs,
    amplitude amp_total / n_modes each, phases uniform in [0, 2 pi)."""
    rng = np.random.Generator(np.random.PCG64(seed + 3))
    modes: List[Mode3] = []
    seen = set()
    while len(modes) < n_modes:
        k = tuple(int(v) for v in rng.integers(-kmax, kmax + 1, size=3))
        if k == (0, 0, 0) or k in seen or tuple(-v for v in k) in seen:
            continue
        seen.add(k)
        modes.append(Mode3(*k, amp_total / n_modes, float(rng.uniform(0.0, 2.0 * math.pi))))
    return modes


def modes_field_3d(modes: Sequence[Mode3], nx: int, ny: int, nz: int, t0: float) -> np.ndarray:
    """t0 + sum of modes on the whole box, shape (nz, ny, nx)."""
    x = np.arange(nx, dtype=np.float64)
    y = np.arange(ny, dtype=np.float64)
    z = np.arange(nz, dtype=np.float64)
    out = np.full((nz, ny, nx), t0, dtype=np.float64)
    for m in modes:
        ex = np.exp(1j * (2.0 * math.pi * m.kx * x / nx + m.phase))
        ey = np.exp(1j * (2.0 * math.pi * m.ky * y / ny))
        ez = np.exp(1j * (2.0 * math.pi * m.kz * z / nz))
        out += m.amp * np.real(ez[:, None, None] * ey[None, :, None] * ex[None, None, :])
    return out


def modes_field_3d_torch(modes: Sequence[Mode3], nx: int, ny: int, nz: int, t0: float, device):
    """Same field as :func:`modes_field_3d`, built with torch on ``device`` in
    FP64, so a 512^3 field needs no host copy."""
    import torch
    x = torch.arange(nx, dtype=torch.float64, device=device)
    y = torch.arange(ny, dtype=torch.float64, device=device)
    z = torch.arange(nz, dtype=torch.float64, device=device)
    out = torch.full((nz, ny, nx), t0, dtype=torch.float64, device=device)
    for m in modes:
        ph = ((2.0 * math.pi * m.kz / nz) * z[:, None, None] + (2.0 * math.pi * m.ky / ny) * y[None, :, None]
              + (2.0 * math.pi * m.kx / nx) * x[None, None, :] + m.phase)
        out.add_(torch.cos(ph), alpha=m.amp)
    return out


def gaussian_field_3d(nx: int, ny: int, nz: int, center, amp: float, sigma: float,
                      t0: float) -> np.ndarray:
    """t0 + amp * exp(-r^2 / (2 sigma^2)) around center = (cx, cy, cz); (nz, ny, nx)."""
    g = [np.exp(-((np.arange(n, dtype=np.float64) - c) ** 2) / (2.0 * sigma * sigma))
         for n, c in zip((nx, ny, nz), center)]
    return t0 + amp * g[2][:, None, None] * g[1][None, :, None] * g[0][None, None, :]


def random_field_3d(nx: int, ny: int, nz: int, amp: float, t0: float, seed: int) -> np.ndarray:
    """Uniform random field t0 + amp * U[-1, 1) (rough; parity tests only)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return t0 + amp * rng.uniform(-1.0, 1.0, size=(nz, ny, nx))


def random_flux_3d(nx: int, ny: int, nz: int, amp: float, seed: int):
    rng = np.random.Generator(np.random.PCG64(seed))
    return tuple(amp * rng.uniform(-1.0, 1.0, size=(nz, ny, nx)) for _ in range(3))


def initial_field_3d(case: Case3D) -> np.ndarray:
    """Initial temperature field of a 3D case, shape (nz, ny, nx)."""
    shape = (case.nz, case.ny, case.nx)
    if case.init == "uniform":
        return np.full(shape, case.t0)
    if case.init == "modes":
        return modes_field_3d(case.init_args["modes"], case.nx, case.ny, case.nz, case.t0)
    if case.init == "gaussian":
        a = case.init_args
        return gaussian_field_3d(case.nx, case.ny, case.nz, a["center"], a["amp"], a["sigma"], case.t0)
    if case.init == "field":
        return np.asarray(case.init_args["T"], dtype=np.float64).reshape(shape)
    raise ValueError(f"unknown init {case.init!r}")


def thermal_waves_3d_case(n: int = 512, tau_n: float = 0.6, tau_r: float = 5.0,
                          steps: int = 200, seed: int = SEED, n_modes: int = 16,
                          kmax: int = 8, amp_total: float = 1e-3) -> Case3D:
    """Periodic n^3 box, T0 = 1 plus n_modes seeded Fourier modes (integer wave
    numbers up to kmax per axis, total amplitude amp_total), no initial flux."""
    return Case3D(f"thermal_waves_{n}", n, n, n, tau_n, tau_r, t0=1.0, steps=steps,
                  init="modes", init_args=dict(modes=draw_modes_3d(n_modes, kmax, amp_total, seed)))


def second_sound_3d_case(n: int = 96, tau_n: float = 0.55, tau_r: float = 50.0,
                         amp: float = 0.01, sigma: float = 4.0, steps: int = 40) -> Case3D:
    """Periodic n^3 box, Gaussian pulse amp * exp(-r^2 / (2 sigma^2)) on T0 = 1 at
    the centre node."""
    return Case3D(f"second_sound_3d_{n}", n, n, n, tau_n, tau_r, t0=1.0, steps=steps,
                  init="gaussian", init_args=dict(center=(n // 2, n // 2, n // 2), amp=amp, sigma=sigma))
