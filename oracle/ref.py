"""ctypes front end of the FP64 C time-stepper (``phonon_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product package.

The stepper follows the paper's order for one step (Sec. 2.2-2.5): moments
(Eqs. 53-54), equilibrium and source (Eqs. 15-16), relaxation (Eq. 13),
advection, then the boundary treatment of the unknown populations (Eqs. 55,
57, 58, 59-60).  The kept state is the pre-collision distribution at time n, so
``moments()`` after ``run(n)`` are the fields at time n.
"""
from __future__ import annotations

import ctypes
import os
import time
from typing import Optional, Tuple

import numpy as np

from . import build as _build

_BC = {"periodic": 0, "isothermal": 1, "diffuse": 2, "gradient": 3, "heatflux": 4}


class _Case(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("tau_n", ctypes.c_double), ("tau_r", ctypes.c_double),
                ("cv", ctypes.c_double),
                ("bc_x", ctypes.c_int), ("bc_y", ctypes.c_int),
                ("t0", ctypes.c_double), ("grad_x", ctypes.c_double),
                ("t_wall", ctypes.c_double * 4), ("q_wall", ctypes.c_double * 4),
                ("wall_kind", ctypes.c_int * 4)]


class _Case3(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("tau_n", ctypes.c_double), ("tau_r", ctypes.c_double),
                ("cv", ctypes.c_double), ("t0", ctypes.c_double)]


_lib = None


def lib():
    """Load the oracle library, compiling it first if it is missing or stale."""
    global _lib
    if _lib is None:
        src_m = max(os.path.getmtime(f) for f in _build.SRCS)
        if not os.path.exists(_build.LIB) or os.path.getmtime(_build.LIB) < src_m:
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        P = ctypes.POINTER
        d = P(ctypes.c_double)
        c = P(_Case)
        L.ora_check.argtypes = [c]
        L.ora_check.restype = ctypes.c_int
        L.ora_collide_node.argtypes = [c, d, d]
        L.ora_init.argtypes = [c, d, d, d, d]
        L.ora_run.argtypes = [c, d, d, ctypes.c_long]
        L.ora_moments.argtypes = [c, d, d, d, d]
        L.ora_totals.argtypes = [c, d, d]
        L.ora_max_threads.restype = ctypes.c_int
        L.ora_set_threads.argtypes = [ctypes.c_int]
        c3 = P(_Case3)
        L.ora3_check.argtypes = [c3]
        L.ora3_check.restype = ctypes.c_int
        L.ora3_collide_node.argtypes = [c3, d, d]
        L.ora3_init.argtypes = [c3, d, d, d, d, d]
        L.ora3_run.argtypes = [c3, d, d, ctypes.c_long]
        L.ora3_moments.argtypes = [c3, d, d, d, d, d]
        L.ora3_totals.argtypes = [c3, d, d]
        _lib = L
    return _lib


def _dptr(a: Optional[np.ndarray]):
    if a is None:
        return ctypes.POINTER(ctypes.c_double)()
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_case(case) -> _Case:
    """Build the C struct from a ``workloads.Case`` (or any object with the same fields)."""
    c = _Case()
    c.nx, c.ny = int(case.nx), int(case.ny)
    c.tau_n, c.tau_r = float(case.tau_n), float(case.tau_r)
    c.cv = float(getattr(case, "cv", 1.0))
    c.bc_x, c.bc_y = _BC[case.bc_x], _BC[case.bc_y]
    c.t0 = float(case.t0)
    c.grad_x = float(getattr(case, "grad_x", 0.0))
    for k, v in enumerate(getattr(case, "t_wall", (0.0,) * 4)):
        c.t_wall[k] = float(v)
    for k, v in enumerate(getattr(case, "q_wall", (0.0,) * 4)):
        c.q_wall[k] = float(v)
    for k, v in enumerate(getattr(case, "wall_bc", (0,) * 4)):
        c.wall_kind[k] = _BC[v] if isinstance(v, str) else int(v)
    return c


class Oracle:
    """One lattice instance advanced by the C stepper in FP64."""

    def __init__(self, case, T0: Optional[np.ndarray] = None,
                 qx: Optional[np.ndarray] = None, qy: Optional[np.ndarray] = None):
        self.case = case
        self.c = make_case(case)
        rc = lib().ora_check(ctypes.byref(self.c))
        if rc != 0:
            raise ValueError(f"oracle rejects case {case.name}: code {rc}")
        n = 8 * case.ny * case.nx
        self.e = np.zeros(n, dtype=np.float64)
        self.work = np.zeros(n, dtype=np.float64)
        if T0 is None:
            T0 = np.tile(case.t_ref(), (case.ny, 1))
        T0 = np.ascontiguousarray(T0, dtype=np.float64)
        qx = None if qx is None else np.ascontiguousarray(qx, dtype=np.float64)
        qy = None if qy is None else np.ascontiguousarray(qy, dtype=np.float64)
        lib().ora_init(ctypes.byref(self.c), _dptr(T0), _dptr(qx), _dptr(qy), _dptr(self.e))
        self.steps = 0

    def run(self, n: int) -> float:
        """Advance n steps; returns wall seconds spent in the stepper."""
        t = time.perf_counter()
        lib().ora_run(ctypes.byref(self.c), _dptr(self.e), _dptr(self.work), int(n))
        self.steps += int(n)
        return time.perf_counter() - t

    def set_wall_flux(self, wall: int, q0: float) -> None:
        """Heat flux into the domain at a heat-flux wall (Eq. 56) for the steps
        that follow; wall 0: x = 0, 1: x = nx-1, 2: y = 0, 3: y = ny-1."""
        self.c.q_wall[wall] = float(q0)

    def moments(self) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
        ny, nx = self.case.ny, self.case.nx
        T = np.empty((ny, nx)); qx = np.empty((ny, nx)); qy = np.empty((ny, nx))
        lib().ora_moments(ctypes.byref(self.c), _dptr(self.e), _dptr(T), _dptr(qx), _dptr(qy))
        return T, qx, qy

    def totals(self) -> np.ndarray:
        out = np.zeros(3)
        lib().ora_totals(ctypes.byref(self.c), _dptr(self.e), _dptr(out))
        return out

    def populations(self) -> np.ndarray:
        """State as (8, ny, nx), directions in the paper's order 1..8."""
        return self.e.reshape(8, self.case.ny, self.case.nx)


def collide_node(case, e_in: np.ndarray) -> np.ndarray:
    """Apply the single-node relaxation of Eq. 13 to 8 populations."""
    c = make_case(case)
    e_in = np.ascontiguousarray(e_in, dtype=np.float64)
    out = np.zeros(8)
    lib().ora_collide_node(ctypes.byref(c), _dptr(e_in), _dptr(out))
    return out


class Oracle3D:
    """One fully periodic D3Q14 lattice advanced by the C stepper in FP64.

    Fields are (nz, ny, nx) arrays, x fastest.  The populations are indexed
    0..5 for the axis movers +x -x +y -y +z -z and 6..13 for the corner movers
    (see ``phonon_oracle_d3q14.c``)."""

    def __init__(self, nx: int, ny: int, nz: int, tau_n: float, tau_r: float,
                 T0: Optional[np.ndarray] = None, q: Optional[Tuple] = None,
                 cv: float = 1.0, t0: float = 1.0):
        c = _Case3()
        c.nx, c.ny, c.nz = int(nx), int(ny), int(nz)
        c.tau_n, c.tau_r, c.cv, c.t0 = float(tau_n), float(tau_r), float(cv), float(t0)
        if lib().ora3_check(ctypes.byref(c)) != 0:
            raise ValueError(f"oracle rejects D3Q14 case {nx}x{ny}x{nz}, tau_n={tau_n}, tau_r={tau_r}")
        self.c, self.shape = c, (int(nz), int(ny), int(nx))
        n = 14 * nx * ny * nz
        self.e = np.zeros(n, dtype=np.float64)
        self.work = np.zeros(n, dtype=np.float64)
        if T0 is None:
            T0 = np.full(self.shape, float(t0))
        T0 = np.ascontiguousarray(np.broadcast_to(T0, self.shape), dtype=np.float64)
        qs = [None, None, None] if q is None else \
            [None if v is None else np.ascontiguousarray(np.broadcast_to(v, self.shape), dtype=np.float64)
             for v in q]
        lib().ora3_init(ctypes.byref(c), _dptr(T0), *[_dptr(v) for v in qs], _dptr(self.e))
        self.steps = 0

    def run(self, n: int) -> float:
        """Advance n steps; returns wall seconds spent in the stepper."""
        t = time.perf_counter()
        lib().ora3_run(ctypes.byref(self.c), _dptr(self.e), _dptr(self.work), int(n))
        self.steps += int(n)
        return time.perf_counter() - t

    def moments(self) -> Tuple[np.ndarray, np.ndarray, np.ndarray, np.ndarray]:
        out = [np.empty(self.shape) for _ in range(4)]
        lib().ora3_moments(ctypes.byref(self.c), _dptr(self.e), *[_dptr(v) for v in out])
        return tuple(out)

    def totals(self) -> np.ndarray:
        """[C_V sum (T - t0), sum q_x, sum q_y, sum q_z]."""
        out = np.zeros(4)
        lib().ora3_totals(ctypes.byref(self.c), _dptr(self.e), _dptr(out))
        return out

    def populations(self) -> np.ndarray:
        """State as (14, nz, ny, nx)."""
        return self.e.reshape((14,) + self.shape)


def collide_node_3d(tau_n: float, tau_r: float, e_in: np.ndarray, cv: float = 1.0) -> np.ndarray:
    """Apply the single-node D3Q14 relaxation (Eq. 13 with Eqs. 15-16) to 14 populations."""
    c = _Case3()
    c.nx = c.ny = c.nz = 1
    c.tau_n, c.tau_r, c.cv, c.t0 = float(tau_n), float(tau_r), float(cv), 0.0
    e_in = np.ascontiguousarray(e_in, dtype=np.float64)
    out = np.zeros(14)
    lib().ora3_collide_node(ctypes.byref(c), _dptr(e_in), _dptr(out))
    return out


def set_threads(n: int) -> None:
    lib().ora_set_threads(int(n))


def max_threads() -> int:
    return int(lib().ora_max_threads())
