"""ctypes binding of the D3Q14 C ABI in ``include/phonon_d3q14.h``.

Argument marshalling only: every step of the three-dimensional path runs in
the HIP kernels of ``libphonon_lbm.so`` (the same library as the D2Q8 path).
The functions carry the C names (``lbm3d_create``, ``lbm3d_init``,
``lbm3d_step``, ...); ``Box`` wraps one handle: it enqueues on torch's current
HIP stream and converts numpy or torch arrays to the pointers the ABI takes.
"""
from __future__ import annotations

import ctypes
import math
from typing import Optional, Sequence, Tuple

import numpy as np

from .lbm import (LAYOUT, LBM_BF16, LBM_F16, LBM_F32, LBM_FLAG_EXTERNAL_MEMORY, LBM_FLAG_ROUND_EVERY_STEP,
                  LBM_FLAG_STOCHASTIC_ROUNDING,
                  LBM_OK, LBMError, library as _library)


class lbm3d_config(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("storage", ctypes.c_int32), ("flags", ctypes.c_int32), ("layout", ctypes.c_int32),
                ("seed", ctypes.c_uint32),
                ("tau_n", ctypes.c_double), ("tau_r", ctypes.c_double), ("cv", ctypes.c_double),
                ("t0", ctypes.c_double), ("scale", ctypes.c_double), ("stream", ctypes.c_void_p)]


class lbm3d_launch_shape(ctypes.Structure):
    _fields_ = [("rows_per_tile", ctypes.c_int32), ("xcd_remap", ctypes.c_int32),
                ("nontemporal", ctypes.c_int32), ("tile_waves", ctypes.c_int32), ("zchunk", ctypes.c_int32)]


STORAGE3 = {"f32": LBM_F32, "f16": LBM_F16, "bf16": LBM_BF16}

_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
SIGNATURES3 = [
    ("lbm3d_last_error", ctypes.c_char_p, [_P]),
    ("lbm3d_required_bytes", ctypes.c_int, [ctypes.POINTER(lbm3d_config), ctypes.POINTER(ctypes.c_size_t)]),
    ("lbm3d_create", ctypes.c_int, [ctypes.POINTER(lbm3d_config), ctypes.POINTER(_P)]),
    ("lbm3d_bind", ctypes.c_int, [_P, _P, ctypes.c_size_t]),
    ("lbm3d_init", ctypes.c_int, [_P, _P, _P, _P, _P, ctypes.c_int32]),
    ("lbm3d_step", ctypes.c_int, [_P, ctypes.c_int64]),
    ("lbm3d_steps_done", ctypes.c_int64, [_P]),
    ("lbm3d_moments", ctypes.c_int, [_P, _P, _P, _P, _P, ctypes.c_int32]),
    ("lbm3d_sample", ctypes.c_int, [_P, _P, ctypes.c_int64, _P, ctypes.c_int32]),
    ("lbm3d_totals", ctypes.c_int, [_P, _D]),
    ("lbm3d_set_launch_shape", ctypes.c_int, [_P, ctypes.POINTER(lbm3d_launch_shape)]),
    ("lbm3d_get_launch_shape", ctypes.c_int, [_P, ctypes.POINTER(lbm3d_launch_shape)]),
    ("lbm3d_set_step_fusion", ctypes.c_int, [_P, ctypes.c_int32]),
    ("lbm3d_get_step_fusion", ctypes.c_int32, [_P]),
    ("lbm3d_autotune", ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_char_p, ctypes.c_size_t]),
    ("lbm3d_destroy", None, [_P]),
]

_bound = False


def library() -> ctypes.CDLL:
    """The HIP library with the D3Q14 entry points typed (raises if not built)."""
    global _bound
    L = _library()
    if not _bound:
        for name, res, args in SIGNATURES3:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _bound = True
    return L


def _check(rc: int, where: str, h=None) -> None:
    if rc != LBM_OK:
        raise LBMError(rc, where, library().lbm3d_last_error(h).decode(errors="replace"))


# --------------------------------------------------------------------- C names

def lbm3d_last_error(h) -> str:
    return library().lbm3d_last_error(h).decode(errors="replace")


def lbm3d_required_bytes(cfg: lbm3d_config) -> int:
    n = ctypes.c_size_t(0)
    _check(library().lbm3d_required_bytes(ctypes.byref(cfg), ctypes.byref(n)), "lbm3d_required_bytes")
    return int(n.value)


def lbm3d_create(cfg: lbm3d_config):
    h = ctypes.c_void_p()
    _check(library().lbm3d_create(ctypes.byref(cfg), ctypes.byref(h)), "lbm3d_create")
    return h


def lbm3d_bind(h, ptr: int, nbytes: int) -> None:
    _check(library().lbm3d_bind(h, ctypes.c_void_p(ptr), nbytes), "lbm3d_bind", h)


def lbm3d_init(h, T_ptr, qx_ptr, qy_ptr, qz_ptr, on_device: int) -> None:
    _check(library().lbm3d_init(h, T_ptr, qx_ptr, qy_ptr, qz_ptr, on_device), "lbm3d_init", h)


def lbm3d_step(h, nsteps: int) -> None:
    _check(library().lbm3d_step(h, int(nsteps)), "lbm3d_step", h)


def lbm3d_steps_done(h) -> int:
    return int(library().lbm3d_steps_done(h))


def lbm3d_moments(h, dT_ptr, qx_ptr, qy_ptr, qz_ptr, on_device: int) -> None:
    _check(library().lbm3d_moments(h, dT_ptr, qx_ptr, qy_ptr, qz_ptr, on_device), "lbm3d_moments", h)


def lbm3d_sample(h, nodes_ptr, count: int, out_ptr, on_device: int) -> None:
    _check(library().lbm3d_sample(h, nodes_ptr, int(count), out_ptr, on_device), "lbm3d_sample", h)


def lbm3d_totals(h) -> np.ndarray:
    out = np.zeros(4)
    _check(library().lbm3d_totals(h, out.ctypes.data_as(_D)), "lbm3d_totals", h)
    return out


def lbm3d_set_launch_shape(h, shape: lbm3d_launch_shape) -> None:
    _check(library().lbm3d_set_launch_shape(h, ctypes.byref(shape)), "lbm3d_set_launch_shape", h)


def lbm3d_set_step_fusion(h, steps: int) -> None:
    _check(library().lbm3d_set_step_fusion(h, int(steps)), "lbm3d_set_step_fusion", h)


def lbm3d_get_step_fusion(h) -> int:
    return int(library().lbm3d_get_step_fusion(h))


def lbm3d_get_launch_shape(h) -> lbm3d_launch_shape:
    s = lbm3d_launch_shape()
    _check(library().lbm3d_get_launch_shape(h, ctypes.byref(s)), "lbm3d_get_launch_shape", h)
    return s


def lbm3d_autotune(h, steps: int = 20) -> str:
    buf = ctypes.create_string_buffer(4096)
    _check(library().lbm3d_autotune(h, int(steps), buf, len(buf)), "lbm3d_autotune", h)
    return buf.value.decode()


def lbm3d_destroy(h) -> None:
    library().lbm3d_destroy(h)


# --------------------------------------------------------------------- wrapper

def _host_ptr(a: Optional[np.ndarray]):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


class Box:
    """One periodic D3Q14 box on the current HIP device.

    Fields are (nz, ny, nx) arrays, x fastest.  Device memory comes from torch
    (bound with ``lbm3d_bind``) and work is enqueued on torch's current stream."""

    def __init__(self, nx: int, ny: int, nz: int, tau_n: float, tau_r: float, storage: str = "f32",
                 t0: float = 1.0, cv: float = 1.0, scale: float = 0.0, stochastic: bool = False,
                 seed: int = 0, layout: str = "auto", every_step: bool = False):
        import torch
        self.torch = torch
        self.shape = (int(nz), int(ny), int(nx))
        cfg = lbm3d_config()
        cfg.nx, cfg.ny, cfg.nz = int(nx), int(ny), int(nz)
        cfg.storage = STORAGE3[storage]
        cfg.flags = (LBM_FLAG_EXTERNAL_MEMORY | (LBM_FLAG_STOCHASTIC_ROUNDING if stochastic else 0)
                     | (LBM_FLAG_ROUND_EVERY_STEP if every_step else 0))
        cfg.layout = LAYOUT[layout]
        cfg.seed = int(seed) & 0xffffffff
        cfg.tau_n, cfg.tau_r, cfg.cv, cfg.t0, cfg.scale = float(tau_n), float(tau_r), float(cv), float(t0), float(scale)
        cfg.stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        self.cfg = cfg
        nbytes = lbm3d_required_bytes(cfg)
        self.mem = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        ptr = self.mem.data_ptr()
        ptr += (-ptr) % 256
        self.h = lbm3d_create(cfg)
        lbm3d_bind(self.h, ptr, nbytes)

    @property
    def nodes(self) -> int:
        return self.shape[0] * self.shape[1] * self.shape[2]

    def init(self, T=None, q: Optional[Sequence] = None) -> None:
        """T and the flux components as numpy (host) or torch CUDA (device) FP64
        arrays of the box shape; None for t0 / zero."""
        q = list(q) if q is not None else [None, None, None]
        arrs = [T] + q
        torch = self.torch
        if any(isinstance(a, torch.Tensor) for a in arrs if a is not None):
            keep = [None if a is None else a.to(dtype=torch.float64).contiguous() for a in arrs]
            ptrs = [None if a is None else ctypes.c_void_p(a.data_ptr()) for a in keep]
            lbm3d_init(self.h, *ptrs, 1)
        else:
            keep = [None if a is None else np.ascontiguousarray(np.broadcast_to(a, self.shape), dtype=np.float64)
                    for a in arrs]
            lbm3d_init(self.h, *[_host_ptr(a) for a in keep], 0)

    def step(self, n: int) -> None:
        lbm3d_step(self.h, n)

    @property
    def steps_done(self) -> int:
        return lbm3d_steps_done(self.h)

    def moments(self) -> Tuple[np.ndarray, np.ndarray, np.ndarray, np.ndarray]:
        """(dT, qx, qy, qz) on the host, FP64."""
        out = [np.empty(self.shape) for _ in range(4)]
        lbm3d_moments(self.h, *[_host_ptr(a) for a in out], 0)
        return tuple(out)

    def moments_device(self):
        """(dT, qx, qy, qz) as torch CUDA FP64 tensors."""
        torch = self.torch
        out = [torch.empty(self.shape, dtype=torch.float64, device="cuda") for _ in range(4)]
        lbm3d_moments(self.h, *[ctypes.c_void_p(a.data_ptr()) for a in out], 1)
        return tuple(out)

    def sample(self, x, y, z) -> np.ndarray:
        """(count, 4) array of (dT, qx, qy, qz) at nodes (x, y, z)."""
        nz, ny, nx = self.shape
        idx = ((np.asarray(z, np.int64) * ny + np.asarray(y, np.int64)) * nx + np.asarray(x, np.int64)).ravel()
        idx = np.ascontiguousarray(idx)
        out = np.empty((idx.size, 4))
        lbm3d_sample(self.h, _host_ptr(idx), idx.size, _host_ptr(out), 0)
        return out

    def totals(self) -> np.ndarray:
        return lbm3d_totals(self.h)

    def set_launch_shape(self, rows_per_tile: int = 4, xcd_remap: int = 0, nontemporal: int = 0,
                         tile_waves: int = 1, zchunk: int = 32) -> None:
        lbm3d_set_launch_shape(self.h, lbm3d_launch_shape(rows_per_tile, xcd_remap, nontemporal, tile_waves,
                                                          zchunk))

    def launch_shape(self) -> dict:
        s = lbm3d_get_launch_shape(self.h)
        return {"rows_per_tile": s.rows_per_tile, "xcd_remap": s.xcd_remap, "nontemporal": s.nontemporal,
                "tile_waves": s.tile_waves, "zchunk": s.zchunk}

    def set_step_fusion(self, steps: int) -> None:
        lbm3d_set_step_fusion(self.h, steps)

    def step_fusion(self) -> int:
        return lbm3d_get_step_fusion(self.h)

    def autotune(self, steps: int = 20) -> dict:
        """Pick the fastest launch shape (before init); returns the timing report."""
        import json
        return json.loads(lbm3d_autotune(self.h, steps))

    def close(self) -> None:
        if getattr(self, "h", None) is not None:
            lbm3d_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
