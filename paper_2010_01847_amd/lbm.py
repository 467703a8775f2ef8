"""ctypes binding of the C ABI in ``include/phonon_lbm.h``.

Argument marshalling only: every step of the lattice Boltzmann path runs in
the HIP kernels of ``libphonon_lbm.so``.  Importing this module fails loudly
when the library has not been built; there is no fallback.

The functions carry the C names (``lbm_create``, ``lbm_init``, ``lbm_step``,
``lbm_moments``, ``lbm_residual``, ...).  ``Lattice`` wraps one handle for
convenience: it allocates the device memory as a torch tensor (bound with
``lbm_bind``), enqueues on torch's current HIP stream, and converts numpy or
torch arrays to the pointers the ABI takes.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Iterable, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libphonon_lbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EHIP, LBM_ESTATE, LBM_EUNSUPPORTED, LBM_ENONFINITE = 0, -1, -2, -3, -4, -5, -6
LBM_F32, LBM_F16, LBM_BF16, LBM_F16_SPLIT, LBM_BF16_SPLIT = 0, 1, 2, 3, 4
LBM_BC_PERIODIC, LBM_BC_ISOTHERMAL, LBM_BC_DIFFUSE, LBM_BC_GRADIENT, LBM_BC_HEATFLUX = 0, 1, 2, 3, 4
LBM_SCHED_BATCHED, LBM_SCHED_PER_INSTANCE, LBM_SCHED_GRAPH = 0, 1, 2
LBM_FLAG_EXTERNAL_MEMORY = 0x1
LBM_FLAG_STOCHASTIC_ROUNDING = 0x2
LBM_FLAG_ROUND_EVERY_STEP = 0x4
LBM_LAYOUT_AUTO, LBM_LAYOUT_PLANES, LBM_LAYOUT_CHUNKED = 0, 1, 2
LAYOUT = {"auto": LBM_LAYOUT_AUTO, "planes": LBM_LAYOUT_PLANES, "chunked": LBM_LAYOUT_CHUNKED}

STORAGE = {"f32": LBM_F32, "f16": LBM_F16, "bf16": LBM_BF16,
           "f16_split": LBM_F16_SPLIT, "bf16_split": LBM_BF16_SPLIT}
BC = {"periodic": LBM_BC_PERIODIC, "isothermal": LBM_BC_ISOTHERMAL, "diffuse": LBM_BC_DIFFUSE,
      "gradient": LBM_BC_GRADIENT, "heatflux": LBM_BC_HEATFLUX}
ERRNAMES = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_ENOMEM", -3: "LBM_EHIP", -4: "LBM_ESTATE",
            -5: "LBM_EUNSUPPORTED", -6: "LBM_ENONFINITE"}


class lbm_instance(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32),
                ("tau_n", ctypes.c_double), ("tau_r", ctypes.c_double),
                ("cv", ctypes.c_double), ("t0", ctypes.c_double), ("grad_x", ctypes.c_double),
                ("t_wall", ctypes.c_double * 4), ("scale", ctypes.c_double),
                ("wall_bc", ctypes.c_int32 * 4)]


class lbm_config(ctypes.Structure):
    _fields_ = [("n_instances", ctypes.c_int32), ("storage", ctypes.c_int32),
                ("check_interval", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("inst", ctypes.POINTER(lbm_instance)), ("stream", ctypes.c_void_p),
                ("layout", ctypes.c_int32), ("seed", ctypes.c_uint32)]


class lbm_check_info(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("residual", ctypes.c_double),
                ("totals", ctypes.c_double * 3)]


class lbm_launch_shape(ctypes.Structure):
    _fields_ = [("vec", ctypes.c_int32), ("block_x", ctypes.c_int32), ("block_y", ctypes.c_int32),
                ("xcd_remap", ctypes.c_int32), ("nontemporal", ctypes.c_int32)]


# (name, restype, argtypes) of every entry point declared in the header
_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_F = ctypes.POINTER(ctypes.c_float)
SIGNATURES = [
    ("lbm_version", ctypes.c_char_p, []),
    ("lbm_last_error", ctypes.c_char_p, [_P]),
    ("lbm_required_bytes", ctypes.c_int, [ctypes.POINTER(lbm_config), ctypes.POINTER(ctypes.c_size_t)]),
    ("lbm_create", ctypes.c_int, [ctypes.POINTER(lbm_config), ctypes.POINTER(_P)]),
    ("lbm_bind", ctypes.c_int, [_P, _P, ctypes.c_size_t]),
    ("lbm_init", ctypes.c_int, [_P, ctypes.c_int32, _D, _D, _D]),
    ("lbm_init_device", ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P]),
    ("lbm_step", ctypes.c_int, [_P, ctypes.c_int64]),
    ("lbm_steps_done", ctypes.c_int64, [_P]),
    ("lbm_moments", ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P, ctypes.c_int32]),
    ("lbm_moments_f64", ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P, ctypes.c_int32]),
    ("lbm_moments_f64_noalloc", ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P]),
    ("lbm_totals", ctypes.c_int, [_P, ctypes.c_int32, _D]),
    ("lbm_residual", ctypes.c_int, [_P, ctypes.c_int32, _D]),
    ("lbm_last_check", ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(lbm_check_info)]),
    ("lbm_coefficients", ctypes.c_int, [_P, ctypes.c_int32, _D]),
    ("lbm_set_wall_flux", ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_double]),
    ("lbm_set_step_fusion", ctypes.c_int, [_P, ctypes.c_int32]),
    ("lbm_get_step_fusion", ctypes.c_int32, [_P]),
    ("lbm_max_step_fusion", ctypes.c_int32, [ctypes.c_int32]),
    ("lbm_set_schedule", ctypes.c_int, [_P, ctypes.c_int32]),
    ("lbm_set_streams", ctypes.c_int, [_P, ctypes.c_int32]),
    ("lbm_get_streams", ctypes.c_int32, [_P]),
    ("lbm_set_launch_shape", ctypes.c_int, [_P, ctypes.POINTER(lbm_launch_shape)]),
    ("lbm_get_launch_shape", ctypes.c_int, [_P, ctypes.POINTER(lbm_launch_shape)]),
    ("lbm_autotune", ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_char_p, ctypes.c_size_t]),
    ("lbm_destroy", None, [_P]),
]

_lib = None


def library() -> ctypes.CDLL:
    """Load ``libphonon_lbm.so`` (raises if it is not built).

    torch is imported first: its wheel carries its own HIP runtime under the
    same soname as the system one the library links, and only a process that
    has loaded torch's before the library's dependency is resolved ends up
    with one HIP runtime (loaded the other way round, torch brings in a second
    copy, which claims the GPU, and the library's own calls find no device)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                               "(build it with python -m paper_2010_01847_amd.build)")
        import torch  # noqa: F401  (see above)
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class LBMError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: {ERRNAMES.get(code, code)}: {msg}")
        self.code = code


def _check(rc: int, where: str, h=None) -> int:
    if rc != LBM_OK:
        msg = library().lbm_last_error(h).decode(errors="replace")
        raise LBMError(rc, where, msg)
    return rc


# --------------------------------------------------------------------- C names

def lbm_version() -> str:
    return library().lbm_version().decode()


def lbm_last_error(h) -> str:
    return library().lbm_last_error(h).decode(errors="replace")


def lbm_required_bytes(cfg: lbm_config) -> int:
    n = ctypes.c_size_t(0)
    _check(library().lbm_required_bytes(ctypes.byref(cfg), ctypes.byref(n)), "lbm_required_bytes")
    return int(n.value)


def lbm_create(cfg: lbm_config):
    h = ctypes.c_void_p()
    _check(library().lbm_create(ctypes.byref(cfg), ctypes.byref(h)), "lbm_create")
    return h


def lbm_bind(h, ptr: int, nbytes: int) -> None:
    _check(library().lbm_bind(h, ctypes.c_void_p(ptr), nbytes), "lbm_bind", h)


def _dptr(a):
    if a is None:
        return ctypes.POINTER(ctypes.c_double)()
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def lbm_init(h, inst: int, T=None, qx=None, qy=None) -> None:
    """Host FP64 fields (C-contiguous numpy (ny, nx)) or None."""
    arrs = [None if a is None else np.ascontiguousarray(a, dtype=np.float64) for a in (T, qx, qy)]
    _check(library().lbm_init(h, inst, *[_dptr(a) for a in arrs]), "lbm_init", h)


def lbm_init_device(h, inst: int, T_ptr: int, qx_ptr: int = 0, qy_ptr: int = 0) -> None:
    _check(library().lbm_init_device(h, inst, ctypes.c_void_p(T_ptr), ctypes.c_void_p(qx_ptr or None),
                                     ctypes.c_void_p(qy_ptr or None)), "lbm_init_device", h)


def lbm_step(h, nsteps: int) -> None:
    _check(library().lbm_step(h, int(nsteps)), "lbm_step", h)


def lbm_steps_done(h) -> int:
    return int(library().lbm_steps_done(h))


def lbm_moments(h, inst: int, T_ptr, qx_ptr, qy_ptr, on_device: int) -> None:
    _check(library().lbm_moments(h, inst, T_ptr, qx_ptr, qy_ptr, on_device), "lbm_moments", h)


def lbm_moments_f64(h, inst: int, dT_ptr, qx_ptr, qy_ptr, on_device: int) -> None:
    _check(library().lbm_moments_f64(h, inst, dT_ptr, qx_ptr, qy_ptr, on_device), "lbm_moments_f64", h)


def lbm_moments_f64_noalloc(h, inst: int, dT_ptr, qx_ptr, qy_ptr) -> None:
    _check(library().lbm_moments_f64_noalloc(h, inst, dT_ptr, qx_ptr, qy_ptr), "lbm_moments_f64_noalloc", h)


def lbm_totals(h, inst: int) -> np.ndarray:
    out = np.zeros(3)
    _check(library().lbm_totals(h, inst, _dptr(out)), "lbm_totals", h)
    return out


def lbm_residual(h, inst: int) -> float:
    r = ctypes.c_double(0.0)
    _check(library().lbm_residual(h, inst, ctypes.byref(r)), "lbm_residual", h)
    return float(r.value)


def lbm_last_check(h, inst: int) -> dict:
    ci = lbm_check_info()
    _check(library().lbm_last_check(h, inst, ctypes.byref(ci)), "lbm_last_check", h)
    return dict(step=int(ci.step), residual=float(ci.residual), totals=[float(v) for v in ci.totals])


def lbm_coefficients(h, inst: int) -> dict:
    out = np.zeros(6)
    _check(library().lbm_coefficients(h, inst, _dptr(out)), "lbm_coefficients", h)
    return dict(inv_tau=out[0], beta=out[1], one_minus_rho=out[2], scale=out[3], tau=out[4], rho=out[5])


def lbm_set_wall_flux(h, inst: int, wall: int, q0: float) -> None:
    _check(library().lbm_set_wall_flux(h, int(inst), int(wall), float(q0)), "lbm_set_wall_flux", h)


def lbm_set_step_fusion(h, steps: int) -> None:
    _check(library().lbm_set_step_fusion(h, int(steps)), "lbm_set_step_fusion", h)


def lbm_get_step_fusion(h) -> int:
    return int(library().lbm_get_step_fusion(h))


def lbm_max_step_fusion(storage: int) -> int:
    return int(library().lbm_max_step_fusion(int(storage)))


def lbm_set_schedule(h, schedule: int) -> None:
    _check(library().lbm_set_schedule(h, int(schedule)), "lbm_set_schedule", h)


def lbm_set_streams(h, n: int) -> None:
    _check(library().lbm_set_streams(h, int(n)), "lbm_set_streams", h)


def lbm_get_streams(h) -> int:
    return int(library().lbm_get_streams(h))


def lbm_set_launch_shape(h, vec: int, block_x: int, block_y: int = 1, xcd_remap: int = 1,
                         nontemporal: int = 0) -> None:
    s = lbm_launch_shape(vec, block_x, block_y, xcd_remap, nontemporal)
    _check(library().lbm_set_launch_shape(h, ctypes.byref(s)), "lbm_set_launch_shape", h)


def lbm_get_launch_shape(h) -> dict:
    s = lbm_launch_shape()
    _check(library().lbm_get_launch_shape(h, ctypes.byref(s)), "lbm_get_launch_shape", h)
    return dict(vec=s.vec, block_x=s.block_x, block_y=s.block_y, xcd_remap=s.xcd_remap,
                nontemporal=s.nontemporal)


def lbm_autotune(h, steps: int = 0) -> str:
    buf = ctypes.create_string_buffer(16384)
    _check(library().lbm_autotune(h, int(steps), buf, len(buf)), "lbm_autotune", h)
    return buf.value.decode()


def lbm_destroy(h) -> None:
    library().lbm_destroy(h)


# --------------------------------------------------------------------- helper

def make_instance(nx: int, ny: int, tau_n: float, tau_r: float, bc_x="periodic", bc_y="periodic",
                  cv: float = 1.0, t0: float = 1.0, grad_x: float = 0.0,
                  t_wall: Sequence[float] = (0.0, 0.0, 0.0, 0.0), scale: float = 0.0,
                  wall_bc: Sequence = (0, 0, 0, 0)) -> lbm_instance:
    it = lbm_instance()
    it.nx, it.ny = int(nx), int(ny)
    it.bc_x = BC[bc_x] if isinstance(bc_x, str) else int(bc_x)
    it.bc_y = BC[bc_y] if isinstance(bc_y, str) else int(bc_y)
    it.tau_n, it.tau_r = float(tau_n), float(tau_r)
    it.cv, it.t0, it.grad_x = float(cv), float(t0), float(grad_x)
    for k in range(4):
        it.t_wall[k] = float(t_wall[k])
    it.scale = float(scale)
    for k in range(4):
        v = wall_bc[k]
        it.wall_bc[k] = BC[v] if isinstance(v, str) else int(v)
    return it


def instance_from_case(case, scale: float = 0.0) -> lbm_instance:
    """From any object with the fields of ``workloads.Case``."""
    return make_instance(case.nx, case.ny, case.tau_n, case.tau_r, case.bc_x, case.bc_y,
                         getattr(case, "cv", 1.0), case.t0, getattr(case, "grad_x", 0.0),
                         getattr(case, "t_wall", (0.0,) * 4), scale, getattr(case, "wall_bc", (0,) * 4))


class Lattice:
    """One handle over one or more instances, memory from torch, stream from torch."""

    def __init__(self, instances: Iterable[lbm_instance], storage="f32", check_interval: int = 0,
                 device=None, stream=None, layout="auto", rounding="nearest", seed: int = 0,
                 every_step: bool = False):
        import torch
        self._torch = torch
        self.instances: List[lbm_instance] = list(instances)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        arr = (lbm_instance * len(self.instances))(*self.instances)
        self._arr = arr
        cfg = lbm_config()
        cfg.n_instances = len(self.instances)
        cfg.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
        cfg.check_interval = int(check_interval)
        if rounding not in ("nearest", "stochastic"):
            raise ValueError("rounding must be 'nearest' or 'stochastic'")
        cfg.flags = (LBM_FLAG_EXTERNAL_MEMORY | (LBM_FLAG_STOCHASTIC_ROUNDING if rounding == "stochastic" else 0)
                     | (LBM_FLAG_ROUND_EVERY_STEP if every_step else 0))
        cfg.seed = int(seed) & 0xffffffff
        cfg.inst = ctypes.cast(arr, ctypes.POINTER(lbm_instance))
        cfg.stream = ctypes.c_void_p(self.stream.cuda_stream)
        cfg.layout = LAYOUT[layout] if isinstance(layout, str) else int(layout)
        self.cfg = cfg
        self.nbytes = lbm_required_bytes(cfg)
        with torch.cuda.device(self.device):
            self.h = lbm_create(cfg)
            # torch's allocator hands out 512-byte aligned blocks
            self.mem = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
        lbm_bind(self.h, self.mem.data_ptr(), self.nbytes)

    # -- lifecycle
    def close(self) -> None:
        if getattr(self, "h", None):
            lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- wrappers
    def init(self, inst: int, T=None, qx=None, qy=None) -> None:
        torch = self._torch
        if T is not None and isinstance(T, torch.Tensor):
            args = [None if a is None else a.to(device=self.device, dtype=torch.float64).contiguous()
                    for a in (T, qx, qy)]
            lbm_init_device(self.h, inst, args[0].data_ptr(), args[1].data_ptr() if args[1] is not None else 0,
                            args[2].data_ptr() if args[2] is not None else 0)
            return
        lbm_init(self.h, inst, T, qx, qy)

    def step(self, n: int) -> None:
        lbm_step(self.h, n)

    @property
    def steps(self) -> int:
        return lbm_steps_done(self.h)

    def moments(self, inst: int = 0) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
        """FP64 (dT, qx, qy) on the host; dT = T - T_ref."""
        it = self.instances[inst]
        out = [np.empty((it.ny, it.nx), dtype=np.float64) for _ in range(3)]
        lbm_moments_f64(self.h, inst, *[o.ctypes.data for o in out], 0)
        return out[0], out[1], out[2]

    def moments_noalloc(self, inst: int = 0) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
        """As moments(), through lbm_moments_f64_noalloc (no device allocation;
        instances of at most 2^20 nodes)."""
        it = self.instances[inst]
        out = [np.empty((it.ny, it.nx), dtype=np.float64) for _ in range(3)]
        lbm_moments_f64_noalloc(self.h, inst, *[o.ctypes.data for o in out])
        return out[0], out[1], out[2]

    def moments_f32(self, inst: int = 0):
        """FP32 absolute (T, qx, qy) on the host (lbm_moments)."""
        it = self.instances[inst]
        out = [np.empty((it.ny, it.nx), dtype=np.float32) for _ in range(3)]
        lbm_moments(self.h, inst, *[o.ctypes.data for o in out], 0)
        return out[0], out[1], out[2]

    def moments_device(self, inst: int = 0, rows: Optional[slice] = None):
        """FP64 (dT, qx, qy) as device tensors (lbm_moments_f64 with on_device)."""
        torch = self._torch
        it = self.instances[inst]
        out = [torch.empty((it.ny, it.nx), dtype=torch.float64, device=self.device) for _ in range(3)]
        lbm_moments_f64(self.h, inst, *[o.data_ptr() for o in out], 1)
        return out

    def totals(self, inst: int = 0) -> np.ndarray:
        return lbm_totals(self.h, inst)

    def residual(self, inst: int = 0) -> float:
        return lbm_residual(self.h, inst)

    def last_check(self, inst: int = 0) -> dict:
        return lbm_last_check(self.h, inst)

    def coefficients(self, inst: int = 0) -> dict:
        return lbm_coefficients(self.h, inst)

    def set_wall_flux(self, inst: int, wall: int, q0: float) -> None:
        """Heat flux into the domain through a HEATFLUX wall (0: x=0, 1: x=nx-1,
        2: y=0, 3: y=ny-1) for the steps enqueued afterwards."""
        lbm_set_wall_flux(self.h, inst, wall, float(q0))

    def set_step_fusion(self, steps: int) -> None:
        """Most time steps per launch where allowed (1: every step on its own)."""
        lbm_set_step_fusion(self.h, steps)

    def step_fusion(self) -> int:
        """Most time steps per launch (on a new handle: the most the storage
        kind's fused kernel takes for large lattices, 1 for small ones)."""
        return lbm_get_step_fusion(self.h)

    def set_schedule(self, name: str) -> None:
        lbm_set_schedule(self.h, {"batched": LBM_SCHED_BATCHED, "per_instance": LBM_SCHED_PER_INSTANCE,
                                  "graph": LBM_SCHED_GRAPH}[name])

    def set_streams(self, n: int) -> None:
        lbm_set_streams(self.h, n)

    def streams(self) -> int:
        return lbm_get_streams(self.h)

    def set_launch_shape(self, **kw) -> None:
        lbm_set_launch_shape(self.h, **kw)

    def launch_shape(self) -> dict:
        return lbm_get_launch_shape(self.h)

    def autotune(self, steps: int = 0) -> str:
        return lbm_autotune(self.h, steps)
