"""Helpers shared by the GPU parity tests: run a case on the HIP path and on
the FP64 oracle from the same seeded inputs, and the error metrics.

Error metrics (relative L2 over all nodes at the compared step):
  eps_T = ||T - T_or|| / ||T_or - t0||        (deviation from the base temperature)
  eps_q = ||q - q_or|| / ||q_or||             (both components)
"""
from __future__ import annotations

import numpy as np

import workloads as W
from oracle import ref
from paper_2010_01847_amd import Lattice, instance_from_case


def oracle_fields(case, steps, T0=None, qx=None, qy=None):
    """(dT, qx, qy) of the oracle after `steps`, dT = T - T_ref."""
    o = ref.Oracle(case, T0, qx, qy)
    o.run(steps)
    T, qxo, qyo = o.moments()
    return T - np.tile(case.t_ref(), (case.ny, 1)), qxo, qyo


def gpu_fields(case, steps, T0=None, qx=None, qy=None, storage="f32", scale=0.0, check=0,
               shape=None, schedule=None, layout="auto", rounding="nearest", seed=0):
    lat = Lattice([instance_from_case(case, scale)], storage=storage, check_interval=check, layout=layout,
                  rounding=rounding, seed=seed)
    if shape:
        lat.set_launch_shape(**shape)
    if schedule:
        lat.set_schedule(schedule)
    lat.init(0, T0, qx, qy)
    lat.step(steps)
    out = lat.moments(0)
    lat.close()
    return out


def eps(case, gpu, ora):
    dT, qx, qy = gpu
    dTo, qxo, qyo = ora
    base = np.tile(case.t_ref(), (case.ny, 1)) - case.t0     # ramp part of T_or - t0
    den_t = np.sqrt(np.sum((dTo + base) ** 2))
    e_t = np.sqrt(np.sum((dT - dTo) ** 2)) / den_t if den_t > 0 else 0.0
    den_q = np.sqrt(np.sum(qxo ** 2 + qyo ** 2))
    e_q = np.sqrt(np.sum((qx - qxo) ** 2 + (qy - qyo) ** 2)) / den_q if den_q > 0 else 0.0
    return float(e_t), float(e_q)


def log(msg: str) -> None:
    print(msg, flush=True)
