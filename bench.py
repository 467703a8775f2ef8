"""Throughput and accuracy of the fused D2Q8 phonon stream-collide step on one
MI355X.

Default workload (the headline line): the second-sound configuration --
8192 x 8192 periodic lattice, Gaussian pulse dT = 0.01 exp(-r^2 / (2 * 20^2))
on T0 = 1 at the centre, tau_N = 0.55, tau_R = 50 -- with FP32 storage of the
scaled deviations, FP32 arithmetic, and FP64 check-step reductions every 100
steps.  A step is one pass of the whole hot path over the lattice:
pull-advection, boundary handling, moments in registers, relaxation with the
resistive source, store, and (on check steps) the FP64 residual and total
reductions.  `value` is MLUPS (million lattice-node updates per second) of the
timed steps, with the populations resident in HBM before the timed region.

Prints one JSON line.  Beside the headline it reports, each with its error
against the FP64 oracle (relative L2 of the temperature deviation and of the
heat flux, pass or fail against 1e-5 for FP32 storage and 5e-3 for 16-bit
storage, computed after the timed region):

* "rows": the same workload in every storage kind (FP16 with stochastic
  rounding and to nearest, BF16 with stochastic rounding, the split FP16 /
  BF16 forms), each run on to the
  workload's 4000 steps and compared on sampled rows with the exact periodic
  solution; "front": the pulse-front speed;
* "walls" (128 x 64 isothermal walls, 5000 steps) and "channel" (1024 x 256
  gradient channel run to steady state): small, cache-resident lattices,
  MLUPS only;
* "sweep": 256 uneven channel instances under the batched (two streams and
  one), graph and one-launch-per-instance schedules;
* "large": the 16384^2 smooth-modes lattice in 16-bit storage, with the FP64
  totals' drift;
* "d3q14": the three-dimensional lattice on a 512^3 periodic box.

Roofline of the dominant kernel (the marching kernel, several time steps per
launch): `achieved` = the HBM bytes the counters measured per launch
(`traffic`, from the committed rocprofv3 summary while its kernel sources
match) over the launch's live duration, against the 8 TB/s peak (the
compulsory bytes, the state read once and written once, stand in while the
summary is stale, and `achieved_bytes` says which); `compulsory` = those bytes
over the same duration; `single_step_equivalent` = the bytes the same updates
would move as single steps (64 B per update in FP32), over the same duration
-- above the peak, since the launch reuses its data on chip; `alu` = the same
launch against the non-packed vector FP32 peak (the kernels are built without
packed FP32); `limiter` names what bounds the launch.

Only the oracle leg (`_oracle_leg`: the host timing of the oracle and every
error evaluation) imports the oracle; the GPU legs collect the HIP path's
fields through the C ABI and hand them over as arrays.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, 8 TB/s
# MI355X vector FP32 without packed instructions: 256 CUs x 4 SIMDs x 16 lanes
# x 2 (fused multiply-add) x 2.4 GHz = 78.6 TFLOP/s (the packed form doubles it;
# the kernels are compiled without packed FP32)
FP32_VECTOR_PEAK_TFLOPS = 78.6
# FP32 operations of one D2Q8 relaxation (moments, equilibrium shares, the
# eight updates; a fused multiply-add counts 2)
FLOP_PER_UPDATE = 81
# 8 population reads + 8 writes per node and step; split storage adds the FP32 energy
BYTES_PER_NODE = {"f32": 64, "f16": 32, "bf16": 32, "f16_split": 40, "bf16_split": 40}
# D3Q14: 14 population reads + 14 writes per node
BYTES_PER_NODE_3D = {"f32": 112, "f16": 56, "bf16": 56}
# error bounds against the FP64 oracle
BOUND = {"f32": 1e-5, "f16": 5e-3, "bf16": 5e-3, "f16_split": 5e-3, "bf16_split": 5e-3}
_CSRC = os.path.join(ROOT, "paper_2010_01847_amd", "csrc")
# the device code and the headers that fix its tiles, descriptors and rounding
KERNEL_SOURCES = [os.path.join(_CSRC, f) for f in ("lbm_device.hip", "lbm_internal.h", "lbm_numeric.h")]
KERNEL_SOURCES_3D = [os.path.join(_CSRC, f) for f in ("d3q14_device.hip", "d3q14_internal.h", "lbm_numeric.h")]
PROFILES = os.path.join(ROOT, "profiles")


def _traffic_from(path: str, sources):
    """HBM bytes per launch from a committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE scaled by a plain copy of known size), or None
    when there is none or the kernel sources changed since the counters were
    taken (SHA-256 of the sources recorded in the summary)."""
    import hashlib
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(("|", "#")):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    sha = hashlib.sha256(b"".join(open(f, "rb").read() for f in sources)).hexdigest()
    if fields.get("kernel_source_sha256") != sha or "traffic_bytes_per_launch" not in fields:
        return None
    return int(float(fields["traffic_bytes_per_launch"]))


def _parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=1000)
    p.add_argument("--warmup", type=int, default=50)
    p.add_argument("--n", type=int, default=8192, help="lattice side")
    p.add_argument("--storage", default="f32", choices=list(BYTES_PER_NODE))
    p.add_argument("--rows", default="f16:stochastic,f16:nearest,bf16:stochastic,f16_split,bf16_split",
                   help="extra rows, storage[:rounding] ('' for none)")
    p.add_argument("--rounding", default=None, choices=["nearest", "stochastic"],
                   help="rounding of the main row's stores (default: stochastic for plain 16-bit "
                        "storage, which stalls on smooth fields when every step is rounded to "
                        "nearest; nearest for the rest)")
    p.add_argument("--accuracy-steps", type=int, default=4000,
                   help="steps after which each second-sound row is compared with the exact solution")
    p.add_argument("--sweep-steps", type=int, default=300, help="timed steps per sweep schedule (0: skip)")
    p.add_argument("--small", type=int, default=1, help="walls and channel rows (0: skip)")
    p.add_argument("--front", type=int, default=1, help="pulse-front speed run (0: skip)")
    p.add_argument("--fusion", default="auto",
                   help="most time steps per launch (auto: the library's default for the storage kind)")
    p.add_argument("--check-interval", type=int, default=100)
    p.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle leg (timing and errors)")
    p.add_argument("--cpu-seconds", type=float, default=12.0)
    p.add_argument("--autotune", action="store_true")
    p.add_argument("--d3q14-steps", type=int, default=200, help="timed steps of the D3Q14 box (0: skip)")
    p.add_argument("--d3q14-n", type=int, default=512, help="side of the periodic D3Q14 box")
    p.add_argument("--d3q14-rows", default="f32,bf16:stochastic,f16:stochastic",
                   help="storage[:rounding] rows of the D3Q14 box")
    p.add_argument("--d3q14-shape", default="auto",
                   help="D3Q14 launch shape rows_per_tile,xcd_remap,nontemporal,tile_waves[,zchunk[,steps "
                        "per launch]] (auto: the autotuner's choice)")
    p.add_argument("--large-steps", type=int, default=200,
                   help="timed steps of each row of the 16384^2 smooth-modes lattice (0: skip)")
    p.add_argument("--large-rows", default="f16_split,bf16_split,f16:stochastic",
                   help="storage[:rounding] rows of the 16384^2 smooth-modes lattice")
    p.add_argument("--copy-probe", action="store_true",
                   help="also run a 1 GiB torch device copy 5 times (counter calibration)")
    return p.parse_args()


def _default_rounding(storage):
    return "stochastic" if storage in ("f16", "bf16") else "nearest"


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def _timed(torch, stream, fn):
    """Milliseconds of fn() by HIP events recorded on `stream`, synchronised
    on both sides."""
    torch.cuda.synchronize()
    e0, e1 = _events(torch)
    e0.record(stream)
    fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


# ---------------------------------------------------------------- GPU legs

def _copy_probe(torch):
    """A plain copy of known size: its FETCH_SIZE / WRITE_SIZE per dispatch
    calibrate the same counters taken on the stream-collide kernel."""
    n = (1 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def _copy_ceiling(torch):
    """Device-to-device copy rate (read + write bytes per second) of a 2 GiB
    torch copy: a reference ceiling for streaming kernels on this part."""
    n = (2 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    stream = torch.cuda.current_stream()
    ms = _timed(torch, stream, lambda: [b.copy_(a) for _ in range(5)]) / 5
    del a, b
    torch.cuda.empty_cache()
    return {"gbs": round(2 * n * 4 / (ms / 1e3) / 1e9, 1), "bytes": 2 * n * 4, "kind": "torch device copy, 2 GiB"}


def _launch_ms(lat, K, fuse, torch):
    """Average duration of the dominant launch by HIP events on the launch
    stream: j fused launches of `fuse` steps (or single steps) issued right
    after a check step and ending before the next one, so every launch is a
    plain one of the full length."""
    if K > 0:
        lat.step((-lat.steps) % K)            # up to the next check step
    if fuse >= 2:
        j = max(1, (K - 1) // fuse - 1) if K > 0 else 15
        return _timed(torch, lat.stream, lambda: lat.step(j * fuse)) / j
    n = max(1, min(50, K - 2)) if K > 0 else 50
    return _timed(torch, lat.stream, lambda: lat.step(n)) / n


def _run_c3(args, storage, rounding, torch, P, W, sample_rows, host_io=False):
    """One storage kind on the second-sound lattice: timed steps, then the
    run continued to the accuracy step count and the moments of the sampled
    rows taken (device readout)."""
    case = W.second_sound_case(n=args.n)
    scale = 2.0 ** -20 if storage.startswith("f16") else 0.0
    lat = P.Lattice([P.instance_from_case(case, scale)], storage=storage,
                    check_interval=args.check_interval, rounding=rounding, seed=1847)
    if args.fusion != "auto":
        lat.set_step_fusion(int(args.fusion))
    fuse = lat.step_fusion()
    tune = lat.autotune(10) if args.autotune else None
    T0 = W.initial_field(case)
    io = None
    if host_io:
        # host FP64 field -> device (PCIe) -> equilibrium init, synchronous
        t = time.perf_counter()
        lat.init(0, T0)
        io = {"init_from_host_s": time.perf_counter() - t}
    Td = torch.from_numpy(T0).to("cuda")
    lat.init(0, Td)
    del Td, T0
    lat.step(args.warmup)
    t0 = time.perf_counter()
    ms = _timed(torch, lat.stream, lambda: lat.step(args.steps))
    wall = time.perf_counter() - t0
    nodes = case.nx * case.ny
    step_s = ms / 1e3 / args.steps
    done = args.warmup + args.steps
    info = lat.last_check(0) if 0 < args.check_interval <= done else None
    if host_io:
        # FP64 (dT, qx, qy) of the final state back to the host
        t = time.perf_counter()
        lat.moments(0)
        io["moments_to_host_s"] = time.perf_counter() - t
        io["pcie_inclusive_mlups"] = nodes * args.steps / (io["init_from_host_s"] + ms / 1e3
                                                           + io["moments_to_host_s"]) / 1e6
    launch_ms = _launch_ms(lat, args.check_interval, fuse, torch)
    shape = lat.launch_shape()
    # accuracy: on to the workload's step count, then the sampled rows
    n_acc = max(args.accuracy_steps, lat.steps)
    lat.step(n_acc - lat.steps)
    dT, qx, qy = lat.moments_device(0)
    idx = torch.as_tensor(sample_rows, device=dT.device)
    samples = [t.index_select(0, idx).cpu().numpy() for t in (dT, qx, qy)]
    del dT, qx, qy
    lat.close()
    torch.cuda.empty_cache()
    return dict(storage=storage, rounding=rounding, fusion=fuse, mlups=nodes / step_s / 1e6,
                ms_per_step=ms / args.steps, gbs=BYTES_PER_NODE[storage] * nodes / step_s / 1e9,
                launch_ms=launch_ms, wall_s=wall, check=info, shape=shape, tune=tune, host_io=io,
                accuracy_steps=n_acc, _samples=samples)


def _run_front(args, torch, P, W):
    """FP32 pulse on the second-sound lattice: the temperature along the
    centre row, from the centre outwards, at t = 150, 200, ..., 400."""
    case = W.second_sound_case(n=args.n)
    a = case.init_args
    lat = P.Lattice([P.instance_from_case(case)], storage="f32", check_interval=-1)
    lat.init(0, torch.from_numpy(W.initial_field(case)).to("cuda"))
    times = list(range(150, 401, 50))
    profiles = []
    for t in times:
        lat.step(t - lat.steps)
        dT, _, _ = lat.moments_device(0)
        profiles.append(dT[a["cy"], a["cx"]:].cpu().numpy())
        del dT
    lat.close()
    torch.cuda.empty_cache()
    return {"times": times, "_profiles": profiles}


def _run_walls(torch, P, W):
    """128 x 64, isothermal walls at T0 +- 0.5 along x, periodic y, 5000
    steps, FP32 (cache-resident: MLUPS only)."""
    case = W.wall_case()
    lat = P.Lattice([P.instance_from_case(case)], storage="f32")
    lat.init(0)
    ms = _timed(torch, lat.stream, lambda: lat.step(case.steps))
    fields = lat.moments(0)
    fuse = lat.step_fusion()
    lat.close()
    nodes = case.nx * case.ny
    return {"workload": f"walls_{case.nx}x{case.ny}", "steps": case.steps, "storage": "f32",
            "mlups": round(nodes * case.steps / (ms / 1e3) / 1e6, 1), "ms_per_step": round(ms / case.steps, 5),
            "steps_per_launch": fuse, "_fields": fields}


def _run_channel(torch, P, W, tau_n=0.6, ratio=100.0):
    """1024 x 256 gradient channel with diffuse walls (tau_R / tau_N = ratio)
    run to steady state (checks every 1000 steps until r < 1e-10 or the
    rounded map stops, r = 0) on the graph schedule, FP32."""
    case = W.poiseuille_case(tau_n, ratio)
    lat = P.Lattice([P.instance_from_case(case)], storage="f32", check_interval=1000)
    lat.set_schedule("graph")
    lat.init(0)
    ms = 0.0
    r = 1.0
    while lat.steps < 100000:
        ms += _timed(torch, lat.stream, lambda: lat.step(1000))
        r = lat.residual(0)
        if r < 1e-10:
            break
    steps = lat.steps
    fields = lat.moments(0)
    fuse = lat.step_fusion()
    lat.close()
    nodes = case.nx * case.ny
    return {"workload": f"channel_{case.nx}x{case.ny}_tau_n{tau_n}_ratio{ratio:g}", "storage": "f32",
            "steps_to_steady": steps, "residual": r, "steps_per_launch": fuse,
            "mlups": round(nodes * steps / (ms / 1e3) / 1e6, 1), "ms_per_step": round(ms / steps, 5),
            "_fields": fields, "_case": (tau_n, ratio)}


def _run_sweep(args, torch, P, W, picks=(0, 1, 2, 3)):
    """Knudsen sweep: 256 channel instances (sides uniform in [64, 512],
    tau_N uniform in [0.51, 1], tau_R log-uniform in [0.6, 1000], gradient
    seam and diffuse walls), FP32, check steps every 100.  MLUPS of each
    schedule over the same timed steps from the same initial state (batched:
    the default two streams, and one); the batched run's fields of a few
    instances for the error."""
    cases = W.knudsen_sweep()
    insts = [P.instance_from_case(c) for c in cases]
    nodes = sum(c.nx * c.ny for c in cases)
    out = {"instances": len(cases), "nodes": nodes, "steps": args.sweep_steps, "storage": "f32"}
    for sched in ("graph", "batched", "batched_one_stream", "per_instance"):
        lat = P.Lattice(insts, check_interval=100)
        lat.set_schedule("batched" if sched == "batched_one_stream" else sched)
        if sched == "batched_one_stream":
            lat.set_streams(1)
        for k in range(len(cases)):
            lat.init(k)
        lat.step(100)                      # warm-up; captures the graphs
        ms = _timed(torch, lat.stream, lambda: lat.step(args.sweep_steps))
        if sched == "batched":
            out["_fields"] = {k: lat.moments(k) for k in picks}
            out["fields_at_step"] = lat.steps
            out["steps_per_launch"] = lat.step_fusion()
            out["batched_streams"] = lat.streams()
        lat.close()
        step_s = ms / 1e3 / args.sweep_steps
        out[sched] = {"mlups": round(nodes / step_s / 1e6, 1), "ms_per_step": round(ms / args.sweep_steps, 4),
                      "gbs": round(64 * nodes / step_s / 1e9, 1)}
    out["batched_over_per_instance"] = round(out["batched"]["mlups"] / out["per_instance"]["mlups"], 2)
    out["graph_over_per_instance"] = round(out["graph"]["mlups"] / out["per_instance"]["mlups"], 2)
    return out


def _run_large(args, torch, P, W, sample_rows):
    """Large bandwidth-bound run: 16384^2 periodic, T0 = 1 plus 16 seeded
    Fourier modes (total amplitude 1e-3), tau_N = 0.6, tau_R = 5, 16-bit
    storage scaled by 2^-22 (FP16), check steps every 100; the field is built
    on the device.  Each row: timed steps, then on to the workload's 1000
    steps, the sampled rows, and the FP64 totals at the start and the end."""
    case = W.smooth_modes_case()
    modes = case.init_args["modes"]
    nodes = case.nx * case.ny
    out = {"workload": f"smooth_modes_{case.nx}x{case.ny}_periodic", "nodes": nodes, "tau_n": case.tau_n,
           "tau_r": case.tau_r, "steps": args.large_steps, "rows": []}
    for item in [r for r in args.large_rows.split(",") if r]:
        st, _, rnd = item.partition(":")
        rnd = rnd or _default_rounding(st)
        scale = 2.0 ** -22 if st.startswith("f16") else 0.0
        lat = P.Lattice([P.instance_from_case(case, scale)], storage=st, check_interval=args.check_interval,
                        rounding=rnd, seed=1847)
        T0 = W.modes_field_torch(modes, case.nx, case.ny, case.t0, device="cuda")
        lat.init(0, T0)
        del T0
        torch.cuda.empty_cache()
        tot0 = lat.totals(0)
        lat.step(20)
        ms = _timed(torch, lat.stream, lambda: lat.step(args.large_steps)) / args.large_steps
        n_acc = max(case.steps, lat.steps)
        lat.step(n_acc - lat.steps)
        tot1 = lat.totals(0)
        dT, qx, qy = lat.moments_device(0)
        idx = torch.as_tensor(sample_rows, device=dT.device)
        samples = [t.index_select(0, idx).cpu().numpy() for t in (dT, qx, qy)]
        del dT, qx, qy
        out["rows"].append({"storage": st, "rounding": rnd, "steps_per_launch": lat.step_fusion(),
                            "mlups": round(nodes / ms / 1e3, 1), "ms_per_step": round(ms, 4),
                            "gbs": round(BYTES_PER_NODE[st] * nodes / ms / 1e6, 1), "accuracy_steps": n_acc,
                            "totals_start": [float(v) for v in tot0], "totals_end": [float(v) for v in tot1],
                            "_samples": samples})
        lat.close()
        torch.cuda.empty_cache()
    return out


def _run_d3q14(args, torch, W, n_sample=4096):
    """D3Q14 thermal-wave box: periodic n^3 (n = 512 by default), T0 = 1 plus
    16 seeded Fourier modes (wave numbers up to 8 per axis, total amplitude
    1e-3), tau_N = 0.6, tau_R = 5, no initial flux; chunked layout, launch
    shape and steps per launch (one, or two with the z-marching kernel) chosen
    by the library's autotuner.  The per-launch time is the HIP-event time
    over the timed steps (consecutive launches on one stream) divided by the
    number of launches.  Each row's fields at n_sample seeded nodes after the
    timed steps."""
    import numpy as np
    from paper_2010_01847_amd.d3q14 import Box
    case = W.thermal_waves_3d_case(args.d3q14_n)
    nodes = case.nodes
    rng = np.random.default_rng(9)
    xs, ys, zs = (rng.integers(0, case.nx, n_sample) for _ in range(3))
    out = {"workload": f"thermal_waves_{case.nx}^3_periodic_d3q14", "nodes": nodes, "tau_n": case.tau_n,
           "tau_r": case.tau_r, "steps": args.d3q14_steps, "rows": [], "_nodes": (xs, ys, zs)}
    for item in [r for r in args.d3q14_rows.split(",") if r]:
        st, _, rnd = item.partition(":")
        rnd = rnd or "nearest"
        scale = 2.0 ** -23 if st == "f16" else 0.0
        box = Box(case.nx, case.ny, case.nz, case.tau_n, case.tau_r, storage=st, scale=scale,
                  stochastic=rnd == "stochastic", seed=1847)
        if args.d3q14_shape == "auto":
            fuse = box.autotune(10)["steps_per_launch"]
        else:
            vals = [int(v) for v in args.d3q14_shape.split(",")]
            box.set_launch_shape(*vals[:5])
            fuse = vals[5] if len(vals) > 5 else (2 if st == "f32" else 1)
            box.set_step_fusion(fuse)
        shape = box.launch_shape()
        T0 = W.modes_field_3d_torch(case.init_args["modes"], case.nx, case.ny, case.nz, case.t0, "cuda")
        box.init(T0)
        del T0
        stream = torch.cuda.current_stream()
        box.step(20)
        ms = _timed(torch, stream, lambda: box.step(args.d3q14_steps)) / args.d3q14_steps
        samples = box.sample(xs, ys, zs)
        done = 20 + args.d3q14_steps
        box.close()
        torch.cuda.empty_cache()
        # algorithmic bytes per launch: 14 reads + 14 writes per update, times
        # the updates one launch performs (fuse = 2 for the z-marching kernel)
        gbs = BYTES_PER_NODE_3D[st] * nodes / (ms / 1e3) / 1e9
        out["rows"].append({"storage": st, "rounding": rnd, "mlups": round(nodes / (ms / 1e3) / 1e6, 1),
                            "ms_per_step": round(ms, 4), "steps_per_launch": fuse,
                            "launch_us": round(ms * fuse * 1e3, 1), "gbs": round(gbs, 1),
                            "frac": round(gbs / HBM_PEAK_GBS, 4), "layout": "chunked", "launch_shape": shape,
                            "accuracy_steps": done, "_samples": samples})
    f32 = [r for r in out["rows"] if r["storage"] == "f32"]
    if f32:
        r = f32[0]
        two = r["steps_per_launch"] == 2
        traffic = _traffic_from(os.path.join(
            PROFILES, f"stream_collide_d3q14_f32{'_pair' if two else ''}_thermal_waves_{case.nx}.md"),
            KERNEL_SOURCES_3D)
        # compulsory bytes of one launch: the state read once and written once;
        # achieved from the counters' bytes while the profile is current
        compulsory = BYTES_PER_NODE_3D["f32"] * nodes
        moved = traffic if traffic is not None else compulsory
        t = r["launch_us"] / 1e6
        out["roofline"] = {"bound": "hbm",
                           "achieved": round(moved / t / 1e9, 1),
                           "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(moved / t / 1e9 / HBM_PEAK_GBS, 4),
                           "traffic": traffic,
                           "achieved_bytes": "measured (rocprofv3 counters)" if traffic is not None else
                                             "compulsory (profile stale)",
                           "kernel": ("d3q14 pair_kernel (two steps per launch, z-marching)" if two
                                      else "d3q14 step_kernel"),
                           "steps_per_launch": r["steps_per_launch"], "kernel_us": r["launch_us"],
                           "bytes_per_launch": moved,
                           "compulsory": {"bytes_per_launch": compulsory, "gbs": round(compulsory / t / 1e9, 1),
                                          "frac": round(compulsory / t / 1e9 / HBM_PEAK_GBS, 4)},
                           "single_step_equivalent": {"gbs": r["gbs"], "x_peak": r["frac"]}}
    return out


# ---------------------------------------------------------------- oracle leg

def _rel_l2(pairs):
    import numpy as np
    num = math.sqrt(sum(float(np.sum((a - b) ** 2)) for a, b in pairs))
    den = math.sqrt(sum(float(np.sum(b ** 2)) for _, b in pairs))
    return num / den if den > 0 else num


def _eps_fields(case, gpu, ora):
    """(eps_T, eps_q) of a GPU readout (dT = T - T_ref, qx, qy) against the
    oracle's (T, qx, qy): eps_T = ||T - T_or|| / ||T_or - t0|| (the ramp of a
    gradient channel included), eps_q = ||q - q_or|| / ||q_or||."""
    import numpy as np
    dT, qx, qy = gpu
    T, qxo, qyo = ora
    ramp = np.broadcast_to(case.t_ref()[: dT.shape[1]][None, :], dT.shape)
    num = float(np.linalg.norm(dT + ramp - T))
    den = float(np.linalg.norm(T - case.t0))
    return (num / den if den > 0 else num), _rel_l2([(qx, qxo), (qy, qyo)])


def _bound_check(storage, e_t, e_q):
    bound = BOUND[storage]
    ok = e_t <= bound and e_q <= bound
    return {"eps_T": float(f"{e_t:.4g}"), "eps_q": float(f"{e_q:.4g}"), "bound": bound, "pass": ok,
            **({} if ok else {"note": "misses the 16-bit bound" if bound == 5e-3 else "misses the FP32 bound"})}


def _cpu_baseline(args, W, ref):
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    ref.set_threads(threads)
    # bounded window of the same workload: 2048 x 2048 centred sub-lattice of
    # the 8192^2 pulse (same pulse, same tau's), stepped on the host
    n = 2048
    case = W.second_sound_case(n=n)
    o = ref.Oracle(case, W.initial_field(case))
    o.run(2)                               # thread start-up, first touch
    per_step = max(o.run(4) / 4, 1e-6)
    steps = max(2, int(args.cpu_seconds / per_step))
    t = o.run(steps)
    mlups = n * n * steps / t / 1e6
    # the same stepper on one thread (512^2 window, about 2 s)
    ref.set_threads(1)
    small = W.second_sound_case(n=512)
    o1 = ref.Oracle(small, W.initial_field(small))
    t1 = o1.run(2)
    s1 = max(2, int(2.0 / max(t1 / 2, 1e-6)))
    t1 = o1.run(s1)
    ref.set_threads(threads)
    return dict(value=mlups, unit="MLUPS", cores=threads, kind="oracle",
                sample=f"{n}x{n} window of the 8192^2 second-sound lattice, {steps} steps, "
                       f"{t:.1f} s, FP64 C stepper with OpenMP over rows",
                value_1_thread=512 * 512 * s1 / t1 / 1e6)


def _oracle_leg(args, W, c3_rows, c3_sample_rows, front, walls, channel, sweep, large, large_rows, d3q14):
    """The oracle on the host: its timing (cpu_baseline) and the error of
    every GPU row against it (exact periodic solutions for the periodic
    lattices, the FP64 stepper for the walled ones)."""
    import numpy as np
    from oracle import bloch, bloch_d3q14, closed_forms as cf, ref
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from measure import front_radius
    out = {}
    # second sound: exact solution on the sampled rows at each row's step count
    case = W.second_sound_case(n=args.n)
    a = case.init_args
    x = np.arange(case.nx, dtype=np.float64)
    f = np.exp(-(x - a["cx"]) ** 2 / (2 * a["sigma"] ** 2))
    exact = {}
    for r in c3_rows:
        n = r["accuracy_steps"]
        if n not in exact:
            exact[n] = bloch.SeparableSolution(f, f, a["amp"], n, case.tau_n, case.tau_r).rows(c3_sample_rows)
        To, qxo, qyo = exact[n]
        dT, qx, qy = r.pop("_samples")
        r["accuracy"] = _bound_check(r["storage"], _rel_l2([(dT, To - 1.0)]), _rel_l2([(qx, qxo), (qy, qyo)]))
        r["accuracy"]["compared"] = f"{len(c3_sample_rows)} rows x {case.nx} after {n} steps vs exact solution"
    # pulse front: ring-peak radius along the centre row, least-squares speed
    if front:
        nn = 2048
        xx = np.arange(nn, dtype=np.float64)
        ff = np.exp(-(xx - nn // 2) ** 2 / (2 * a["sigma"] ** 2))
        r_gpu = [front_radius(p) for p in front.pop("_profiles")]
        r_ora = [front_radius(bloch.SeparableSolution(ff, ff, a["amp"], t, case.tau_n, case.tau_r)
                              .rows([nn // 2])[0][0, nn // 2:] - 1.0) for t in front["times"]]
        front["speed_gpu"] = float(np.polyfit(front["times"], r_gpu, 1)[0])
        front["speed_oracle"] = float(np.polyfit(front["times"], r_ora, 1)[0])
        front["radius_max_diff"] = float(max(abs(p - q) for p, q in zip(r_gpu, r_ora)))
        front["hydrodynamic_speed"] = cf.second_sound_speed()
        front["unit"] = "nodes/step"
    # walls: FP64 stepper, whole lattice
    if walls:
        wc = W.wall_case()
        o = ref.Oracle(wc)
        o.run(wc.steps)
        T, qxo, qyo = o.moments()
        walls["accuracy"] = _bound_check("f32", *_eps_fields(wc, walls.pop("_fields"), (T, qxo, qyo)))
    # channel: FP64 steady state (the solution is uniform along x: 4 columns)
    if channel:
        tau_n, ratio = channel.pop("_case")
        cc = W.poiseuille_case(tau_n, ratio)
        o = ref.Oracle(W.poiseuille_case(tau_n, ratio, nx=4))
        prev = None
        while o.steps < 200000:
            o.run(1000)
            _, qxo, _ = o.moments()
            if prev is not None and np.abs(qxo - prev).max() <= 1e-12 * np.abs(qxo).max():
                break
            prev = qxo.copy()
        T, qxo, qyo = o.moments()
        dT, qx, qy = channel.pop("_fields")
        channel["accuracy"] = _bound_check("f32", *_eps_fields(cc, (dT[:, :4], qx[:, :4], qy[:, :4]), (T, qxo, qyo)))
        channel["accuracy"]["compared"] = "columns 0-3 (the solution is uniform along x), all rows"
        d = cc.ny - 1
        kn_c = cf.knudsen(cf.scheme_constants(tau_n, cc.tau_r)["tau_c"], d)
        kn_r = cf.knudsen(cc.tau_r, d)
        channel["conductivity_ratio"] = float((qx[:, 0] / cf.poiseuille_q_scale(cc.tau_r, cc.grad_x)).mean())
        channel["conductivity_ratio_eq69"] = float(cf.poiseuille_conductivity_eq69(kn_c, kn_r))
    # sweep: FP64 stepper on a few instances at the batched run's step count
    if sweep and "_fields" in sweep:
        cases = W.knudsen_sweep()
        worst_t = worst_q = 0.0
        for k, fields in sweep.pop("_fields").items():
            c = cases[k]
            o = ref.Oracle(c)
            o.run(sweep["fields_at_step"])
            e_t, e_q = _eps_fields(c, fields, o.moments())
            worst_t, worst_q = max(worst_t, e_t), max(worst_q, e_q)
        sweep["accuracy"] = _bound_check("f32", worst_t, worst_q)
        sweep["accuracy"]["compared"] = "worst of instances 0-3, all nodes"
    # large: exact 16-mode solution on the sampled rows; totals against the
    # exact invariants (energy kept, heat flux times rho per step)
    if large:
        lc = W.smooth_modes_case()
        sol = {}
        rho = cf.scheme_constants(lc.tau_n, lc.tau_r)["rho"]
        for r in large["rows"]:
            n = r["accuracy_steps"]
            if n not in sol:
                sol[n] = bloch.ModeSolution(lc.init_args["modes"], lc.nx, lc.ny, n, lc.tau_n, lc.tau_r).rows(large_rows)
            To, qxo, qyo = sol[n]
            dT, qx, qy = r.pop("_samples")
            r["accuracy"] = _bound_check(r["storage"], _rel_l2([(dT, To - 1.0)]), _rel_l2([(qx, qxo), (qy, qyo)]))
            r["accuracy"]["compared"] = f"{len(large_rows)} rows x {lc.nx} after {n} steps vs exact solution"
            e0, e1 = r["totals_start"][0], r["totals_end"][0]
            amp = 1e-3 * lc.nx * lc.ny     # the field's amplitude times the node count
            r["totals_drift"] = {"energy_abs": e1 - e0, "energy_rel_to_amplitude": abs(e1 - e0) / amp,
                                 "qx_expected_factor": rho ** n}
    # D3Q14: exact 16-mode solution at the sampled nodes
    if d3q14:
        dc = W.thermal_waves_3d_case(args.d3q14_n)
        xs, ys, zs = d3q14.pop("_nodes")
        for r in d3q14["rows"]:
            s = r.pop("_samples")
            T, qx, qy, qz = bloch_d3q14.ModeSolution(dc.init_args["modes"], dc.nx, dc.ny, dc.nz, r["accuracy_steps"],
                                                    dc.tau_n, dc.tau_r).at(xs, ys, zs)
            r["accuracy"] = _bound_check(r["storage"], _rel_l2([(s[:, 0], T - 1.0)]),
                                     _rel_l2([(s[:, 1], qx), (s[:, 2], qy), (s[:, 3], qz)]))
    out["cpu_baseline"] = _cpu_baseline(args, W, ref)
    return out


def _strip(d):
    """Drop the arrays handed to the oracle leg when it did not run."""
    if isinstance(d, dict):
        return {k: _strip(v) for k, v in d.items() if not k.startswith("_")}
    if isinstance(d, list):
        return [_strip(v) for v in d]
    return d


def _round(d):
    if isinstance(d, dict):
        return {k: _round(v) for k, v in d.items()}
    if isinstance(d, list):
        return [_round(v) for v in d]
    if isinstance(d, float):
        return float(f"{d:.6g}")
    return d


def main():
    args = _parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    import workloads as W
    import paper_2010_01847_amd as P
    torch.cuda.set_device(0)
    if args.copy_probe:
        _copy_probe(torch)
    copy = _copy_ceiling(torch)
    # sampled rows of the second-sound lattice: offsets 17 and 31 within the
    # fused kernel's 32-row chunks, and the pulse's centre row
    n = args.n
    c3_sample_rows = sorted(set(list(range(17, n, 64)) + list(range(31, n, 128)) + [n // 2]))
    main_rounding = args.rounding or _default_rounding(args.storage)
    main_row = _run_c3(args, args.storage, main_rounding, torch, P, W, c3_sample_rows, host_io=True)
    rows = [main_row]
    for item in [r for r in args.rows.split(",") if r]:
        st, _, rnd = item.partition(":")
        rnd = rnd or _default_rounding(st)
        if (st, rnd) != (args.storage, main_rounding):
            rows.append(_run_c3(args, st, rnd, torch, P, W, c3_sample_rows))
    front = _run_front(args, torch, P, W) if args.front else None
    walls = _run_walls(torch, P, W) if args.small else None
    channel = _run_channel(torch, P, W) if args.small else None
    sweep = _run_sweep(args, torch, P, W) if args.sweep_steps > 0 else None
    large_rows = sorted(list(range(17, 16384, 128)) + list(range(95, 16384, 256)))
    large = _run_large(args, torch, P, W, large_rows) if args.large_steps > 0 else None
    d3q14 = _run_d3q14(args, torch, W) if args.d3q14_steps > 0 else None
    oracle = None if args.no_cpu_baseline else _oracle_leg(args, W, rows, c3_sample_rows, front, walls, channel,
                                                           sweep, large, large_rows, d3q14)

    # roofline of the dominant kernel (see the module docstring)
    nodes = args.n * args.n
    fuse = main_row["fusion"]
    t_launch = main_row["launch_ms"] / 1e3
    compulsory = BYTES_PER_NODE[args.storage] * nodes
    traffic = _traffic_from(os.path.join(PROFILES, f"stream_collide_{args.storage}_second_sound_{args.n}.md"),
                            KERNEL_SOURCES)
    flops = FLOP_PER_UPDATE * nodes * fuse / t_launch / 1e12
    # achieved: the HBM bytes the counters measured per launch (profiles/) over
    # the live launch time; the compulsory bytes (state read once and written
    # once) stand in, and say so, while the profile is stale
    moved = traffic if traffic is not None else compulsory
    roofline = {
        "bound": "hbm", "achieved": moved / t_launch / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": moved / t_launch / 1e9 / HBM_PEAK_GBS, "traffic": traffic,
        "achieved_bytes": ("measured: rocprofv3 FETCH_SIZE + WRITE_SIZE per launch, scaled by a 2 GiB copy"
                           if traffic is not None else
                           "compulsory (the profile's kernel sources differ from these): state read once and "
                           "written once per launch"),
        "limiter": "VALU issue (alu below; instruction counters in profiles/)" if fuse >= 6 else
                   "memory requests",
        "kernel": (f"march_kernel ({fuse} time steps per launch, y-marching temporal blocking)" if fuse >= 2
                   else "wave_kernel (pull-advection + boundary + moments + relaxation, one step)"),
        "steps_per_launch": fuse, "kernel_us": main_row["launch_ms"] * 1e3, "bytes_per_launch": moved,
        "compulsory": {"bytes_per_launch": compulsory, "gbs": compulsory / t_launch / 1e9,
                       "frac": compulsory / t_launch / 1e9 / HBM_PEAK_GBS,
                       "note": "the state read once and written once per launch"},
        "measured_hbm": (None if traffic is None else
                         {"gbs": traffic / t_launch / 1e9, "frac": traffic / t_launch / 1e9 / HBM_PEAK_GBS,
                          "over_compulsory": traffic / compulsory}),
        "single_step_equivalent": {"bytes_per_launch": compulsory * fuse,
                                   "gbs": compulsory * fuse / t_launch / 1e9,
                                   "x_peak": compulsory * fuse / t_launch / 1e9 / HBM_PEAK_GBS,
                                   "single_step_roofline_mlups": HBM_PEAK_GBS * 1e3 / BYTES_PER_NODE[args.storage]},
        "alu": {"achieved": flops, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": flops / FP32_VECTOR_PEAK_TFLOPS, "flop_per_update": FLOP_PER_UPDATE,
                "peak_note": "vector FP32 without packed instructions"},
        "copy_ceiling": {**copy, "frac": moved / t_launch / 1e9 / copy["gbs"]},
    }
    out = {
        "metric": "MLUPS and % of HBM roofline, FP32 vs 16-bit storage vs FP64 oracle error",
        "value": round(main_row["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_row["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.storage,
        "data": "synthetic",
        "config": {"workload": f"second_sound_{args.n}x{args.n}_periodic", "nx": args.n, "ny": args.n,
                   "tau_n": 0.55, "tau_r": 50.0, "storage": args.storage, "rounding": main_rounding,
                   "check_interval": args.check_interval, "launch_shape": main_row["shape"]},
        "accuracy": main_row.get("accuracy"),
        "roofline": roofline,
        "cpu_baseline": None if oracle is None else oracle["cpu_baseline"],
        "rows": [{k: v for k, v in r.items() if k not in ("tune", "host_io")} for r in rows],
        "front": front,
        "walls": walls,
        "channel": channel,
        "sweep": sweep,
        "large": large,
        "d3q14": d3q14,
        "host_io": main_row["host_io"],
    }
    print(json.dumps(_round(_strip(out))), flush=True)


if __name__ == "__main__":
    main()
