"""Throughput of the fused D2Q8 phonon stream-collide step on one MI355X.

Default workload: the second-sound configuration -- 8192 x 8192 periodic
lattice, Gaussian pulse dT = 0.01 exp(-r^2 / (2 * 20^2)) on T0 = 1 at the
centre, tau_N = 0.55, tau_R = 50 -- with FP32 storage of the scaled
deviations, FP32 arithmetic, and FP64 check-step reductions every 100 steps.
A step is one pass of the whole hot path over the lattice: pull-advection,
boundary handling, moments in registers, relaxation with the resistive
source, store, and (on check steps) the FP64 snapshot/residual/total
reductions.

Prints one JSON line.  `value` is MLUPS (million lattice-node updates per
second) of the timed steps, with the populations resident in HBM before the
timed region starts.  Extra storage types (FP16 scaled, BF16; stochastic
rounding of the stores, which keeps smooth fields from stalling) of the same
workload are reported under "rows".  "sweep" reports the batched Knudsen
sweep (256 uneven channel instances in one handle) under the three
schedules: one launch for all instances, the same captured in HIP graphs,
and one launch per instance.  "large" reports the 16384^2 smooth-modes
lattice with FP16 storage.  "d3q14" reports the three-dimensional lattice on
a 512^3 periodic box (FP32, BF16 and FP16 storage) with its own roofline.
The oracle (plain FP64 C stepper) is timed on a bounded window of the same
workload on the host cores ("cpu_baseline").

The dominant launch advances several steps per pass over HBM (temporal
blocking), so the roofline's "achieved" (algorithmic bytes of the updates it
performs over its duration) exceeds the HBM peak; "traffic" is the measured
HBM bytes per launch, and "alu" states the same launch against the vector
FP32 peak.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, 8 TB/s
# 8 population reads + 8 writes per node; split storage adds the FP32 energy
# FP32 operations of one D2Q8 relaxation (moments, equilibrium shares, the
# eight updates; a fused multiply-add counts 2), and MI355X's vector FP32 peak
FLOP_PER_UPDATE = 81
FP32_VECTOR_PEAK_TFLOPS = 157.3
BYTES_PER_NODE = {"f32": 64, "f16": 32, "bf16": 32, "f16_split": 40, "bf16_split": 40}
# D3Q14: 14 population reads + 14 writes per node
BYTES_PER_NODE_3D = {"f32": 112, "f16": 56, "bf16": 56}
_CSRC = os.path.join(ROOT, "paper_2010_01847_amd", "csrc")
# the device code and the headers that fix its tiles, descriptors and rounding
KERNEL_SOURCES = [os.path.join(_CSRC, f) for f in ("lbm_device.hip", "lbm_internal.h", "lbm_numeric.h")]
KERNEL_SOURCES_3D = [os.path.join(_CSRC, f) for f in ("d3q14_device.hip", "d3q14_internal.h", "lbm_numeric.h")]
PROFILES = os.path.join(ROOT, "profiles")


def _measured_traffic(storage: str, n: int):
    """HBM bytes per launch of the D2Q8 step kernel from the committed
    rocprofv3 counter summary (FETCH_SIZE and WRITE_SIZE scaled by a 1 GiB
    copy), or None when no summary covers this workload or the kernel source
    changed since the counters were taken (hash of the device sources)."""
    return _traffic_from(os.path.join(PROFILES, f"stream_collide_{storage}_second_sound_{n}.md"), KERNEL_SOURCES)


def _traffic_from(path: str, sources):
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
    p.add_argument("--rows", default="f16:stochastic,bf16:stochastic,f16_split,bf16_split",
                   help="extra rows, storage[:rounding] ('' for none)")
    p.add_argument("--rounding", default=None, choices=["nearest", "stochastic"],
                   help="rounding of the main row's stores (default: stochastic for plain 16-bit "
                        "storage, which stalls on smooth fields otherwise; nearest for the rest)")
    p.add_argument("--sweep-steps", type=int, default=300, help="timed steps per sweep schedule (0: skip)")
    p.add_argument("--fusion", default="auto",
                   help="most time steps per launch (auto: the library's default for the storage kind)")
    p.add_argument("--check-interval", type=int, default=100)
    p.add_argument("--no-cpu-baseline", action="store_true")
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
    p.add_argument("--large-rows", default="f16:stochastic,f16_split",
                   help="storage[:rounding] rows of the 16384^2 smooth-modes lattice")
    p.add_argument("--copy-probe", action="store_true",
                   help="also run a 1 GiB torch device copy 5 times (counter calibration)")
    return p.parse_args()


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


def _run_gpu(args, storage, rounding, torch, P, W, host_io=False):
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
    stream = lat.stream
    lat.step(args.warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    t0 = time.perf_counter()
    lat.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    nodes = case.nx * case.ny
    step_s = ms / 1e3 / args.steps
    mlups = nodes / step_s / 1e6
    gbs = BYTES_PER_NODE[storage] * nodes / step_s / 1e9
    done = args.warmup + args.steps
    info = lat.last_check(0) if 0 < args.check_interval <= done else None
    if host_io:
        # FP64 (dT, qx, qy) of the final state back to the host
        t = time.perf_counter()
        lat.moments(0)
        io["moments_to_host_s"] = time.perf_counter() - t
        io["pcie_inclusive_mlups"] = nodes * args.steps / (io["init_from_host_s"] + ms / 1e3
                                                           + io["moments_to_host_s"]) / 1e6
    launch_ms = _plain_launch_ms(lat, args.check_interval, fuse, torch)
    shape = lat.launch_shape()
    lat.close()
    # algorithmic bytes per launch: the per-update figure (read and write the
    # eight populations once) times the updates one launch performs
    alg = BYTES_PER_NODE[storage] * nodes * fuse
    return dict(storage=storage, rounding=rounding, fusion=fuse, mlups=mlups, ms_per_step=ms / args.steps,
                gbs=gbs, launch_ms=launch_ms, kernel_gbs=alg / (launch_ms / 1e3) / 1e9,
                wall_s=wall, check=info, shape=shape, tune=tune, host_io=io)


def _plain_launch_ms(lat, K, fuse, torch, n=95):
    """Average duration of the dominant launch (the plain stream-collide
    launch, or the fused launch of `fuse` steps), by HIP events on the launch
    stream around steps that hold no check-step work (strictly between two
    check steps, snapshot step excluded).  With fusion a call of 1 + j * fuse
    steps issues j fused launches and one single step (the last step of a
    call is never fused), timed by a separate one-step call."""
    if K > 2:
        lat.step((-lat.steps) % K + 1)      # past the next check step and the shift step after it
        n = min(n, K - 4)
    j = max(1, (n - 1) // fuse)
    n = 1 + j * fuse
    def timed(k):
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(lat.stream)
        lat.step(k)
        e1.record(lat.stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)
    t_run = timed(n)
    t_one = timed(1)
    if fuse >= 2:
        return (t_run - t_one) / j
    return (t_run + t_one) / (n + 1)


def _run_sweep(args, torch, P, W):
    """Knudsen sweep: 256 channel instances (sides uniform in [64, 512],
    tau_N uniform in [0.51, 1], tau_R log-uniform in [0.6, 1000], gradient
    seam and diffuse walls), FP32, check steps every 100.  MLUPS of each
    schedule over the same timed steps from the same initial state."""
    cases = W.knudsen_sweep()
    insts = [P.instance_from_case(c) for c in cases]
    nodes = sum(c.nx * c.ny for c in cases)
    out = {"instances": len(cases), "nodes": nodes, "steps": args.sweep_steps, "storage": "f32"}
    for sched in ("graph", "batched", "per_instance"):
        lat = P.Lattice(insts, check_interval=100)
        lat.set_schedule(sched)
        for k in range(len(cases)):
            lat.init(k)
        lat.step(100)                      # warm-up; captures the graphs
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(lat.stream)
        lat.step(args.sweep_steps)
        e1.record(lat.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        lat.close()
        step_s = ms / 1e3 / args.sweep_steps
        out[sched] = {"mlups": round(nodes / step_s / 1e6, 1), "ms_per_step": round(ms / args.sweep_steps, 4),
                      "gbs": round(64 * nodes / step_s / 1e9, 1)}
    out["batched_over_per_instance"] = round(out["batched"]["mlups"] / out["per_instance"]["mlups"], 2)
    out["graph_over_per_instance"] = round(out["graph"]["mlups"] / out["per_instance"]["mlups"], 2)
    return out


def _run_d3q14(args, torch, W):
    """D3Q14 thermal-wave box: periodic n^3 (n = 512 by default), T0 = 1 plus
    16 seeded Fourier modes (wave numbers up to 8 per axis, total amplitude
    1e-3), tau_N = 0.6, tau_R = 5, no initial flux; chunked layout, launch
    shape and steps per launch (one, or two with the z-marching kernel) chosen
    by the library's autotuner.  The per-launch time is the HIP-event time
    over the timed steps (consecutive launches on one stream) divided by the
    number of launches."""
    from paper_2010_01847_amd.d3q14 import Box
    case = W.thermal_waves_3d_case(args.d3q14_n)
    nodes = case.nodes
    out = {"workload": f"thermal_waves_{case.nx}^3_periodic_d3q14", "nodes": nodes, "tau_n": case.tau_n,
           "tau_r": case.tau_r, "steps": args.d3q14_steps, "rows": []}
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
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        box.step(args.d3q14_steps)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.d3q14_steps
        box.close()
        # algorithmic bytes per launch: 14 reads + 14 writes per update, times
        # the updates one launch performs (fuse = 2 for the z-marching kernel)
        gbs = BYTES_PER_NODE_3D[st] * nodes / (ms / 1e3) / 1e9
        out["rows"].append({"storage": st, "rounding": rnd, "mlups": round(nodes / (ms / 1e3) / 1e6, 1),
                            "ms_per_step": round(ms, 4), "steps_per_launch": fuse,
                            "launch_us": round(ms * fuse * 1e3, 1), "gbs": round(gbs, 1),
                            "frac": round(gbs / HBM_PEAK_GBS, 4), "layout": "chunked", "launch_shape": shape})
    f32 = [r for r in out["rows"] if r["storage"] == "f32"]
    if f32:
        r = f32[0]
        two = r["steps_per_launch"] == 2
        out["roofline"] = {"bound": "hbm", "achieved": r["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": r["frac"],
                           "kernel": ("d3q14 pair_kernel (two steps per launch, z-marching)" if two
                                      else "d3q14 step_kernel"),
                           "steps_per_launch": r["steps_per_launch"], "kernel_us": r["launch_us"],
                           "bytes_per_launch": BYTES_PER_NODE_3D["f32"] * nodes * r["steps_per_launch"],
                           "traffic": _traffic_from(os.path.join(
                               PROFILES, f"stream_collide_d3q14_f32{'_pair' if two else ''}_thermal_waves_{case.nx}.md"),
                               KERNEL_SOURCES_3D)}
    return out


def _run_large(args, torch, P, W):
    """Large bandwidth-bound run: 16384^2 periodic, T0 = 1 plus 16 seeded
    Fourier modes (total amplitude 1e-3), tau_N = 0.6, tau_R = 5, FP16
    storage scaled by 2^-22 (plain FP16 and the split form), check steps every
    100; the field is built on the device."""
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
        lat.step(20)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(lat.stream)
        lat.step(args.large_steps)
        e1.record(lat.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.large_steps
        out["rows"].append({"storage": st, "rounding": rnd, "steps_per_launch": lat.step_fusion(),
                            "mlups": round(nodes / ms / 1e3, 1), "ms_per_step": round(ms, 4),
                            "gbs": round(BYTES_PER_NODE[st] * nodes / ms / 1e6, 1)})
        lat.close()
    return out


def _default_rounding(storage):
    return "stochastic" if storage in ("f16", "bf16") else "nearest"


def _cpu_baseline(args, W):
    from oracle import ref
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
    main_rounding = args.rounding or _default_rounding(args.storage)
    main_row = _run_gpu(args, args.storage, main_rounding, torch, P, W, host_io=True)
    rows = [main_row]
    for item in [r for r in args.rows.split(",") if r]:
        st, _, rnd = item.partition(":")
        rnd = rnd or _default_rounding(st)
        if (st, rnd) != (args.storage, main_rounding):
            rows.append(_run_gpu(args, st, rnd, torch, P, W))
    sweep = _run_sweep(args, torch, P, W) if args.sweep_steps > 0 else None
    large = _run_large(args, torch, P, W) if args.large_steps > 0 else None
    d3q14 = _run_d3q14(args, torch, W) if args.d3q14_steps > 0 else None
    cpu = None if args.no_cpu_baseline else _cpu_baseline(args, W)
    gbs = main_row["kernel_gbs"]
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
        "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4),
                     "traffic": _measured_traffic(args.storage, args.n),
                     "kernel": (f"march_kernel ({main_row['fusion']} time steps per launch, y-marching "
                                "temporal blocking)" if main_row["fusion"] >= 2 else
                                "wave_kernel (fused pull-advection + boundary + moments + relaxation)"),
                     "steps_per_launch": main_row["fusion"],
                     "kernel_us": round(main_row["launch_ms"] * 1e3, 1),
                     "bytes_per_launch": BYTES_PER_NODE[args.storage] * args.n * args.n * main_row["fusion"],
                     # the fused kernel's real limit is VALU issue: the same launch
                     # against the vector FP32 peak, 81 algorithmic flops per update
                     "alu": {"achieved": round(FLOP_PER_UPDATE * args.n * args.n * main_row["fusion"]
                                               / (main_row["launch_ms"] * 1e-3) / 1e12, 2),
                             "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                             "frac": round(FLOP_PER_UPDATE * args.n * args.n * main_row["fusion"]
                                           / (main_row["launch_ms"] * 1e-3) / 1e12 / FP32_VECTOR_PEAK_TFLOPS, 4),
                             "flop_per_update": FLOP_PER_UPDATE}},
        "cpu_baseline": cpu,
        "sweep": sweep,
        "large": large,
        "d3q14": d3q14,
        "host_io": {k: round(v, 4) for k, v in main_row["host_io"].items()},
        "rows": [{k: (round(v, 3) if isinstance(v, float) else v) for k, v in r.items()
                  if k not in ("tune", "host_io")} for r in rows],
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
