"""The five workloads at their full sizes on the HIP path, checked against the
FP64 oracle.

* second sound 8192^2 and smooth modes 16384^2: exact periodic solutions
  (separable spectral route / 16-mode solution), compared on sampled rows;
* Poiseuille channels 1024 x 256: run to steady state on the GPU and against
  the oracle's FP64 steady state (the solution is uniform along x, so the
  oracle runs 4 columns);
* Knudsen sweep: 256 uneven channel instances in one batched handle, a subset
  stepped by the oracle, and the batched / per-instance / graph schedules.

Tolerances (relative L2 of the temperature deviation and of the heat flux):
FP32 storage 1e-5; 16-bit storage 5e-3.  The 16-bit runs use the library's
default step rounding (a fused launch of six steps rounds the state it stores
to 16 bits; its other steps stay in FP32 registers).  The split 16-bit kinds
(FP32 energy, 16-bit non-equilibrium shares) and plain FP16 population
storage (the eight populations in 16 bits), with either rounding, meet 5e-3
on every workload.  Plain BF16 storage misses the 16-bit bound on the heat
flux: on these smooth fields the heat flux is about a hundredth of the stored
populations, so its 8-bit-mantissa rounding noise is about a hundred times
larger relative to it.  Those misses are asserted as a band around the
measured value (the runs are deterministic: fixed seeds), so that a change in
either direction shows, and every row is also held to the per-node maximum
error bound.

Sampled rows of the full-size workloads sit off the 32-row marching chunks'
first rows (offsets 17 and 31 within a chunk), where the fused kernel's
carried pipeline state decides the result.
"""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import bloch, closed_forms as cf, ref
from measure import front_radius
from parity_util import eps, log, oracle_fields
from paper_2010_01847_amd import Lattice, instance_from_case

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "f16_split": 5e-3, "bf16_split": 5e-3}
TOL16 = 5e-3
# plain 16-bit kinds that miss the 16-bit bound on a workload: the measured
# (eps_T, eps_q) of the fixed-seed run; None where the bound is met
MISSES = {
    ("second_sound", "bf16", "stochastic"): (None, 8.584e-3),
    ("second_sound", "bf16", "nearest"): (None, 1.432e-2),
    ("smooth_modes", "bf16", "stochastic"): (None, 1.859e-2),
    ("smooth_modes", "bf16", "nearest"): (None, 1.691e-2),
}
BAND = (0.8, 1.25)
# per-node maximum error over the field's maximum magnitude: FP32 storage
# 3e-5 (measured up to 1.07e-5), split 16-bit kinds 1e-2 (measured up to
# 2.6e-3), FP16 3e-2 (up to 1.03e-2), BF16 0.5 (up to 0.13)
MAXREL = {"f32": 3e-5, "f16_split": 1e-2, "bf16_split": 1e-2, "f16": 3e-2, "bf16": 0.5}


def _rel(a, b, base):
    den = math.sqrt(float(np.sum(base ** 2)))
    return math.sqrt(float(np.sum((a - b) ** 2))) / den if den > 0 else 0.0


def _max_rel(pairs):
    """Per-node maximum error relative to the field's maximum magnitude."""
    num = max(float(np.abs(a - b).max()) for a, b in pairs)
    den = max(float(np.abs(b).max()) for _, b in pairs)
    return num / den if den > 0 else num


def _assert_eps(workload, storage, rounding, e_t, e_q):
    """FP32 1e-5, 16-bit 5e-3; a plain 16-bit kind that misses the 16-bit
    bound is held within BAND of its measured error."""
    if storage in TOL:
        assert e_t < TOL[storage] and e_q < TOL[storage], (workload, storage, rounding, e_t, e_q)
        return
    miss = MISSES.get((workload, storage, rounding), (None, None))
    for got, meas, name in ((e_t, miss[0], "eps_T"), (e_q, miss[1], "eps_q")):
        if meas is None:
            assert got < TOL16, (workload, storage, rounding, name, got)
        else:
            log(f"  {workload} {storage} {rounding} {name} misses the 16-bit bound: {got:.3e} "
                f"(measured {meas:.3e})")
            assert BAND[0] * meas <= got <= BAND[1] * meas, (workload, storage, rounding, name, got, meas)


def _run_rows(case, storage, scale, steps, rows, T0, check=100, rounding="nearest"):
    lat = Lattice([instance_from_case(case, scale)], storage=storage, check_interval=check,
                  rounding=rounding, seed=1847)
    lat.init(0, T0)
    lat.step(steps)
    dT, qx, qy = lat.moments_device(0)
    idx = torch.as_tensor(np.asarray(rows), device=dT.device)
    out = [t.index_select(0, idx).cpu().numpy() for t in (dT, qx, qy)]
    info = lat.last_check(0) if check > 0 and steps >= check else None
    del dT, qx, qy
    lat.close()
    torch.cuda.empty_cache()
    return out, info


# ---------------------------------------------------------------- second sound

@pytest.fixture(scope="module")
def second_sound_exact():
    case = W.second_sound_case()
    a = case.init_args
    x = np.arange(case.nx, dtype=np.float64)
    f = np.exp(-(x - a["cx"]) ** 2 / (2 * a["sigma"] ** 2))
    sol = bloch.SeparableSolution(f, f, a["amp"], case.steps, case.tau_n, case.tau_r)
    # offsets 17 and 31 within the 32-row chunks, and the pulse's centre rows
    rows = sorted(set(list(range(17, case.ny, 32)) + list(range(31, case.ny, 64))
                      + [a["cy"] + k for k in (-1, 0, 1, 2)]))
    return case, rows, sol.rows(rows)


SPLIT_ROWS = [("f16_split", "nearest"), ("bf16_split", "nearest"), ("f16_split", "stochastic"),
              ("bf16_split", "stochastic")]


@pytest.mark.parametrize("storage,rounding", [("f32", "nearest"), ("f32", "stochastic"),
                                              ("f16", "stochastic"), ("bf16", "stochastic"),
                                              ("f16", "nearest"), ("bf16", "nearest")] + SPLIT_ROWS)
def test_second_sound_8192(second_sound_exact, storage, rounding):
    """8192^2 periodic, Gaussian pulse, tau_N = 0.55, tau_R = 50, 4000 steps."""
    case, rows, (To, qxo, qyo) = second_sound_exact
    scale = 2.0 ** -20 if storage.startswith("f16") else 0.0
    T0 = W.initial_field(case)
    (dT, qx, qy), info = _run_rows(case, storage, scale, case.steps, rows, T0, rounding=rounding)
    e_t = _rel(dT, To - 1.0, To - 1.0)
    e_q = math.sqrt(float(np.sum((qx - qxo) ** 2 + (qy - qyo) ** 2))) / math.sqrt(float(np.sum(qxo ** 2 + qyo ** 2)))
    m_t = _max_rel([(dT, To - 1.0)])
    m_q = _max_rel([(qx, qxo), (qy, qyo)])
    exact_total = 0.01 * 2 * math.pi * 20.0 ** 2            # sum of the pulse over the plane
    log(f"second sound 8192^2 {storage} {rounding}: eps_T={e_t:.3e} eps_q={e_q:.3e} max_T={m_t:.3e} "
        f"max_q={m_q:.3e} total E={info['totals'][0]:.8f} (exact {exact_total:.8f}) r={info['residual']:.3e}")
    _assert_eps("second_sound", storage, rounding, e_t, e_q)
    assert m_t < MAXREL[storage] and m_q < MAXREL[storage]
    if storage == "f32":
        assert info["totals"][0] == pytest.approx(exact_total, rel=1e-6)


@pytest.mark.parametrize("storage", ["f32", "f16_split"])
def test_second_sound_front_speed_8192(storage):
    """Front of the 8192^2 pulse: ring radius (outermost maximum of dT along
    the centre row) at t = 150 ... 400, least-squares speed, against the same
    measurement on the exact solution.  Up to t = 400 nothing has travelled
    more than 400 nodes, so the exact solution on a 2048^2 lattice around the
    same pulse is the 8192^2 one near the centre.  The hydrodynamic second
    sound speed v_g / sqrt(3) (Sec. 3.4) is reported beside it: at tau_R = 50
    the ring is damped and lags it (a property of the scheme, pinned on the
    oracle side with tau_R = 1e5)."""
    case = W.second_sound_case()
    a = case.init_args
    times = list(range(150, 401, 50))
    scale = 2.0 ** -20 if storage.startswith("f16") else 0.0
    lat = Lattice([instance_from_case(case, scale)], storage=storage, check_interval=-1)
    lat.init(0, W.initial_field(case))
    gpu = []
    for t in times:
        lat.step(t - lat.steps)
        dT, _, _ = lat.moments_device(0)
        gpu.append(dT[a["cy"], a["cx"]:].cpu().numpy())
        del dT
    lat.close()
    torch.cuda.empty_cache()
    n = 2048
    x = np.arange(n, dtype=np.float64)
    f = np.exp(-(x - n // 2) ** 2 / (2 * a["sigma"] ** 2))
    ora = [bloch.SeparableSolution(f, f, a["amp"], t, case.tau_n, case.tau_r).rows([n // 2])[0][0, n // 2:] - 1.0
           for t in times]
    r_gpu = [front_radius(p) for p in gpu]
    r_ora = [front_radius(p) for p in ora]
    v_gpu = float(np.polyfit(times, r_gpu, 1)[0])
    v_ora = float(np.polyfit(times, r_ora, 1)[0])
    log(f"second sound 8192^2 {storage} front: speed {v_gpu:.5f} nodes/step (oracle {v_ora:.5f}; "
        f"hydrodynamic v_g/sqrt(3) = {cf.second_sound_speed():.5f}); radii gpu {np.round(r_gpu, 3).tolist()}")
    assert max(abs(p - q) for p, q in zip(r_gpu, r_ora)) < (1e-3 if storage == "f32" else 0.2)
    assert v_gpu == pytest.approx(v_ora, rel=1e-4 if storage == "f32" else 1e-2)


# ---------------------------------------------------------------- smooth modes

@pytest.mark.parametrize("storage,rounding", [("f16", "stochastic"), ("f32", "nearest"),
                                              ("f32", "stochastic"), ("bf16", "stochastic"),
                                              ("f16", "nearest"), ("bf16", "nearest")] + SPLIT_ROWS)
def test_smooth_modes_16384(storage, rounding):
    """16384^2 periodic, 16 seeded Fourier modes (total amplitude 1e-3),
    tau_N = 0.6, tau_R = 5, 1000 steps; FP16 with scale 2^-22."""
    case = W.smooth_modes_case()
    modes = case.init_args["modes"]
    # offsets 17 and 31 within the 32-row chunks
    rows = sorted(list(range(17, case.ny, 64)) + list(range(63, case.ny, 64)))
    sol = bloch.ModeSolution(modes, case.nx, case.ny, case.steps, case.tau_n, case.tau_r)
    To, qxo, qyo = sol.rows(rows)
    T0 = W.modes_field_torch(modes, case.nx, case.ny, case.t0, device="cuda")
    scale = 2.0 ** -22 if storage.startswith("f16") else 0.0
    (dT, qx, qy), info = _run_rows(case, storage, scale, case.steps, rows, T0, rounding=rounding)
    del T0
    torch.cuda.empty_cache()
    e_t = _rel(dT, To - 1.0, To - 1.0)
    e_q = math.sqrt(float(np.sum((qx - qxo) ** 2 + (qy - qyo) ** 2))) / math.sqrt(float(np.sum(qxo ** 2 + qyo ** 2)))
    m_t = _max_rel([(dT, To - 1.0)])
    m_q = _max_rel([(qx, qxo), (qy, qyo)])
    log(f"smooth modes 16384^2 {storage} {rounding}: eps_T={e_t:.3e} eps_q={e_q:.3e} max_T={m_t:.3e} "
        f"max_q={m_q:.3e} total E={info['totals'][0]:.3e}")
    _assert_eps("smooth_modes", storage, rounding, e_t, e_q)
    assert m_t < MAXREL[storage] and m_q < MAXREL[storage]


# ---------------------------------------------------------------- Poiseuille

def _oracle_steady(case):
    o = ref.Oracle(case)
    prev = None
    while o.steps < 200000:
        o.run(1000)
        _, qx, _ = o.moments()
        if prev is not None and np.abs(qx - prev).max() <= 1e-12 * np.abs(qx).max():
            break
        prev = qx.copy()
    return o.moments(), o.steps


@pytest.mark.parametrize("rounding", ["stochastic", "nearest"])
@pytest.mark.parametrize("ratio", W.POISEUILLE_RATIOS)
@pytest.mark.parametrize("tau_n", W.POISEUILLE_TAU_N)
def test_poiseuille_steady_1024x256(tau_n, ratio, rounding):
    """Channel 1024 x 256 (gradient seam G = 1e-3, diffuse walls) run to steady
    state on the GPU against the oracle's FP64 steady state, both roundings
    held to the FP32 bound 1e-5 (the reference state tracks the mean flux, so
    the stored values are the small departures from it even at tau_R / tau_N =
    1000).  Round to nearest: check every 1000 steps until r < 1e-10 or r = 0
    (the rounded map's fixed point).  Stochastic rounding keeps converging in
    expectation; the one-step residual then stays at the rounding-noise level,
    so it runs twice the steps the FP64 oracle needed."""
    case = W.poiseuille_case(tau_n, ratio)
    small = W.poiseuille_case(tau_n, ratio, nx=4)
    (To, qxo, qyo), osteps = _oracle_steady(small)
    lat = Lattice([instance_from_case(case)], check_interval=1000, rounding=rounding, seed=3)
    lat.set_schedule("graph")
    lat.init(0)
    r = 1.0
    budget = 200000 if rounding == "nearest" else 2 * osteps
    while lat.steps < budget:
        lat.step(1000)
        r = lat.residual(0)
        if r < 1e-10:
            break
    dT, qx, qy = lat.moments(0)
    steps = lat.steps
    lat.close()
    # the GPU solution is exactly uniform along x
    if rounding == "nearest":
        assert np.array_equal(qx, np.tile(qx[:, :1], (1, case.nx)))
    qx = qx.mean(axis=1, keepdims=True) if rounding == "stochastic" else qx
    qy = qy.mean(axis=1, keepdims=True) if rounding == "stochastic" else qy
    q_o = qxo[:, 0]
    e_q = float(np.linalg.norm(qx[:, 0] - q_o) / np.linalg.norm(q_o))
    e_qy = float(np.abs(qy[:, 0] - qyo[:, 0]).max() / np.abs(q_o).max())
    d = case.ny - 1
    kn_c = cf.knudsen(cf.scheme_constants(tau_n, case.tau_r)["tau_c"], d)
    kn_r = cf.knudsen(case.tau_r, d)
    Q = qx[:, 0] / cf.poiseuille_q_scale(case.tau_r, case.grad_x)
    cond = float(Q.mean())
    log(f"poiseuille tn={tau_n} ratio={ratio:g} {rounding}: gpu steps={steps} r={r:.2e} oracle steps={osteps} "
        f"eps_q={e_q:.3e} eps_qy={e_qy:.1e} lambda_eff/lambda={cond:.5f} (Eq.69 "
        f"{cf.poiseuille_conductivity_eq69(kn_c, kn_r):.5f})")
    assert e_q < 1e-5 and e_qy < 1e-5
    assert cond == pytest.approx(cf.poiseuille_conductivity_eq69(kn_c, kn_r), rel=0.01)


# ---------------------------------------------------------------- Knudsen sweep

@pytest.mark.parametrize("rounding", ["stochastic", "nearest"])
def test_knudsen_sweep_256_instances(rounding):
    """256 uneven channel instances in one handle, 2000 steps under each of the
    batched (on two streams, the default, and on one), per-instance and graph
    schedules: all agree bit for bit on the compared instances (from both
    parts of the two-stream split), and six of them match the oracle to the
    FP32 bound."""
    cases = W.knudsen_sweep()
    insts = [instance_from_case(c) for c in cases]
    steps = 2000
    picks = (0, 1, 2, 3, 4, 5, 200, 255)
    outs = {}
    for sched in ("graph", "batched", "batched_one_stream", "per_instance"):
        lat = Lattice(insts, check_interval=100, rounding=rounding, seed=7)
        lat.set_schedule("batched" if sched == "batched_one_stream" else sched)
        if sched == "batched_one_stream":
            lat.set_streams(1)
        for k in range(len(cases)):
            lat.init(k)
        lat.step(steps)
        outs[sched] = [lat.moments(k) for k in picks]
        lat.close()
    for sched in ("per_instance", "graph", "batched_one_stream"):
        for j, k in enumerate(picks):
            for a, b in zip(outs[sched][j], outs["batched"][j]):
                assert np.array_equal(a, b), (sched, k)
    worst = 0.0
    for j, k in enumerate(picks[:6]):
        case = cases[k]
        e_t, e_q = eps(case, outs["batched"][j], oracle_fields(case, steps))
        worst = max(worst, e_t, e_q)
        log(f"sweep {rounding} instance {k} {case.nx}x{case.ny} tau_n={case.tau_n:.3f} "
            f"tau_r={case.tau_r:.3g}: eps_T={e_t:.3e} eps_q={e_q:.3e}")
    assert worst < 1e-5
