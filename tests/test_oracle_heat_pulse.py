"""Heat-flux boundary (Eqs. 56-57) and the transient heat pulse of Sec. 3.4.

First the analytical route of Appendix B (Laplace transform of the
hydrodynamic model, Eqs. 72-80, inverted by the Riemann sum of Eqs. B14-B15)
is pinned on its own: boundary values, the energy balance, the diffusive
limit against a cosine-series solution, and the second-sound front.  Then the
FP64 stepper with the heat-flux wall is pinned: the wall identity of Eq. 56,
the terminal temperature rise the paper prints (0.129), the arrival speed
v_g/sqrt(3), and agreement with the hydrodynamic model that improves under
grid refinement in the wave regimes.

The Riemann sum is used with gamma t* = 6 rather than the paper's 3: its
aliasing error is about exp(-2 gamma t*) of the late-time signal, 2.5e-3 at
3, which would mask the stepper's 4e-4 agreement in the diffusive regime
(results at gamma t* = 6 and 8 agree to 1e-5).  20k terms leave a truncation
error of about 2e-4 of the largest Theta.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import closed_forms as cf, ref

KN_N = W.HEAT_PULSE_KN_N
GT = 6.0
TERMS = 20000


@pytest.fixture(autouse=True, scope="module")
def _threads():
    ref.set_threads(min(8, max(1, ref.max_threads())))


def _pulse_case(kn_r, nodes=401):
    tn, tr = cf.lattice_relaxation_times(nodes - 1, KN_N, kn_r)
    return W.heat_pulse_case(tn, tr, nodes=nodes), round(100.0 * tn)


def _theta(o, case):
    T, qx, _ = o.moments()
    q0 = case.q_wall[0]
    return (T[1] - case.t0) * cf.VG / q0, qx[1] / q0


def _run_pulse(case, pulse, stops):
    """Oracle through the pulse (flux on for `pulse` steps, then off), with
    (Theta, Q) of row 1 at each step count in `stops`."""
    o = ref.Oracle(case)
    out = []
    for n in stops:
        if o.steps < pulse <= n:
            o.run(pulse - o.steps)
            o.set_wall_flux(0, 0.0)
        o.run(n - o.steps)
        out.append(_theta(o, case))
    return o, out


# ---------------------------------------------------------------- Appendix B route

@pytest.mark.parametrize("kn_r", W.HEAT_PULSE_KN_R)
def test_laplace_route_boundary_and_energy(kn_r):
    """Q(0, t*) is the pulse of Eq. 80, Q(1, t*) = 0, and the energy balance
    (Eq. 77 integrated over the plate) gives int Theta dX = Kn_N min(t*, 100).
    Points cluster at X = 0, where the diffusive profile is thin early on."""
    X = np.linspace(0.0, 1.0, 601) ** 2
    for ts, q_left in ((40.0, 1.0), (260.0, 0.0), (900.0, 0.0)):
        th, Q = cf.heat_pulse_solution(X, ts, KN_N, kn_r, gamma_t=GT, n_terms=TERMS)
        assert Q[0] == pytest.approx(q_left, abs=2e-3)
        assert Q[-1] == pytest.approx(0.0, abs=2e-3)
        integral = float(np.sum((th[1:] + th[:-1]) / 2.0 * np.diff(X)))
        assert integral == pytest.approx(KN_N * min(ts, 100.0), rel=2e-3)


def test_laplace_route_diffusive_limit():
    """With Kn_R << Kn_N the model is the heat equation with diffusivity
    Kn_N Kn_R / 3: the inverted transform equals its cosine-series solution
    (interior points; on X = 0 the sum converges more slowly)."""
    kn_n, kn_r = 1e-2, 1e-4
    X = np.linspace(0.005, 0.4, 80)
    for ts in (3e3, 3e4, 2e5):
        th, _ = cf.heat_pulse_solution(X, ts, kn_n, kn_r, gamma_t=GT, n_terms=TERMS)
        ser = cf.heat_pulse_diffusive_limit(X, ts, kn_n, kn_r)
        assert np.max(np.abs(th - ser)) < 2e-3 * np.max(np.abs(ser)), ts


def test_laplace_route_second_sound_front():
    """Dominant normal scattering: the leading edge (half height of the
    first plateau) travels at v_g/sqrt(3), i.e. Kn_N/sqrt(3) in X per t*."""
    X = np.linspace(0.0, 1.0, 1001)
    for ts in (300.0, 600.0):
        th, _ = cf.heat_pulse_solution(X, ts, KN_N, 1.29e3, gamma_t=GT, n_terms=TERMS)
        peak = th.max()
        front = X[np.nonzero(th > 0.5 * peak)[0][-1]]
        assert front == pytest.approx(KN_N / math.sqrt(3.0) * ts, rel=0.02), ts


# ---------------------------------------------------------------- stepper

@pytest.mark.parametrize("kn_r", W.HEAT_PULSE_KN_R)
def test_heatflux_wall_identity(kn_r):
    """Eq. 57 makes Eq. 56 hold exactly: during the pulse the heat flux at the
    wall node is q0, afterwards 0 (adiabatic), at every step."""
    case, pulse = _pulse_case(kn_r, nodes=41)
    o = ref.Oracle(case)
    for n in range(1, 2 * pulse + 5):
        if n == pulse + 1:
            o.set_wall_flux(0, 0.0)
        o.run(1)
        _, qx, _ = o.moments()
        want = case.q_wall[0] if n <= pulse else 0.0
        assert np.allclose(qx[:, 0], want, rtol=1e-12, atol=1e-15)
        assert np.allclose(qx[:, -1], 0.0, atol=1e-15)


def test_heatflux_wall_on_y_axis():
    """The same identity on walls across y (q0 into the domain at y = 0 is
    +y, at y = ny - 1 it is -y), with periodic x."""
    case = W.Case("hf_y", 17, 12, 0.7, 3.0, bc_x="periodic", bc_y="heatflux", q_wall=(0, 0, 2e-3, 5e-4))
    o = ref.Oracle(case)
    for _ in range(7):
        o.run(1)
        _, _, qy = o.moments()
        assert np.allclose(qy[0], 2e-3, rtol=1e-12)
        assert np.allclose(qy[-1], -5e-4, rtol=1e-12)


def test_heat_pulse_terminal_rise():
    """Diffusive regime (Kn_R = Kn_N = 1.29e-3): the temperature of the whole
    plate, and of its far face, approaches the terminal rise Theta = Kn_N t_p*
    = 0.129 (energy input over heat capacity, Sec. 3.4).  101 nodes keep the
    diffusion time short (d^2 / alpha ~ 2e5 steps); 100k steps leave the far
    face within 1%."""
    case, pulse = _pulse_case(1.29e-3, nodes=101)
    tn = case.tau_n
    o, [(th, _)] = _run_pulse(case, pulse, [100000])
    rise = KN_N * pulse / tn
    assert rise == pytest.approx(0.129, abs=1e-3)
    assert th.mean() == pytest.approx(rise, rel=1e-4)
    assert th[-1] == pytest.approx(rise, rel=1e-2)


def test_heat_pulse_arrival_speed():
    """Second-sound regime (Kn_R = 1.29e3) on the 401-node plate: the far face
    receives the leading edge (half of its first plateau) after d / (v_g /
    sqrt(3)) steps, within 1%."""
    case, pulse = _pulse_case(1.29e3)
    o = ref.Oracle(case)
    d = case.nx - 1
    far = []
    while o.steps < 700:
        if o.steps == pulse:
            o.set_wall_flux(0, 0.0)
        o.run(1)
        far.append(_theta(o, case)[0][-1])
    far = np.array(far)
    first = far[: int(d / cf.second_sound_speed()) + pulse]
    half = 0.5 * first.max()
    k = int(np.nonzero(first > half)[0][0])
    t_cross = k + (half - first[k - 1]) / (first[k] - first[k - 1])    # steps 1..; index k is step k+1
    speed = d / (t_cross + 1.0)
    assert speed == pytest.approx(cf.second_sound_speed(), rel=1e-2)


@pytest.mark.parametrize("kn_r", W.HEAT_PULSE_KN_R)
def test_heat_pulse_matches_hydrodynamic_model(kn_r):
    """401-node plate against the Appendix B solution at t* = 250, 700, 1250:
    relative L2 of Theta within 3% with a travelling front (the LBM smears the
    pulse edges over a few nodes) and 0.2% in the diffusive regime (where at
    t* = 250 the heated layer is still only ~10 nodes thick; 4e-4 later); in
    the wave regimes the gap at least halves on the 801-node plate (same Kn)."""
    errs = {}
    for nodes in (401, 801):
        case, pulse = _pulse_case(kn_r, nodes)
        X = np.arange(nodes) / (nodes - 1)
        stops = [round(ts * case.tau_n) for ts in (250.0, 700.0, 1250.0)]
        _, fields = _run_pulse(case, pulse, stops)
        e = []
        for n, (th, _) in zip(stops, fields):
            ref_th, _ = cf.heat_pulse_solution(X, n / case.tau_n, KN_N, kn_r, t_pulse=pulse / case.tau_n,
                                               gamma_t=GT, n_terms=TERMS)
            e.append(float(np.linalg.norm(th - ref_th) / np.linalg.norm(ref_th)))
        errs[nodes] = e
        if kn_r < 1.0:
            break
    if kn_r < 1.0:
        assert max(errs[401]) < 2e-3
    else:
        assert max(errs[401]) < 3e-2
        assert all(b < 0.5 * a for a, b in zip(errs[401], errs[801])), errs
