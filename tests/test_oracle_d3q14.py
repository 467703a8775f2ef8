"""Pins of the D3Q14 oracle against what the paper and the mathematics fix.

The paper gives the scheme on D2Q8 and only names D3Q14 as a direct extension
(Sec. 2.2).  The 3D oracle keeps Eqs. 13, 15-16, 19/54 and 48-49 and takes
the weights that make the moment identities of Sec. 2.3 (Eqs. 22-28) hold on
the 14 velocities.  These tests pin it from four independent sides:

* the moment identities themselves, on the C stepper's relaxation;
* exact agreement with the 2D oracle (already pinned to the paper) for fields
  that vary along one axis only, where both lattices reduce to the same three
  groups of movers (c_a = +1, 0, -1) with equal group weights;
* the Fourier-mode matrix power (weights solved there from the moment
  conditions, not typed in), which must equal the stepper to rounding;
* the continuum limit Eq. 52 of the Bloch eigenvalues in every direction.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import bloch_d3q14 as b3, closed_forms as cf, ref
from measure import front_radius

# the D3Q14 velocity set (axis movers, then corner movers), as the lattice defines it
AXIS = [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
CORNER = [(sx, sy, sz) for sz in (1, -1) for sy in (1, -1) for sx in (1, -1)]
CV = np.array(AXIS + CORNER, dtype=np.float64)
CX, CY, CZ = CV[:, 0], CV[:, 1], CV[:, 2]

REGIMES = [(0.6, 0.8), (0.55, 50.0), (0.7, 3.0), (2.3, 0.2), (0.51, math.inf), (1.0, 1000.0)]


def _collision_matrix(tau_n, tau_r):
    return np.stack([ref.collide_node_3d(tau_n, tau_r, np.eye(14)[j]) for j in range(14)], axis=1)


# ---------------------------------------------------------------- single node

@pytest.mark.parametrize("tau_n,tau_r", REGIMES)
def test_collision_moments(tau_n, tau_r):
    """One relaxation step moves each velocity moment as Eqs. 22-28 and 54
    fix: energy kept; first moments scaled by rho; diagonal second moments
    relaxed toward (5/9) C_V T at rate 1/tau, off-diagonal ones toward 0;
    third moments c_a^3 and c_a c_b^2 toward q_a and q_a/3 (Eq. 25) with the
    source's share, c_x c_y c_z toward 0."""
    p = cf.scheme_constants(tau_n, tau_r)
    tau, rho, beta = p["tau"], p["rho"], p["beta"]
    kappa = 1.0 / tau - (0.0 if math.isinf(tau_r) else (1.0 - 0.5 / tau) / tau_r)
    rng = np.random.default_rng(17)
    cv = 1.7
    for _ in range(20):
        e = rng.uniform(-1, 1, 14) + 0.3
        s = ref.collide_node_3d(tau_n, tau_r, e, cv=cv)
        E = e.sum()
        j = [CX @ e, CY @ e, CZ @ e]
        assert s.sum() == pytest.approx(E, abs=1e-14)
        for a, ca in enumerate((CX, CY, CZ)):
            assert ca @ s == pytest.approx(rho * j[a], abs=1e-14)
        for a, ca in enumerate((CX, CY, CZ)):
            for bb, cb in enumerate((CX, CY, CZ)):
                m, ms = (ca * cb) @ e, (ca * cb) @ s
                target = (5.0 / 9.0) * E if a == bb else 0.0
                assert ms == pytest.approx((1 - 1 / tau) * m + target / tau, abs=1e-14)
        for a, ca in enumerate((CX, CY, CZ)):
            m, ms = (ca ** 3) @ e, (ca ** 3) @ s
            assert ms == pytest.approx((1 - 1 / tau) * m + kappa * beta * j[a], abs=1e-14)
            for cb in (CX, CY, CZ):
                if cb is ca:
                    continue
                m, ms = (ca * cb * cb) @ e, (ca * cb * cb) @ s
                assert ms == pytest.approx((1 - 1 / tau) * m + kappa * beta * j[a] / 3.0, abs=1e-14)
        m, ms = (CX * CY * CZ) @ e, (CX * CY * CZ) @ s
        assert ms == pytest.approx((1 - 1 / tau) * m, abs=1e-14)


@pytest.mark.parametrize("tau_n,tau_r", REGIMES)
def test_collision_eigenvalues(tau_n, tau_r):
    """Eigenvalues of the relaxation: 1 (energy), rho three times (heat flux),
    1 - 1/tau for the ten non-conserved moments."""
    p = cf.scheme_constants(tau_n, tau_r)
    lam = np.sort_complex(np.linalg.eigvals(_collision_matrix(tau_n, tau_r)))
    want = np.sort_complex(np.array([1.0] + [p["rho"]] * 3 + [1 - 1 / p["tau"]] * 10, dtype=complex))
    assert np.allclose(lam, want, atol=1e-10)


def test_uniform_equilibrium_is_fixed_point():
    """e_i = omega_i C_V T with zero flux relaxes to itself (weights sum to 1);
    the weights are read back from the stepper's relaxation of single-direction
    states and equal the ones solved from the moment conditions."""
    tau = cf.scheme_constants(0.6, 0.8)["tau"]
    M = _collision_matrix(0.6, 0.8)
    # symmetric part over a +/- pair removes the flux term; what remains off
    # the diagonal is omega_i / tau
    om = np.array([(M[i, 0] + M[i, 1]) / 2.0 * tau for i in range(14)])
    om[0] -= (1 - 1 / tau) * tau / 2.0
    om[1] -= (1 - 1 / tau) * tau / 2.0
    assert np.allclose(om, b3.OMEGA3, atol=1e-13)
    e = b3.OMEGA3 * 2.0 * 1.3
    assert np.allclose(ref.collide_node_3d(0.6, 0.8, e, cv=2.0), e, atol=1e-15)


def test_weights_closed_form():
    """The moment conditions have the unique solution omega = 1/9, 1/24 and
    a = 1/5, 1/40 (axis, corner); on D2Q8 the same conditions give the paper's
    Eqs. 17-18 (2/9, 1/36 and 1/5, 1/20), which the 2D stepper uses."""
    assert np.allclose(b3.OMEGA3[:6], 1 / 9, atol=1e-15) and np.allclose(b3.OMEGA3[6:], 1 / 24, atol=1e-15)
    assert np.allclose(b3.A3[:6], 1 / 5, atol=1e-15) and np.allclose(b3.A3[6:], 1 / 40, atol=1e-15)
    # the same solve on the D2Q8 velocities
    c2 = np.array([[1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]], float)
    ax = np.abs(c2).sum(1) == 1

    def cls(v):
        return [v[ax].sum(), v[~ax].sum()]

    A = np.array([cls(np.ones(8)), cls(c2[:, 0] ** 2)])
    w = np.linalg.solve(A, [1.0, 5 / 9])
    B = np.array([cls(c2[:, 0] ** 2), cls(c2[:, 0] ** 2 * c2[:, 1] ** 2)])
    a = np.linalg.solve(B, [0.6, 0.2])
    assert np.allclose(w, [2 / 9, 1 / 36], atol=1e-15) and np.allclose(a, [1 / 5, 1 / 20], atol=1e-15)


# ---------------------------------------------------------------- advection

def test_advection_direction():
    """With tau_N = tau_R huge the relaxation is the identity to 1e-12, so one
    step moves a lone population e_i by c_i, with periodic wrap."""
    nx, ny, nz = 7, 6, 5
    for i in range(14):
        o = ref.Oracle3D(nx, ny, nz, 1e12, 1e12, t0=0.0)
        pops = o.populations()
        pops[...] = 0.0
        x0, y0, z0 = 6, 0, 2           # on the x and y seams
        pops[i, z0, y0, x0] = 1.0
        o.run(1)
        pops = o.populations()
        x1, y1, z1 = (x0 + int(CX[i])) % nx, (y0 + int(CY[i])) % ny, (z0 + int(CZ[i])) % nz
        assert pops[i, z1, y1, x1] == pytest.approx(1.0, abs=1e-11)
        pops[i, z1, y1, x1] = 0.0
        assert np.abs(pops).max() < 1e-11


# ---------------------------------------------------------------- periodic box

@pytest.mark.parametrize("tau_n,tau_r", REGIMES)
def test_stepper_matches_bloch(tau_n, tau_r):
    """The C stepper equals the Fourier-mode matrix power on a non-cubic box
    from a random non-equilibrium state."""
    nx, ny, nz, n = 10, 8, 6, 23
    T0 = W.random_field_3d(nx, ny, nz, 0.01, 1.0, 1)
    q = W.random_flux_3d(nx, ny, nz, 1e-3, 2)
    o = ref.Oracle3D(nx, ny, nz, tau_n, tau_r, T0, q)
    rng = np.random.default_rng(3)
    o.populations()[...] += 1e-3 * rng.standard_normal((14, nz, ny, nx))
    e0 = o.populations().copy()
    o.run(n)
    eb = b3.evolve_populations(e0, n, tau_n, tau_r)
    assert np.abs(o.populations() - eb).max() < 1e-13


@pytest.mark.parametrize("tau_n,tau_r", REGIMES)
def test_periodic_invariants(tau_n, tau_r):
    """Total energy is constant and the total heat flux is multiplied by
    rho = (2 tau_r - 1)/(2 tau_r + 1) per step."""
    nx, ny, nz, n = 9, 7, 5, 30
    o = ref.Oracle3D(nx, ny, nz, tau_n, tau_r, W.random_field_3d(nx, ny, nz, 0.05, 1.0, 11),
                     W.random_flux_3d(nx, ny, nz, 0.01, 12))
    a = o.totals()
    o.run(n)
    bt = o.totals()
    rho = cf.scheme_constants(tau_n, tau_r)["rho"]
    # the energy total is a difference of two sums of size C_V t0 nodes (315):
    # rounding allows about 1e-13 of that magnitude
    assert bt[0] == pytest.approx(a[0], abs=1e-13 * nx * ny * nz)
    for k in (1, 2, 3):
        assert bt[k] == pytest.approx(a[k] * rho ** n, abs=1e-12)


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("tau_n,tau_r", [(0.6, 0.8), (0.55, 50.0), (2.3, 0.2)])
def test_one_dimensional_fields_match_d2q8(axis, tau_n, tau_r):
    """A field that varies along one axis only evolves exactly as on the D2Q8
    lattice: both lattices split into movers with c_a = +1, 0, -1 whose summed
    weights agree (omega 5/18, 4/9, 5/18; a 3/10, 0, 3/10), so the grouped
    dynamics are the same.  Compared against the 2D stepper on an x-varying
    field, for each of the three axes of the 3D box."""
    L, n = 23, 60
    rng = np.random.Generator(np.random.PCG64(5))
    T1 = 1.0 + 0.02 * rng.uniform(-1, 1, L)
    q1 = 0.003 * rng.uniform(-1, 1, L)
    # 2D reference: x-varying, periodic, 3 rows
    case2 = W.Case("line", L, 3, tau_n, tau_r)
    o2 = ref.Oracle(case2, np.tile(T1, (3, 1)), np.tile(q1, (3, 1)), np.zeros((3, L)))
    o2.run(n)
    T2, qx2, qy2 = o2.moments()
    # 3D: the same profile along `axis`, 3 x 4 across
    dims = [4, 3, 5]                       # nx, ny, nz before placing L
    dims[axis] = L
    nx, ny, nz = dims
    shape = (nz, ny, nx)
    bshape = [1, 1, 1]
    bshape[2 - axis] = L
    T3 = np.broadcast_to(T1.reshape(bshape), shape)
    q3 = [np.zeros(shape)] * 3
    q3[axis] = np.broadcast_to(q1.reshape(bshape), shape)
    o3 = ref.Oracle3D(nx, ny, nz, tau_n, tau_r, T3, q3)
    o3.run(n)
    m = o3.moments()
    line = [slice(0, 1)] * 3
    line[2 - axis] = slice(None)
    Tl = m[0][tuple(line)].ravel()
    ql = m[1 + axis][tuple(line)].ravel()
    assert np.abs(Tl - T2[0]).max() < 1e-13
    assert np.abs(ql - qx2[0]).max() < 1e-14
    # uniform across, no transverse flux
    assert np.ptp(m[0], axis=tuple(a for a in range(3) if a != 2 - axis)).max() < 1e-13
    for k in range(3):
        if k != axis:
            assert np.abs(m[1 + k]).max() < 1e-14


@pytest.mark.parametrize("tau_n,tau_r", [(0.55, 50.0), (0.6, 5.0), (0.8, 0.8), (0.51, 1000.0)])
def test_bloch_dispersion_is_eq52(tau_n, tau_r):
    """Slow Bloch eigenvalues reproduce the temperature equation Eq. 52 for
    long waves along an axis, a face diagonal, the body diagonal and a
    generic direction (the lattice is isotropic to this order)."""
    tau_c = cf.scheme_constants(tau_n, tau_r)["tau_c"]
    dirs = [(1, 0, 0), (0, 1, 1), (1, 1, 1), (0.3, -0.5, 0.81)]
    for k in (0.01, 0.02, 0.04):
        want = [w for w in cf.telegraph_rates(k, tau_r, tau_c) if abs(w) < 0.1]
        assert want
        for d in dirs:
            u = np.array(d, dtype=np.float64) / np.linalg.norm(d)
            s = np.log(b3.slow_eigenvalues(k * u, tau_n, tau_r, count=3))
            for w in want:
                err = np.min(np.abs(s - w)) / abs(w)
                assert err < 5e-3, (k, d, s, want)


def test_mode_solution_equals_stepper():
    """The per-mode evaluation used at full size equals the stepper on a box
    small enough for it."""
    nx, ny, nz, n = 16, 12, 10, 31
    modes = [W.Mode3(1, 2, -1, 3e-4, 0.3), W.Mode3(-3, 1, 2, 2e-4, 1.9), W.Mode3(0, 0, 4, 1e-4, 4.0)]
    T0 = W.modes_field_3d(modes, nx, ny, nz, 1.0)
    o = ref.Oracle3D(nx, ny, nz, 0.6, 5.0, T0)
    o.run(n)
    T, qx, qy, qz = o.moments()
    sol = b3.ModeSolution(modes, nx, ny, nz, n, 0.6, 5.0)
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    Ts, qxs, qys, qzs = sol.at(xx, yy, zz)
    assert np.abs(Ts - T).max() < 1e-15 + 1e-12
    for a, bb in ((qxs, qx), (qys, qy), (qzs, qz)):
        assert np.abs(a - bb).max() < 1e-15


def test_second_sound_front_3d():
    """With dominant normal scattering a pulse spreads as a spherical front at
    v_g / sqrt(3) (Sec. 3.4: sqrt(5)/3 nodes per step), along an axis and along
    the body diagonal alike.  For a spherical wave the peak of T sits about one
    pulse width ahead of v t, and the width grows as the damping term
    of Eq. 52 spreads the pulse (variance sigma^2 + (4/15) tau_C v_g^2 t); that
    width is subtracted before the slope is fitted."""
    c = W.second_sound_3d_case(n=96, sigma=3.0, tau_n=0.55, tau_r=1e5)
    o = ref.Oracle3D(c.nx, c.ny, c.nz, c.tau_n, c.tau_r, W.initial_field_3d(c))
    h = c.nz // 2
    tau_c = cf.scheme_constants(c.tau_n, c.tau_r)["tau_c"]
    ts, r_axis, r_diag = np.arange(12, 49, 6), [], []
    done = 0
    for t in ts:
        o.run(int(t) - done)
        done = int(t)
        T = o.moments()[0] - 1.0
        width = math.sqrt(3.0 ** 2 + (4.0 / 15.0) * tau_c * cf.VG ** 2 * t)
        r_axis.append(front_radius(T[h, h, h:]) - width)
        r_diag.append(front_radius(np.array([T[h + k, h + k, h + k] for k in range(h)])) * math.sqrt(3.0)
                      - width)
    v = cf.second_sound_speed()
    assert np.polyfit(ts, r_axis, 1)[0] == pytest.approx(v, rel=0.025)
    assert np.polyfit(ts, r_diag, 1)[0] == pytest.approx(v, rel=0.025)
