"""Pins of the oracle's drag law (Eq. beta, C_D, Re_p) and DEM contact
(Sec. 2.2) against textbook forms written differently from the paper's."""
import math

import numpy as np
import pytest

from paper_2002_03120_amd import workloads as W

MU, RHO = 0.1, 1.0


def _drag_force(oracle_lib, eps, dv, d, rho=RHO):
    """Per-particle drag magnitude B V_s |dv| (B = beta/(1-eps))."""
    vs = math.pi * d ** 3 / 6.0
    return oracle_lib.drag_b(eps, dv, d, rho, MU) * vs * dv


# the fluid densities of the workloads: 1 and the slurry channel's 3 (Sec. 4.1),
# where a density dropped from Re_p or from the inertial terms shows
DENSITIES = [1.0, 3.0]


@pytest.mark.parametrize("d", [1.0, 3.0, 8.0])
def test_stokes_limit(oracle_lib, d):
    dv = 1e-9
    assert _drag_force(oracle_lib, 1.0, dv, d) == pytest.approx(3 * math.pi * MU * d * dv, rel=1e-6)


@pytest.mark.parametrize("rho", DENSITIES)
@pytest.mark.parametrize("re", [0.5, 10.0, 300.0, 999.0])
def test_single_sphere_drag_equation(oracle_lib, re, rho):
    # F = 1/2 C_D rho A v^2 with C_D = 24/Re (1 + 0.15 Re^0.687), A = pi d^2/4
    d = 2.0
    dv = re * MU / (rho * d)
    cd = 24.0 / re * (1.0 + 0.15 * re ** 0.687)
    expect = 0.5 * cd * rho * math.pi * d * d / 4.0 * dv * dv
    assert _drag_force(oracle_lib, 1.0, dv, d, rho) == pytest.approx(expect, rel=1e-12)


@pytest.mark.parametrize("rho", DENSITIES)
@pytest.mark.parametrize("eps", [0.81, 0.9, 1.0])
def test_newton_regime_with_voidage_factor(oracle_lib, eps, rho):
    # Re_p > 1000: C_D = 0.44 and the swarm factor eps^(-1.65) of Wen and Yu
    d = 2.0
    dv = 5000.0 * MU / (rho * d * eps)
    expect = 0.5 * 0.44 * rho * math.pi * d * d / 4.0 * dv * dv * eps ** -1.65
    assert _drag_force(oracle_lib, eps, dv, d, rho) == pytest.approx(expect, rel=1e-12)


@pytest.mark.parametrize("rho", DENSITIES)
@pytest.mark.parametrize("eps", [0.35, 0.5, 0.8])
@pytest.mark.parametrize("dv", [1e-3, 0.2, 3.0])
def test_ergun_pressure_drop(oracle_lib, eps, dv, rho):
    # dense branch: the interphase force per bed volume beta |dv| balances
    # eps times the Ergun pressure gradient at superficial velocity eps |dv|
    d = 1.5
    U = eps * dv
    dpdl = (150.0 * MU * (1 - eps) ** 2 * U / (eps ** 3 * d * d)
            + 1.75 * rho * (1 - eps) * U * U / (eps ** 3 * d))
    beta = oracle_lib.drag_b(eps, dv, d, rho, MU) * (1.0 - eps)
    assert beta * dv == pytest.approx(eps * dpdl, rel=1e-12)


def _dem_params(**over):
    p = W.base_params(E_dem=7881.0, nu_dem=0.3, mu_fric=0.3, dt=1e-3)
    p.update(over)
    return p


def test_hertz_stiffness_via_contact_time(oracle_lib):
    """Undamped head-on contact: duration pi sqrt(m*/K), elastic rebound,
    with K = (4/3) E* sqrt(R*), E* = E / (2 (1 - nu^2)), R* = R/2."""
    E, nu, R, m = 7881.0, 0.3, 1.5, 35.0
    p = _dem_params(dem_damping=0.0)
    K = 4.0 / 3.0 * (E / (2 * (1 - nu * nu))) * math.sqrt(R / 2.0)
    mstar = m / 2.0
    z3 = np.zeros(3)
    # integrate the relative coordinate with velocity Verlet in the test
    dt = 2e-5
    x, v = 2 * R, -0.05  # centre distance and its rate
    t, t_in, t_out = 0.0, None, None
    f = 0.0
    while t < 5.0:
        v += 0.5 * dt * f / mstar
        x += dt * v
        t += dt
        if x < 2 * R:
            if t_in is None:
                t_in = t
            fn = oracle_lib.dem_pair(p, [x, 0, 0], [v, 0, 0], z3, z3, z3, R, R, m, m, z3)[0]
            f = fn[0]  # force on i along +x; relative coordinate x = x_i - x_j
        else:
            f = 0.0
            if t_in is not None:
                t_out = t
                break
        v += 0.5 * dt * f / mstar
    assert t_out is not None
    assert (t_out - t_in) == pytest.approx(math.pi * math.sqrt(mstar / K), rel=2e-3)
    assert v == pytest.approx(0.05, rel=2e-3)


def test_damped_contact_dissipates(oracle_lib):
    p = _dem_params()
    z3 = np.zeros(3)
    fn0 = oracle_lib.dem_pair(dict(p, dem_damping=0.0), [2.9, 0, 0], [-0.1, 0, 0], z3, z3, z3,
                              1.5, 1.5, 35.0, 35.0, z3)[0]
    fn1 = oracle_lib.dem_pair(p, [2.9, 0, 0], [-0.1, 0, 0], z3, z3, z3, 1.5, 1.5, 35.0, 35.0, z3)[0]
    # approaching pair: the dashpot adds repulsion
    assert fn1[0] > fn0[0] > 0


def test_coulomb_slider(oracle_lib):
    p = _dem_params()
    z3 = np.zeros(3)
    d = [2.95, 0.0, 0.0]
    for vt in (1e-4, 1e-2, 1.0):
        fn, ft, dto, sl = oracle_lib.dem_pair(p, d, [0, vt, 0], z3, z3, z3, 1.5, 1.5, 35.0, 35.0, z3)
        if sl:
            assert np.linalg.norm(ft) == pytest.approx(p["mu_fric"] * np.linalg.norm(fn), rel=1e-14)
        else:
            assert np.linalg.norm(ft) < p["mu_fric"] * np.linalg.norm(fn)
        # friction opposes the tangential slip
        assert ft[1] < 0 and abs(ft[0]) < 1e-12 * np.linalg.norm(ft)
    # fast slip must slide
    assert oracle_lib.dem_pair(p, d, [0, 1.0, 0], z3, z3, z3, 1.5, 1.5, 35.0, 35.0, z3)[3]


def test_stick_history_integrates_slip(oracle_lib):
    # while sticking, Eq. tandispn accumulates v_t dt along a fixed direction
    p = _dem_params(dt=1e-3)
    z3 = np.zeros(3)
    d = [2.9, 0.0, 0.0]
    vt = 1e-5
    dt_ = np.zeros(3)
    for k in range(20):
        fn, ft, dt_, sl = oracle_lib.dem_pair(p, d, [0, 0, vt], z3, z3, z3, 1.5, 1.5, 35.0, 35.0, dt_)
        assert not sl
    assert dt_ == pytest.approx([0.0, 0.0, 20 * vt * 1e-3], rel=1e-12, abs=1e-20)


def test_spin_enters_tangential_velocity(oracle_lib):
    # rolling without slip: R_i w_i + R_j w_j cancels the tangential velocity
    p = _dem_params()
    z3 = np.zeros(3)
    R = 1.5
    d = np.array([2.95, 0.0, 0.0])
    n = d / np.linalg.norm(d)
    v_rel = np.array([0.0, 0.3, 0.0])
    # (R w_i + R w_j) x n = -v_t  ->  choose w along z
    w = np.array([0.0, 0.0, -0.3 / (2 * R)])
    rot = np.cross(2 * R * w, n)
    assert np.allclose(v_rel + rot, 0.0)
    fn, ft, dto, sl = oracle_lib.dem_pair(p, d, v_rel, z3, w, w, R, R, 35.0, 35.0, z3)
    assert np.linalg.norm(ft) < 1e-12


def test_dem_pair_antisymmetric(oracle_lib):
    p = _dem_params()
    rng = np.random.default_rng(0)
    for k in range(50):
        d = rng.standard_normal(3)
        d *= 2.9 / np.linalg.norm(d)
        vi, vj, wi, wj, dt0 = (rng.standard_normal(3) * 0.01 for _ in range(5))
        a = oracle_lib.dem_pair(p, d, vi, vj, wi, wj, 1.5, 1.5, 35.0, 35.0, dt0)
        b = oracle_lib.dem_pair(p, -d, vj, vi, wj, wi, 1.5, 1.5, 35.0, 35.0, -dt0)
        assert np.allclose(a[0], -b[0], rtol=1e-13, atol=1e-15)
        assert np.allclose(a[1], -b[1], rtol=1e-13, atol=1e-15)
        assert np.allclose(a[2], -b[2], rtol=1e-13, atol=1e-18)
        assert a[3] == b[3]
