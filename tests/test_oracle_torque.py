"""Pins of the oracle's torques (Sec. 2.6) and of the size of the lubrication
force (Eq. lubri, Sec. 2.3).

Torques.  Eq. newton2 turns each particle by its own lever: half the initial
spacing dx for fluid particles, the radius R for rigid ones, along -e_ij
(reading R8).  For an isolated pair the rate of change of the total angular
momentum is then r_ij x F_ij + N_i + N_j, which these tests check against
its closed form: zero for fluid particles exactly dx apart (the two levers
then span the pair), (1 - dx/|r|) r_ij x F_ij at any other separation, and
(L - R_i - R_j) n x F_t for two spheres in contact (Sec. 2.2).  A flipped
lever, or Mueller's lever |r_ij|/2, fails them.

Lubrication.  For two equal spheres approaching head-on, Reynolds' squeeze
film between spheres gives 6 pi mu R*^2 u / gap with the reduced radius
R* = R_i R_j / (R_i + R_j) -- a different expression, which equals the
paper's 3 pi mu d^2 u / (8 gap) exactly when d is the mean diameter
R_i + R_j.  A radius in place of the diameter, or a factor 2, fails it.
"""
import math

import numpy as np
import pytest

from paper_2002_03120_amd import workloads as W

RHO0, DX = 3.0, 0.5
MF = RHO0 * DX ** 3


def _params(**over):
    p = W.base_params(L=[6.0, 6.0, 6.0], periodic=[1, 1, 1], dx=DX, h=2 * DX, rho0=RHO0,
                      mass_fluid=MF, inertia_fluid=0.1 * MF * DX ** 2, eta=2.0,
                      xi=2.0 * 20 / 21, kBT=1e-3, dt=1e-3, p0=1.0, beta_eos=1.0)
    p.update(over)
    return p


def _two(types, pos, vel, spin, radius=(0.0, 0.0), mass=(MF, MF), inertia=None):
    inertia = inertia or tuple(0.1 * m * DX ** 2 for m in mass)
    return dict(id=np.array([0, 1]), type=np.array(types, np.uint8),
                pos=np.array(pos, float), vel=np.array(vel, float),
                angvel=np.array(spin, float), mass=np.array(mass, float),
                inertia=np.array(inertia, float), radius=np.array(radius, float))


def _unit(rng):
    e = rng.standard_normal(3)
    return e / np.linalg.norm(e)


@pytest.mark.parametrize("sep_over_dx", [1.0, 1.6, 0.7])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_fluid_pair_torques(oracle_lib, sep_over_dx, seed):
    rng = np.random.default_rng(seed)
    c = np.array([3.0, 3.0, 3.0])
    r = sep_over_dx * DX * _unit(rng)
    parts = _two([W.FLUID, W.FLUID], [c + r / 2, c - r / 2],
                 rng.standard_normal((2, 3)) * 0.3, rng.standard_normal((2, 3)) * 0.5)
    o = oracle_lib.Oracle(_params(), parts)
    o.compute_forces()
    F, N = o.read_field("F_SDPD"), o.read_field("N_SDPD")
    assert np.array_equal(F[1], -F[0])
    tq = np.cross(r, F[0])
    assert np.linalg.norm(tq) > 1e-3 * np.linalg.norm(r) * np.linalg.norm(F[0])
    rate = tq + N[0] + N[1]  # d/dt of the pair's total angular momentum
    expect = (1.0 - DX / np.linalg.norm(r)) * tq
    scale = np.linalg.norm(r) * np.linalg.norm(F[0])
    assert np.allclose(rate, expect, atol=1e-13 * scale, rtol=0)
    if sep_over_dx == 1.0:
        assert np.linalg.norm(rate) < 1e-13 * scale


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_dem_pair_torques(oracle_lib, seed):
    rng = np.random.default_rng(seed)
    Ri, Rj = 0.75, 0.45
    n = _unit(rng)
    Lc = (Ri + Rj) * 0.95  # overlapping
    c = np.array([3.0, 3.0, 3.0])
    vi, vj = rng.standard_normal(3) * 0.2, rng.standard_normal(3) * 0.2
    wi, wj = rng.standard_normal(3) * 0.3, rng.standard_normal(3) * 0.3
    mi, mj = 2.5 * RHO0 * 4 / 3 * math.pi * Ri ** 3, 2.5 * RHO0 * 4 / 3 * math.pi * Rj ** 3
    parts = _two([W.RIGID, W.RIGID], [c + Lc * n / 2, c - Lc * n / 2], [vi, vj], [wi, wj],
                 radius=(Ri, Rj), mass=(mi, mj),
                 inertia=(0.4 * mi * Ri * Ri, 0.4 * mj * Rj * Rj))
    o = oracle_lib.Oracle(_params(kBT=0.0, enable_lub=0), parts)
    o.compute_forces()
    F, N = o.read_field("F_DEM"), o.read_field("N_DEM")
    assert np.allclose(F[1], -F[0], rtol=0, atol=1e-15 * np.linalg.norm(F[0]))
    Ft = F[0] - np.dot(F[0], n) * n
    assert np.linalg.norm(Ft) > 1e-3 * np.linalg.norm(F[0])
    r = Lc * n
    rate = np.cross(r, F[0]) + N[0] + N[1]
    expect = (Lc - Ri - Rj) * np.cross(n, Ft)
    scale = (Ri + Rj) * np.linalg.norm(F[0])
    assert np.allclose(rate, expect, atol=1e-12 * scale, rtol=0)
    # each sphere's own lever is its radius: |N_i| = R_i |F_t| (torque normal to n)
    assert np.linalg.norm(N[0]) == pytest.approx(Ri * np.linalg.norm(Ft), rel=1e-12)
    assert np.linalg.norm(N[1]) == pytest.approx(Rj * np.linalg.norm(Ft), rel=1e-12)
    assert abs(np.dot(N[0], n)) < 1e-12 * np.linalg.norm(N[0])


def _lub_pair(oracle_lib, gap, u, R=0.75, seed=0, **over):
    rng = np.random.default_rng(seed)
    n = _unit(rng)
    Lc = 2 * R + gap
    c = np.array([3.0, 3.0, 3.0])
    m = 2.5 * RHO0 * 4 / 3 * math.pi * R ** 3
    # approaching head-on at relative speed u along n
    parts = _two([W.RIGID, W.RIGID], [c + Lc * n / 2, c - Lc * n / 2],
                 [-0.5 * u * n, 0.5 * u * n], np.zeros((2, 3)), radius=(R, R), mass=(m, m),
                 inertia=(0.4 * m * R * R,) * 2)
    p = _params(kBT=0.0, **over)
    o = oracle_lib.Oracle(p, parts)
    o.compute_forces()
    return o.read_field("F_LUB"), n, p


@pytest.mark.parametrize("gap", [0.05, 0.3, 0.9])
def test_lubrication_matches_squeeze_film(oracle_lib, gap):
    R, u = 0.75, 0.2
    F, n, p = _lub_pair(oracle_lib, gap, u, R)
    rstar = R * R / (R + R)
    expect = 6.0 * math.pi * p["eta"] * rstar ** 2 * u / gap
    # pushes the spheres apart, equal and opposite
    assert np.allclose(F[0], expect * n, rtol=1e-12, atol=0)
    assert np.allclose(F[1], -expect * n, rtol=1e-12, atol=0)


def test_lubrication_gap_floor_and_cutoff(oracle_lib):
    R, u, gmin = 0.75, 0.2, 0.02
    F_floor, n, p = _lub_pair(oracle_lib, gmin, u, R, lub_gap_min=gmin)
    F_below, _, _ = _lub_pair(oracle_lib, 0.4 * gmin, u, R, lub_gap_min=gmin)
    # below the floor the resistance stays at its value at the floor
    assert np.allclose(F_below, F_floor, rtol=1e-12, atol=0)
    F_out, _, p = _lub_pair(oracle_lib, 1.001 * 2 * DX, u, R)
    assert np.abs(F_out).max() == 0.0  # the gap is beyond the support h
