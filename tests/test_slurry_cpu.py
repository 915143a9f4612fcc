"""Host side of the reverse-Poiseuille viscometer and the slurry experiment
(Secs. 4.1 and 4.3): the profile fits against closed forms, and the slurry
generator's concentrations and layout against the paper's numbers."""
import math

import numpy as np
import pytest

from paper_2002_03120_amd import slurry as SL
from paper_2002_03120_amd import workloads as W


def exact_profile(z, D, rho, g, mu, delta=0.0):
    """Plane Poiseuille flow between v = 0 at z = -delta and z = D in the lower
    half (drive -g), mirrored with the opposite sign in the upper half."""
    z = np.asarray(z, float)
    up = z >= D
    zeta = np.where(up, 2 * D - z, z)
    v = rho * g / (2 * mu) * (zeta + delta) * (D - zeta)
    return np.where(up, v, -v)


def test_fit_recovers_the_viscosity_of_an_exact_profile():
    D, rho, g, mu = 5.0, 3.0, 1.5, 22.0
    z = (np.arange(20) + 0.5) * 0.5
    got, c = SL.fit_viscosity(z, exact_profile(z, D, rho, g, mu), D, rho, g)
    assert got == pytest.approx(mu, rel=1e-12)
    assert c == pytest.approx(rho * g / (2 * mu), rel=1e-12)


def test_mean_half_velocity_is_eq_poiseuave():
    # mean of v over a half from the closed form, by fine quadrature
    D, rho, g, mu = 5.0, 3.0, 1.5, 25.0
    z = np.linspace(0.0, D, 200001)
    v = -exact_profile(z[:-1], D, rho, g, mu)
    mean = np.trapezoid(np.append(v, 0.0), z) / D
    c = rho * g / (2 * mu)
    assert SL.mean_half_velocity(c, D) == pytest.approx(mean, rel=1e-9)
    assert SL.mean_half_velocity(c, D) == pytest.approx(rho * g * D * D / (12 * mu), rel=1e-14)


@pytest.mark.parametrize("delta", [0.0, 0.3, -0.2])
def test_slip_fit_recovers_viscosity_and_plane(delta):
    D, rho, g, mu = 5.0, 3.1, 1.5, 17.0
    z = (np.arange(20) + 0.5) * 0.5
    v = exact_profile(z, D, rho, g, mu, delta)
    got, c, d = SL.fit_viscosity_slip(z, v, D, rho, g)
    assert got == pytest.approx(mu, rel=1e-10)
    assert d == pytest.approx(delta, abs=1e-10)
    # the fixed-plane fit is biased by the slip, the way Eq. poiseuave reads it
    fixed = SL.fit_viscosity(z, v, D, rho, g)[0]
    assert (fixed < mu) == (delta > 0) or delta == 0.0


@pytest.mark.parametrize("interval,conc", [(15, 3.67), (10, 5.5), (5, 11.0)])
def test_interleave_concentrations_match_the_paper(interval, conc):
    p, parts, info = W.slurry_channel(interval, walls=True)
    assert round(100 * info["concentration"], 2) == conc
    nsites = 42 * 82 * 20
    assert info["n_rigid"] == nsites // interval
    assert info["n_fluid"] + info["n_rigid"] == nsites
    # spheres of 0.55 dx^3 at every interval-th site (id order, x fastest)
    R = parts["radius"][parts["type"] == W.RIGID]
    assert np.allclose(4.0 / 3.0 * math.pi * R ** 3, 0.55 * p["dx"] ** 3)


@pytest.mark.parametrize("interval", [15, 10, 5])
def test_interleaved_spheres_never_touch(interval):
    p, parts, info = W.slurry_channel(interval)
    x = parts["pos"][parts["type"] == W.RIGID]
    L = np.asarray(p["L"])
    # nearest periodic distance from every sphere to all others
    best = np.inf
    for k in range(x.shape[0]):
        d = x - x[k]
        d -= L * np.rint(d / L)
        r = np.sqrt((d * d).sum(axis=1))
        r[k] = np.inf
        best = min(best, r.min())
    assert best > 2.0 * parts["radius"][parts["type"] == W.RIGID][0]


def test_channel_layout():
    p, parts, info = W.slurry_channel(0, walls=True)
    assert p["periodic"] == [1, 1, 0]
    assert p["gravity_type"] == 1 and p["gravity_axis"] == 2 and p["f"] == [0.0, 1.5, 0.0]
    w = parts["pos"][parts["type"] >= W.INNER_WALL]
    assert np.all((w[:, 2] < 0) | (w[:, 2] > p["L"][2]))
    fl = parts["pos"][parts["type"] == W.FLUID]
    assert fl[:, 2].min() > 0 and fl[:, 2].max() < p["L"][2]
    q, qparts, _ = W.slurry_channel(0, walls=False)
    assert q["periodic"] == [1, 1, 1] and qparts["id"].shape[0] == 42 * 82 * 20
