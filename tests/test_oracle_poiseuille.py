"""Reverse-Poiseuille flow (the viscometer of Sec. 4.1) against its
closed-form solution.

A periodic box driven by +g along y where z - org >= L/2 and -g below
obeys, layer by layer, dv/dt = nu d2v/dz2 + f(z) with the square-wave f;
its Fourier solution from rest is

    v_y(z, t) = -(4 g / pi) sum_{k odd} (1 - exp(-nu q_k^2 t)) sin(q_k z) / (k nu q_k^2),
    q_k = 2 pi k / L,

which tends to the paper's parabolic profiles.  The SDPD fluid on a simple
cubic lattice has a lattice shear viscosity eta_lat(h) that differs from
the input eta at small h/dx (0.62 eta at h = 1.5 dx); it is measured here
independently, from the virial of a sheared lattice (Lees-Edwards box),
and the flow must follow the series with nu = eta_lat / rho.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2002_03120_amd import workloads as W
from test_oracle_shear import sheared_lattice


def series(z, t, g, L, nu, kmax=4001):
    v = np.zeros_like(z)
    for k in range(1, kmax, 2):
        q = 2.0 * math.pi * k / L
        v += -(4.0 * g / math.pi) * (1.0 - math.exp(-nu * q * q * t)) * np.sin(q * z) / (k * nu * q * q)
    return v


def lattice_viscosity(h):
    gd = 0.0625
    p, parts = sheared_lattice(8, h, gd)
    o = O.Oracle(p, parts)
    o.compute_forces()
    return -o.stress()[2, 0] / gd / p["eta"]


@pytest.mark.parametrize("h,tol", [(1.5, 0.01), (2.0, 0.02)])
def test_reverse_poiseuille_follows_the_series(oracle_lib, h, tol):
    n, eta, g, dt, steps = 12, 1.0, 1e-3, 0.02, 500
    p, parts, _ = W.reverse_poiseuille(n_side=(n, n, n), kBT=0.0, g=g, dt=dt, h=h, eta=eta,
                                       xi=20.0 * eta / 21.0, max_neighbors=200)
    o = O.Oracle(p, parts)
    o.step(steps)
    v, x = o.read_field("VEL"), o.read_field("POS")
    layer = np.floor(x[:, 2]).astype(int) % n
    prof = np.array([v[layer == k, 1].mean() for k in range(n)])
    ratio = lattice_viscosity(h)
    ref = series(np.arange(n) + 0.5, steps * dt, g, float(n), ratio * eta / p["rho0"])
    err = np.abs(prof - ref).max() / np.abs(ref).max()
    assert err < tol, (h, ratio, err)
    # the layers slide past each other: v_x and v_z stay small
    assert np.abs(v[:, [0, 2]]).max() < 0.01 * np.abs(ref).max()
