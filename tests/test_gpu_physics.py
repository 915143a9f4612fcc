"""Physics of the GPU path over long runs, where the oracle would be too
slow: the reverse-Poiseuille flow (Sec. 4.1) against its closed-form
series with the lattice viscosity measured by the GPU itself (virial of a
sheared lattice), and the terminal velocity of the sedimenting sphere
(Sec. 4.2 in the Stokes regime) against the Stokes value."""
import math

import numpy as np
import pytest

from paper_2002_03120_amd import workloads as W
from test_oracle_poiseuille import series
from test_oracle_shear import sheared_lattice

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_03120_amd import sdpdem
    sdpdem.lib()
    return sdpdem


def gpu_lattice_viscosity(S, h, eta=None):
    gd = 0.0625
    p, parts = sheared_lattice(8, h, gd)
    if eta is not None:
        p.update(eta=eta, xi=20.0 * eta / 21.0)
    g = S.System(p, parts)
    g.set_stress(True)
    g.compute_forces()
    inst, _, _ = g.box_stress()
    return -inst[0] / gd / p["eta"]


@pytest.mark.parametrize("n,eta,dt,steps", [(12, 1.0, 0.02, 1000), (20, 1.0, 0.01, 2000)])
def test_reverse_poiseuille_profile(S, n, eta, dt, steps):
    """The reverse-Poiseuille box at kT = 0 run to two e-folds of its
    slowest mode.  The strain stays small, so the particles keep their
    lattice and its viscosity; at eta = 0.1 the same box shears the lattice
    apart within t = 200 and the disordered fluid's viscosity differs (the
    profile then deviates by about 12 % from the lattice-viscosity series)."""
    g0 = 1e-3
    p, parts, _ = W.reverse_poiseuille(n_side=(n, n, n), kBT=0.0, g=g0, dt=dt, eta=eta,
                                       xi=20.0 * eta / 21.0)
    print(f"[case] reverse Poiseuille n={n} eta={eta} steps={steps}", flush=True)
    ratio = gpu_lattice_viscosity(S, p["h"], eta)
    g = S.System(p, parts)
    g.step(steps)
    v, x = g.read_field("VEL"), g.read_field("POS")
    layer = np.floor(x[:, 2]).astype(int) % n
    prof = np.array([v[layer == k, 1].mean() for k in range(n)])
    ref = series(np.arange(n) + 0.5, steps * dt, g0, float(n), ratio * eta / p["rho0"])
    err = np.abs(prof - ref).max() / np.abs(ref).max()
    print(f"  lattice viscosity {ratio:.4f} eta, max |v| {np.abs(ref).max():.4e}, "
          f"profile error {err:.4f}", flush=True)
    assert err < 0.02


def test_sedimenting_sphere_reaches_a_terminal_velocity(S):
    """The sphere of the sedimentation box (d = 8, density ratio 2.5,
    g = 2e-5) released at rest: its velocity levels off at a terminal value
    of the order of the Stokes velocity d^2 (rho_s - rho) g / (18 eta).  The
    coupling is unresolved (the fluid inside the sphere is dragged along)
    and the walls are near, so the ratio is reported and only bounded."""
    p, parts, info = W.sedimentation()
    g = S.System(p, parts)
    rid = int(np.nonzero(parts["type"] == W.RIGID)[0][0])
    vz = []
    block = 500
    for _ in range(info["steps"] // block):
        g.step(block)
        vz.append(g.read_field("VEL")[rid, 2])
    vz = np.array(vz)
    d, ratio, g0, eta = 8.0, 2.5, 2e-5, p["eta"]
    v_stokes = d * d * (ratio - 1.0) * p["rho0"] * g0 / (18.0 * eta)
    term = -vz[-8:].mean()
    drift = np.abs(np.diff(vz[-8:])).max() / abs(term)
    print(f"[case] sedimentation: v_term {term:.4e}, Stokes {v_stokes:.4e}, ratio "
          f"{term / v_stokes:.3f}, last-blocks drift {drift:.3f}", flush=True)
    assert term > 0 and 0.2 < term / v_stokes < 5.0
    assert drift < 0.05
