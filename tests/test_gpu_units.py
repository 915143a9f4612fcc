"""GPU library vs the FP64 oracle away from unit density and spacing, across
wall faces, and in the drag branches the other parity cases do not reach.

* The slurry channel of Secs. 4.1 and 4.3 at the paper's constants
  (rho0 = 3, eta = 25, p0 = beta = 100; dx = 0.5, m_f = 0.375, h = 2 dx,
  kT = 1): fully periodic and wall-periodic, with interleaved spheres.
  Here the number density rho/m_f (Eqs. FijC, gamma), C_W m_f (Eq.
  compdens) and rho0 V_s/m_f (Eq. F_fpi_PG) do not cancel.
* Particles whose drift crosses a wall face, an edge and a corner, with
  slip and no-slip walls (Sec. 2.5).
* A sphere at Re_p > 1000 (Newton drag, Sec. 2.4), one in a cluster dense
  enough for the eps_min clamp (Ergun branch), one with 0.8 < eps < 1.

Neighbour sets bit for bit; force fields within 1e-5 of the per-particle
sum of pair-term magnitudes; rho, p, eps as in the other parity tests.
"""
import math

import numpy as np
import pytest

from _parity import (VECTOR_FIELDS, assert_force_field, assert_same_neighbors,
                     assert_scalar_fields)
from paper_2002_03120_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_03120_amd import sdpdem
    sdpdem.lib()
    return sdpdem


def _check_all(g, o, p, fields=VECTOR_FIELDS):
    rc_g = g.compute_forces(check=False)
    rc_o = o.compute_forces(check=False)
    assert rc_g == rc_o == 0, (rc_g, rc_o)
    nnz = assert_same_neighbors(g, o)
    assert_scalar_fields(g, o, p)
    worst = {f: assert_force_field(g, o, f) for f in fields}
    print("  nnz", nnz, "worst rel", {k: f"{v:.1e}" for k, v in worst.items()}, flush=True)
    return worst


@pytest.mark.parametrize("interval,walls", [(0, False), (5, True), (10, False), (15, True)])
def test_slurry_channel_single_step(S, oracle_lib, interval, walls):
    p, parts, info = W.slurry_channel(interval, walls=walls)
    parts = W.perturb(parts, p, jitter=0.1, kT=p["kBT"], seed=7, spin=True)
    print(f"[case] slurry channel interval={interval} walls={walls}: n={parts['id'].shape[0]}, "
          f"{int((parts['type'] == W.RIGID).sum())} spheres", flush=True)
    g = S.System(p, parts)
    o = oracle_lib.Oracle(p, parts)
    _check_all(g, o, p)


def test_slurry_channel_short_trajectory(S, oracle_lib):
    """Ten steps of the wall-periodic slurry at interval 5 on a 22 x 22 x 20
    site box (no two face-adjacent sites are spheres): positions stay within
    1e-5 dx of the oracle's and the contact tables agree."""
    p, parts, _ = W.slurry_channel(5, walls=True, L=(11.0, 11.0, 10.0))
    parts = W.perturb(parts, p, jitter=0.05, kT=p["kBT"], seed=8, spin=True)
    print(f"[case] slurry trajectory: n={parts['id'].shape[0]}", flush=True)
    g = S.System(p, parts)
    o = oracle_lib.Oracle(p, parts)
    g.step(10)
    o.step(10)
    dxm = np.abs(g.read_field("POS") - o.read_field("POS")).max()
    dv = np.abs(g.read_field("VEL") - o.read_field("VEL")).max()
    print(f"  10 steps: max |dx| {dxm:.2e}, max |dv| {dv:.2e}", flush=True)
    assert dxm < 1e-5 * p["dx"]
    pg, tg = g.read_contacts()
    po, to = o.read_contacts()
    assert np.array_equal(pg, po)
    if len(po):
        assert np.abs(tg - to).max() <= 1e-6 * max(1e-12, np.abs(to).max())


def _crossing_box(noslip):
    """A walled 8^3 box: a cloud of particles in its centre and, isolated from
    it (farther than h), particles that cross a face, an edge and a corner
    in the first drift, plus one that stays inside."""
    rng = np.random.default_rng(4)
    n_cloud = 40
    cloud = 2.0 + rng.random((n_cloud, 3)) * 4.0
    movers = np.array([[0.05, 4.0, 4.0], [7.97, 0.02, 4.0], [0.03, 7.96, 0.04],
                       [7.9, 7.9, 7.9], [0.3, 0.3, 7.6]])
    vmov = np.array([[-10.0, 0.5, 0.2], [5.0, -5.0, 0.3], [-5.0, 5.0, -7.0],
                     [1.0, 1.0, 1.0], [-1.0, 2.0, -3.0]])
    pos = np.vstack([cloud, movers])
    n = pos.shape[0]
    vel = np.vstack([rng.standard_normal((n_cloud, 3)) * 0.05, vmov])
    parts = dict(id=np.arange(n), type=np.zeros(n, np.uint8), pos=pos, vel=vel,
                 angvel=np.zeros((n, 3)), mass=np.ones(n), inertia=np.full(n, 0.1),
                 radius=np.full(n, 0.5))
    p = W.base_params(L=[8.0, 8.0, 8.0], periodic=[0, 0, 0], noslip=noslip, kBT=0.0, dt=0.01,
                      g=[0.0, 0.0, 0.0])
    return p, parts, np.arange(n_cloud, n)


@pytest.mark.parametrize("noslip", [1, 0])
def test_wall_face_edge_and_corner_crossing(S, oracle_lib, noslip):
    p, parts, movers = _crossing_box(noslip)
    print(f"[case] wall crossing noslip={noslip}: n={parts['id'].shape[0]}", flush=True)
    g = S.System(p, parts)
    o = oracle_lib.Oracle(p, parts)
    g.step(1)
    o.step(1)
    xg, xo = g.read_field("POS"), o.read_field("POS")
    vg, vo = g.read_field("VEL"), o.read_field("VEL")
    # the isolated movers feel no force: the update is exact FP64 on both sides
    assert np.array_equal(vg[movers], vo[movers]), (vg[movers], vo[movers])
    assert np.abs(xg[movers] - xo[movers]).max() < 1e-14
    v0 = parts["vel"][movers]
    crossed = [[True, False, False], [True, True, False], [True, True, True],
               [False, False, False], [False, False, False]]
    for k, c in enumerate(crossed):
        if noslip:
            expect = -v0[k] if any(c) else v0[k]
        else:
            expect = np.where(c, -v0[k], v0[k])
        assert np.array_equal(vo[movers[k]], expect), (k, vo[movers[k]], expect)
    assert np.all((xg >= 0.0) & (xg <= 8.0))
    # the cloud: FP32 pair forces, each within 1e-5 of the sum of its pair
    # magnitudes, enter two half-kicks and one drift
    A = o.read_field("F_SDPD_ABS")[:, None]
    assert np.all(np.abs(vg - vo) <= 2e-5 * p["dt"] * A + 1e-13)
    assert np.all(np.abs(xg - xo) <= 2e-5 * p["dt"] ** 2 * A + 1e-13)


def _spheres_in_fluid(centres, vels, d=3.0, n=24, **over):
    p, parts, _ = W.reverse_poiseuille(n_side=(n, n, n), kBT=0.0, g=0.0, **over)
    R = d / 2
    vs = 4.0 / 3.0 * math.pi * R ** 3
    ks = []
    for c, v in zip(centres, vels):
        k = int(np.argmin(((parts["pos"] - np.asarray(c)) ** 2).sum(axis=1)))
        parts["type"][k] = W.RIGID
        parts["pos"][k] = c
        parts["vel"][k] = v
        parts["mass"][k] = 2.5 * vs
        parts["inertia"][k] = 0.4 * 2.5 * vs * R * R
        parts["radius"][k] = R
        ks.append(k)
    return p, parts, ks


def test_drag_branches_newton_and_eps_clamp(S, oracle_lib):
    """Newton drag (Re_p > 1000) for an isolated sphere and for one with a
    partner (eps = 0.875, the Wen-Yu voidage factor); a sphere with four
    partners inside its support, whose eps = 0.5 is clamped to eps_min = 0.6
    (Ergun branch); the partners sit at eps = 0.875 in Schiller-Naumann."""
    a = 2.95  # centre distance of the slightly overlapping cluster
    c0 = np.array([16.5, 16.5, 16.5])
    centres = [(6.5, 6.5, 6.5),                        # isolated, fast
               (6.5, 17.0, 17.0), (6.5 + a, 17.0, 17.0),  # pair, fast
               tuple(c0), tuple(c0 + [a, 0, 0]), tuple(c0 - [a, 0, 0]),
               tuple(c0 + [0, a, 0]), tuple(c0 - [0, a, 0])]
    vels = [(40.0, 3.0, -2.0), (0.0, 60.0, 1.0), (0.0, 0.0, 0.0),
            (0.1, -0.05, 0.02), (0.0, 0.1, 0.0), (0.05, 0.0, 0.0), (0.0, 0.0, -0.1),
            (0.02, 0.0, 0.0)]
    p, parts, ks = _spheres_in_fluid(centres, vels, eps_min=0.6)
    print(f"[case] drag branches: n={parts['id'].shape[0]}", flush=True)
    g = S.System(p, parts)
    o = oracle_lib.Oracle(p, parts)
    _check_all(g, o, p)
    eps = o.read_field("EPS")[ks]
    assert eps[0] == 1.0 and eps[1] == pytest.approx(0.875, rel=1e-14) and eps[3] == 0.6
    re = p["rho0"] * 3.0 * eps * np.linalg.norm(np.asarray(vels), axis=1) / p["eta"]
    assert re[0] > 1000 and re[1] > 1000 and re[3] < 1000
    assert np.allclose(g.read_field("F_DG")[ks], o.read_field("F_DG")[ks], rtol=1e-11, atol=0)
