"""Lees-Edwards shear cells and batched boxes on the GPU, against the oracle.

A sheared box must give the oracle's neighbour sets bit for bit (the x
offset of the images and the image velocities included), its force fields
within the single-step tolerances and its shear stress P_zx within the
tolerance of the FP32 pair virial, at cells of h and at the autotuner's
smaller cells.  A batch of independent boxes must give, box by box, the
same bits as each box run on its own (thermal noise included: its counter
uses ids relative to the box's smallest id).  Every call goes through the
C ABI.
"""
import numpy as np
import pytest

from _parity import (assert_force_field, assert_same_neighbors, assert_scalar_fields)
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


def stress_scale(o, p):
    """|P_zx| bound of the FP32 pair virial: every pair term is at most
    h |F_ij|, so sum_i h sum_j |F_ij| / V bounds the virial's magnitude."""
    a = o.read_field("F_SDPD_ABS").sum() + o.read_field("F_DEM_ABS").sum() \
        + o.read_field("F_DG_ABS").sum() + o.read_field("F_PG_ABS").sum()
    L = p["L"]
    return 4.0 * max(p["h"], 1.0) * a / (L[0] * L[1] * L[2])


def cell(n, phi, d, kT, gd, itr, seed=0, jitter=0.1):
    p, parts, info = W.shear_cell(n, phi, d, kBT=kT, shear_rate=gd, seed=seed, dt=5e-3,
                                  itr_start=itr, max_neighbors=96)
    if jitter:
        rng = np.random.default_rng(seed + 17)
        m = parts["type"] == W.FLUID
        parts["pos"][m] += rng.uniform(-jitter, jitter, size=(int(m.sum()), 3))
        parts["pos"] %= p["L"][0]
    return p, parts, info


@pytest.mark.parametrize("cf", [1.0, 0.5, 0.34])
@pytest.mark.parametrize("itr,gd,kT", [(137, 0.05, 1e-3), (4001, -0.03, 0.0), (0, 0.08, 2e-3)])
def test_sheared_fluid_single_step(S, oracle_lib, itr, gd, kT, cf):
    p, parts, _ = cell(10, 0.0, 0.0, kT, gd, itr, seed=itr)
    print(f"[case] sheared fluid itr={itr} gd={gd} kT={kT} cell_factor={cf}", flush=True)
    g = S.System(dict(p, cell_factor=cf), parts)
    o = oracle_lib.Oracle(p, parts)
    g.set_stress(True)
    assert g.compute_forces(check=False) == 0
    assert o.compute_forces(check=False) == 0
    nnz = assert_same_neighbors(g, o)
    assert_scalar_fields(g, o, p)
    worst = {f: assert_force_field(g, o, f) for f in ("F_SDPD", "F_CD", "N_SDPD")}
    inst, _, _ = g.box_stress()
    ref = o.stress()[2, 0]
    tol = 1e-5 * stress_scale(o, p)
    print("  nnz", nnz, worst, "P_zx gpu", inst[0], "oracle", ref, "tol", tol, flush=True)
    assert abs(inst[0] - ref) <= tol


def le_shift(p):
    import math
    v = (p["shear_rate"] * p["L"][2]) * (p["itr_start"] * p["dt"])
    s = math.fmod(v, p["L"][0])
    return s + p["L"][0] if s < 0 else s


def _le_sep(p, xa, xb):
    """minimum-image separation xa - xb through the sheared faces"""
    L = p["L"][0]
    e = xa - xb
    kz = np.round(e[2] / L)
    e[2] -= kz * L
    e[0] -= kz * le_shift(p)
    e[:2] -= np.round(e[:2] / L) * L
    return e


def contact_across_sheared_face(p, parts):
    """Raise a sphere A of the top layer along z until it overlaps (by 5 %)
    the image, seen through the top face, of a sphere B of the bottom layer:
    a DEM contact then acts across the sheared face.  Of all such pairs the
    one with the smallest horizontal offset is taken; raising A moves it
    away from its own layer, and every new overlap is checked to be shallow."""
    L = p["L"][0]
    rig = np.nonzero(parts["type"] == W.RIGID)[0]
    x = parts["pos"]
    R = parts["radius"]
    zs = x[rig, 2]
    top = rig[zs > zs.max() - R[rig].max()]  # the highest layer
    bot = rig[zs < zs.min() + R[rig].max()]  # the lowest layer
    best = None
    for a in top:
        for b in bot:
            img = x[b].copy()
            img[2] += L
            img[0] = (img[0] + le_shift(p)) % L
            e = x[a] - img
            e[:2] -= np.round(e[:2] / L) * L
            hz = np.hypot(e[0], e[1])
            if hz < 0.8 * (R[a] + R[b]) and (best is None or hz < best[0]):
                best = (hz, a, b, img, e)
    assert best is not None, "no pair to bring into contact"
    hz, a, b, img, e = best
    d = 0.95 * (R[a] + R[b])
    new = x[a].copy()
    new[2] = img[2] - np.sqrt(d * d - hz * hz)
    assert x[a, 2] <= new[2] < L
    x[a] = new
    for k in rig:
        if k in (a, b):
            continue
        e = _le_sep(p, x[a].copy(), x[k])
        # other contacts may form, none deeper than 10 %
        assert np.sqrt(e @ e) > 0.9 * (R[a] + R[k]), "the raised sphere overlaps another"
    parts["vel"][a] += np.array([0.01, -0.02, -0.03])


@pytest.mark.parametrize("cf", [1.0, 0.5])
@pytest.mark.parametrize("phi,d,itr", [(0.3, 2.0, 55), (0.25, 4.0, 1234)])
def test_sheared_suspension_single_step(S, oracle_lib, phi, d, itr, cf):
    p, parts, info = cell(14, phi, d, 1e-3, 0.04, itr, seed=itr)
    p["enable_lub"] = 1
    contact_across_sheared_face(p, parts)
    print(f"[case] sheared suspension phi={phi} d={d} n_rigid={info['n_rigid']} "
          f"cell_factor={cf}", flush=True)
    g = S.System(dict(p, cell_factor=cf), parts)
    o = oracle_lib.Oracle(p, parts)
    g.set_stress(True)
    assert g.compute_forces(check=False) == 0
    assert o.compute_forces(check=False) == 0
    assert_same_neighbors(g, o)
    assert_scalar_fields(g, o, p)
    worst = {f: assert_force_field(g, o, f) for f in
             ("F_SDPD", "F_CD", "N_SDPD", "F_DG", "F_PG", "F_RXN", "F_DEM", "F_LUB", "N_DEM")}
    inst, _, _ = g.box_stress()
    ref = o.stress()[2, 0]
    tol = 1e-5 * stress_scale(o, p)
    print("  ", {k: f"{v:.1e}" for k, v in worst.items()}, "P_zx", inst[0], ref, tol, flush=True)
    assert np.abs(o.read_field("F_DEM")).max() > 0  # the contact across the face acts
    assert abs(inst[0] - ref) <= tol


def test_sheared_suspension_trajectory(S, oracle_lib):
    """40 steps with spheres crossing the sheared faces: positions stay close
    to the oracle's and the summed stress samples agree."""
    p, parts, info = cell(12, 0.3, 3.0, 0.0, 0.1, 77, seed=5, jitter=0.05)
    print(f"[case] sheared trajectory n={info['n']} n_rigid={info['n_rigid']}", flush=True)
    g = S.System(p, parts)
    o = oracle_lib.Oracle(p, parts)
    g.set_stress(True)
    steps = 40
    ref = []
    for _ in range(steps):
        o.step(1)
        ref.append(o.stress()[2, 0])
    g.step(steps)
    _, tot, m = g.box_stress()
    assert m == steps
    xg, xo = g.read_field("POS"), o.read_field("POS")
    d = xg - xo
    d -= np.round(d / p["L"][0]) * p["L"][0]
    err = np.abs(d).max()
    print("  max |dx|", err, "sum P_zx", tot[0], sum(ref), flush=True)
    assert err < 1e-6
    assert abs(tot[0] - sum(ref)) <= 1e-4 * sum(abs(x) for x in ref)


def _run(S, p, parts, steps, boxes=None, box_of=None):
    g = S.System(p, parts, boxes=boxes, box_of=box_of)
    g.set_stress(True)
    g.step(steps)
    out = dict(pos=g.read_field("POS"), vel=g.read_field("VEL"), w=g.read_field("ANGVEL"))
    out["stress"] = g.box_stress()
    g.close()
    return out


@pytest.mark.parametrize("kT", [0.0, 1e-3])
def test_batch_equals_separate_boxes(S, kT):
    """Three cells of different sizes, shear rates and sphere loads, run
    as one batch and one by one: every particle's state and every box's
    stress sum agree bit for bit (with noise too: its counters use ids
    relative to the box's smallest id)."""
    cells = [W.shear_cell(12, 0.3, 2.5, kBT=kT, shear_rate=0.05, seed=1, itr_start=10),
             W.shear_cell(10, 0.0, 0.0, kBT=kT, shear_rate=-0.02, seed=2, itr_start=10),
             W.shear_cell(16, 0.2, 4.0, kBT=kT, shear_rate=0.1, seed=3, itr_start=10)]
    steps = 25
    parts, boxes, box_of = W.stack_cells(cells)
    print(f"[case] batch of {len(cells)} boxes, n={parts['id'].shape[0]}, kT={kT}", flush=True)
    batch = _run(S, cells[0][0], parts, steps, boxes=boxes, box_of=box_of)
    off = 0
    for b, (p, pp, info) in enumerate(cells):
        one = _run(S, p, pp, steps)
        n = info["n"]
        for k in ("pos", "vel", "w"):
            assert np.array_equal(batch[k][off:off + n], one[k]), (b, k)
        assert batch["stress"][1][b] == one["stress"][1][0], b
        off += n


def test_batch_with_noise_is_repeatable(S):
    sh, cells = W.viscometer_batch(6, seed=4, side=(10, 14), steps=10)
    parts, boxes, box_of = W.stack_cells(cells)
    print(f"[case] noisy batch n={parts['id'].shape[0]}", flush=True)
    a = _run(S, sh, parts, 10, boxes=boxes, box_of=box_of)
    b = _run(S, sh, parts, 10, boxes=boxes, box_of=box_of)
    assert np.array_equal(a["pos"], b["pos"]) and np.array_equal(a["vel"], b["vel"])
    assert np.array_equal(a["stress"][1], b["stress"][1])
