"""Neighbour-candidate reuse (skin > 0) against the FP64 oracle.

With a skin the library searches the cell grid for partners within
h + skin and, until some particle has moved skin/2 from where that search
saw it, takes each drift's lists from those candidates instead of sorting
and searching again (Alg. 1's neighbour step, Sec. 3.2).  The neighbour
sets must stay exactly {j : r_ij < h}.  Each case runs a moving system long
enough for several searches and many reusing steps, then hands its state
(positions, velocities, spins, DEM contacts, step number) to the oracle,
which searches from scratch: neighbour sets bit for bit, rho and p to
1e-12, forces to the single-step tolerance, with the library's last lists
taken from the candidates.
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


def _hand_over(S, oracle_lib, g, p, parts, fields):
    """The oracle from g's current state; one force evaluation on each (g
    keeps the lists its last step took from the candidates)."""
    state = {k: np.array(v, copy=True) for k, v in parts.items()}
    state["pos"], state["vel"], state["angvel"] = (g.read_field(f) for f in ("POS", "VEL", "ANGVEL"))
    o = oracle_lib.Oracle(dict(p, itr_start=g.current_step), state)
    pairs, dts = g.read_contacts()
    if len(pairs):
        o.load_contacts(pairs, dts)
    rc_g = g.compute_forces(check=False)
    rc_o = o.compute_forces(check=False)
    assert rc_g == rc_o == 0, (rc_g, rc_o)
    nnz = assert_same_neighbors(g, o)
    assert_scalar_fields(g, o, p)
    worst = {f: assert_force_field(g, o, f) for f in fields}
    print("  nnz", nnz, "worst rel", {k: f"{v:.1e}" for k, v in worst.items()}, flush=True)


def _run(S, p, parts, skin, steps, graph=0, **gpu_only):
    g = S.System(dict(p, skin=skin, **gpu_only), parts)
    if graph:
        g.set_graph(graph)
    g.step(steps)
    info = g.info()
    print(f"  {steps} steps: {info[13]} searches, {info[14]} lists from candidates", flush=True)
    return g, info


@pytest.mark.parametrize("cf", [0.5, 0.55, 1.0])
def test_dam_break_reused_lists_equal_a_fresh_search(S, oracle_lib, cf):
    """Walls, inner walls, spheres with contacts and the coupling (whose
    search in the grid of the last sort reaches skin/2 farther), thermal
    noise; particles set moving so that the skin runs out several times."""
    p, parts, _ = W.dam_break(tank=(40, 16, 30), column=(20, 16, 20), n_rigid=60, seed=7,
                              kBT=1e-4)
    parts = W.perturb(parts, p, jitter=0.1, kT=4e-2, seed=9, spin=True)
    print(f"[case] dam break 40x16x30 skin 0.2h cell_factor={cf}", flush=True)
    g, info = _run(S, p, parts, 0.3, 160, cell_factor=cf)
    assert info[13] >= 3 and info[14] >= 60
    _hand_over(S, oracle_lib, g, p, parts, VECTOR_FIELDS)


def test_periodic_lattice_with_fast_particles(S, oracle_lib):
    """A fully periodic jittered lattice at a high temperature: particles
    wrap around the box between searches (the displacement is taken
    through the minimum image) and the skin runs out every few steps."""
    q, parts, _ = W.reverse_poiseuille(n_side=(14, 14, 14), dt=5e-3, kBT=2e-2)
    parts = W.perturb(parts, q, jitter=0.1, kT=0.5, seed=22, spin=True)
    print("[case] periodic lattice 14^3, fast particles, skin 0.2h", flush=True)
    g, info = _run(S, q, parts, 0.3, 60)
    assert info[13] >= 3 and info[14] >= 20
    _hand_over(S, oracle_lib, g, q, parts, ["F_SDPD", "F_CD", "N_SDPD"])


@pytest.mark.parametrize("noslip", [1, 0])
def test_wall_crossings_between_searches(S, oracle_lib, noslip):
    """A box with wall faces on every axis and no wall particles: fast
    particles cross the faces (mirror and velocity reversal, Sec. 2.5)
    while the lists come from the candidates."""
    q, parts, _ = W.reverse_poiseuille(n_side=(12, 12, 12), dt=5e-3, kBT=0.0,
                                       periodic=[0, 0, 0], g=0.0, noslip=noslip)
    parts = W.perturb(parts, q, jitter=0.1, kT=0.5, seed=32, spin=True)
    print(f"[case] walled lattice 12^3 noslip={noslip}, skin 0.3h", flush=True)
    g, info = _run(S, q, parts, 0.45, 60)
    assert info[14] >= 20
    _hand_over(S, oracle_lib, g, q, parts, ["F_SDPD", "F_CD", "N_SDPD"])


def test_wall_periodic_slurry_at_the_papers_units(S, oracle_lib):
    """The slurry channel of Sec. 4.3 at the paper's constants (rho0 = 3,
    m_f = 0.375, h = 2 dx, kT = 1): periodic in x and y, wall faces on z
    (outer walls sorted behind the active particles, seams on two axes),
    interleaved spheres with contacts; the thermal motion runs the skin out
    several times."""
    p, parts, _ = W.slurry_channel(5, walls=True, L=(11.0, 11.0, 10.0))
    parts = W.perturb(parts, p, jitter=0.05, kT=p["kBT"], seed=31, spin=True)
    print(f"[case] wall-periodic slurry, n={parts['id'].shape[0]}, skin 0.3h", flush=True)
    g, info = _run(S, p, parts, 0.3 * p["h"], 80)
    assert info[13] >= 2 and info[14] >= 20
    _hand_over(S, oracle_lib, g, p, parts, VECTOR_FIELDS)


def test_graph_replay_searches_every_step(S, oracle_lib):
    """Inside a captured graph the host cannot decide, so every replayed step
    searches (and refreshes the candidates); eager steps after the replays
    reuse them again."""
    p, parts, _ = W.dam_break(tank=(40, 16, 30), column=(20, 16, 20), n_rigid=60, seed=8,
                              kBT=0.0)
    parts = W.perturb(parts, p, jitter=0.1, kT=4e-2, seed=10, spin=True)
    import torch
    print("[case] dam break, skin 0.2h, 4-step graphs", flush=True)
    g = S.System(dict(p, skin=0.3), parts, stream=torch.cuda.Stream())  # capture needs one
    g.set_graph(4)
    g.step(17)  # one eager step (first search, then its drift), four graphs of four
    info = g.info()
    assert info[11] == 16 and info[13] >= 17 and info[13] + info[14] == 18, info[11:15]
    g.set_graph(0)
    g.step(6)
    info = g.info()
    assert info[14] >= 1, info[11:15]
    _hand_over(S, oracle_lib, g, p, parts, VECTOR_FIELDS)


def test_batch_of_boxes_with_reuse(S, oracle_lib):
    """A batch of three unsheared periodic cells with spheres (the batched
    viscometer's boxes at zero shear rate), run with a skin: any box's
    drift past skin/2 makes the whole batch search again.  Each box's
    state afterwards goes to an oracle of its own."""
    cells = [W.shear_cell(n_side=n, phi=0.2, d=3.0, kBT=0.05, shear_rate=0.0, seed=40 + n)
             for n in (10, 12, 11)]
    parts, boxes, box_of = W.stack_cells(cells)
    print(f"[case] batch of 3 unsheared cells, skin 0.3: n={parts['id'].shape[0]}", flush=True)
    g = S.System(dict(cells[0][0], skin=0.3), parts, boxes=boxes, box_of=box_of)
    g.step(80)
    inf = g.info()
    print(f"  80 steps: {inf[13]} searches, {inf[14]} lists from candidates", flush=True)
    assert inf[14] >= 20
    g.compute_forces()
    pos, vel, ang = (g.read_field(f) for f in ("POS", "VEL", "ANGVEL"))
    rows, cols = g.read_neighbors()
    rho = g.read_field("DENS")
    fs = g.read_field("F_SDPD")
    off = 0
    for p, pp, info in cells:
        n = pp["id"].shape[0]
        st = {k: np.array(v, copy=True) for k, v in pp.items()}
        st["pos"], st["vel"], st["angvel"] = pos[off:off + n], vel[off:off + n], ang[off:off + n]
        o = oracle_lib.Oracle(dict(p, itr_start=g.current_step), st)
        assert o.compute_forces(check=False) == 0
        ro, co = o.read_neighbors()
        assert np.array_equal(rows[off:off + n + 1] - rows[off], ro)
        assert np.array_equal(cols[rows[off]:rows[off + n]] - off, co)
        assert np.allclose(rho[off:off + n], o.read_field("DENS"), rtol=1e-12, atol=0)
        sc = o.read_field("F_SDPD_ABS")
        err = np.linalg.norm(fs[off:off + n] - o.read_field("F_SDPD"), axis=1)
        assert np.all(err <= 1e-5 * sc + 1e-30)
        off += n


def _search_steps(g, steps):
    """Step g one step at a time; the steps (0-based) whose build was a
    cell-grid search, after the first step's initial build."""
    g.step(1)
    last = g.info()[13]
    assert last == 1  # the initial build, ahead of the first pass
    searched = []
    for m in range(1, steps):
        g.step(1)
        n = g.info()[13]
        assert n - last in (0, 1)
        if n > last:
            searched.append(m)
        last = n
    print(f"  searches at steps {searched}", flush=True)
    return searched


def test_search_comes_when_a_translation_reaches_half_the_skin(S):
    """A periodic fluid lattice moving as a whole (every velocity the same,
    no noise) feels no net force: relative velocities vanish and the
    neighbourhoods stay centrosymmetric.  Each drift moves every particle
    by |v| dt, so the lists come from the candidates until the distance
    from the searched positions passes skin/2: a search every K =
    ceil(skin / (2 |v| dt)) steps, the first interval counted from the
    positions the initial build saw."""
    dt, skin = 5e-3, 0.3
    v = np.array([0.48, -0.2, 0.0])
    p, parts, _ = W.shear_cell(12, 0.0, 0.0, kBT=0.0, shear_rate=0.0, dt=dt)
    parts["vel"][:] = v
    parts["angvel"][:] = 0.0
    ratio = skin / (2.0 * np.linalg.norm(v) * dt)
    K = math.ceil(ratio)
    assert 0.1 < ratio % 1.0 < 0.9  # the threshold falls well between two steps
    print(f"[case] translating lattice n={parts['id'].shape[0]}, |v| {np.linalg.norm(v):.3f}, "
          f"skin {skin}, K {K}", flush=True)
    g = S.System(dict(p, skin=skin), parts)
    searched = _search_steps(g, 3 * K + 2)
    g.close()
    assert searched == [K - 1, 2 * K - 1, 3 * K - 1]


@pytest.mark.parametrize("start", ["fresh", "compute_forces", "restart"])
def test_sheared_search_comes_when_the_flow_reaches_the_skin(S, start):
    """A fluid lattice in exact affine shear flow (v_x = rate (z - L/2), no
    noise, no spheres) keeps a centrosymmetric neighbourhood around every
    particle, so the pair forces cancel to rounding and each drift is the
    flow's.  The reuse criterion is then decided by its time term alone: a
    search as soon as the time between the searched positions and the
    drifted ones reaches skin / (|rate| (h + skin)), i.e. every K =
    ceil(skin / (|rate| (h + skin) dt)) steps.  The first interval counts
    from the positions the initial build saw, those of the start of the
    first step, like every later one (a search between the two passes sees
    the positions the step's drift made); counting it from the first drift
    instead would let a pair across the sheared face close in by one step
    of image offset, rate L_z dt, that the skin does not cover.  The same
    schedule whichever way the first build comes: a new system, a force
    evaluation ahead of the first step, a restart at a later step."""
    rate, dt, skin = 1.5, 5e-3, 0.3
    p, parts, _ = W.shear_cell(12, 0.0, 0.0, kBT=0.0, shear_rate=rate, dt=dt)
    if start == "restart":
        a = S.System(p, parts)
        a.step(7)
        parts = {k: np.array(v, copy=True) for k, v in parts.items()}
        parts["pos"], parts["vel"], parts["angvel"] = (a.read_field(f)
                                                       for f in ("POS", "VEL", "ANGVEL"))
        p = dict(p, itr_start=a.current_step)
        a.close()
    K = math.ceil(skin / (abs(rate) * (p["h"] + skin) * dt))
    frac = skin / (abs(rate) * (p["h"] + skin) * dt) % 1.0
    assert 0.1 < frac < 0.9  # the threshold falls well between two steps
    print(f"[case] affine shear lattice n={parts['id'].shape[0]}, rate {rate}, skin {skin}, "
          f"K {K}, {start}", flush=True)
    g = S.System(dict(p, skin=skin), parts)
    if start == "compute_forces":
        g.compute_forces()
    searched = _search_steps(g, 3 * K + 2)
    g.close()
    assert searched == [K - 1, 2 * K - 1, 3 * K - 1]


def test_sheared_batch_with_reuse(S, oracle_lib):
    """Three Lees-Edwards cells at different shear rates with spheres,
    contacts and thermal noise, run with a skin: a particle's drift is
    measured against the flow's and the limit shrinks with the time since
    the search, so the fastest-sheared cell (the flow's term alone allows
    some 180 steps there) makes the batch search again.  Each box's state then goes to an oracle of its own, which
    searches from scratch (its image offset from the step number)."""
    cells = [W.shear_cell(12, 0.2, 3.0, kBT=5e-3, shear_rate=0.1, seed=61),
             W.shear_cell(10, 0.0, 0.0, kBT=2e-3, shear_rate=-0.03, seed=62),
             W.shear_cell(14, 0.3, 2.5, kBT=1e-3, shear_rate=0.05, seed=63)]
    parts, boxes, box_of = W.stack_cells(cells)
    print(f"[case] batch of 3 sheared cells, skin 0.3: n={parts['id'].shape[0]}", flush=True)
    g = S.System(dict(cells[0][0], skin=0.3), parts, boxes=boxes, box_of=box_of)
    g.step(160)
    inf = g.info()
    print(f"  160 steps: {inf[13]} searches, {inf[14]} lists from candidates", flush=True)
    assert inf[13] >= 2 and inf[14] >= 60
    pos, vel, ang = (g.read_field(f) for f in ("POS", "VEL", "ANGVEL"))
    pairs, dts = g.read_contacts()
    assert g.compute_forces(check=False) == 0
    rows, cols = g.read_neighbors()
    fields = {f: g.read_field(f) for f in VECTOR_FIELDS + ["DENS"]}
    off = 0
    for b, (p, pp, _info) in enumerate(cells):
        n = pp["id"].shape[0]
        st = {k: np.array(v, copy=True) for k, v in pp.items()}
        st["pos"], st["vel"], st["angvel"] = pos[off:off + n], vel[off:off + n], ang[off:off + n]
        o = oracle_lib.Oracle(dict(p, itr_start=g.current_step), st)
        mine = np.all((pairs >= off) & (pairs < off + n), axis=1)
        if mine.any():
            o.load_contacts(pairs[mine] - off, dts[mine])
        assert o.compute_forces(check=False) == 0
        ro, co = o.read_neighbors()
        assert np.array_equal(rows[off:off + n + 1] - rows[off], ro), b
        assert np.array_equal(cols[rows[off]:rows[off + n]] - off, co), b
        assert np.allclose(fields["DENS"][off:off + n], o.read_field("DENS"), rtol=1e-12, atol=0)
        worst = 0.0
        for f in VECTOR_FIELDS:
            sc = o.read_field(f + "_ABS")
            err = np.linalg.norm(fields[f][off:off + n] - o.read_field(f), axis=1)
            tiny = 1e-30 + 1e-12 * (sc.max() if sc.size else 0.0)
            assert np.all(err <= 1e-5 * sc + tiny), (b, f)
            worst = max(worst, float((err / (sc + tiny)).max()))
        print(f"  box {b}: n {n}, nnz {co.size}, worst rel {worst:.1e}", flush=True)
        off += n


def test_candidate_overflow_is_reported(S):
    """Rows too short for the partners (18 within h on this lattice) and for
    the candidates within h + skin (56): the candidate search reports the
    neighbour overflow instead of writing past a row."""
    p, parts, _ = W.reverse_poiseuille(n_side=(10, 10, 10), kBT=1e-3)
    print("[case] candidate rows of max_neighbors 8 x ((h + skin)/h)^3", flush=True)
    g = S.System(dict(p, skin=0.75, max_neighbors=8), parts)
    assert g.step(1, check=False) == S.E_NBR_OVERFLOW
