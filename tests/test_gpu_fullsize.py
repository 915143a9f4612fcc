"""Parity at the full sizes of the measured workloads, in the launch
configurations the benchmark uses (fluid cells of 0.55 h; the dam break
and the scale box also stepped with neighbour-candidate reuse at skin
h/15; the viscometer batch at 0.67 h, its tuner's pick, also stepped with
candidate reuse under shear) and at cells of h: the sedimentation box
(101,080 particles), the dam break (1,534,168 particles, 2^20 moving) and
the periodic scale box (8,388,608 particles).  The oracle evaluates every
particle of a box it is given; neighbour sets must match bit for bit."""
import numpy as np
import pytest

from _parity import VECTOR_FIELDS, assert_force_field, assert_same_neighbors, assert_scalar_fields
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


@pytest.mark.parametrize("name,cf", [("sedimentation", 0.5), ("sedimentation", 1.0),
                                     ("dam_break", 0.55), ("dam_break", 1.0),
                                     ("periodic_scale", 0.55)])
def test_full_size_single_step(S, oracle_lib, name, cf):
    p, parts, info = W.CONFIGS[name]()
    parts = W.perturb(parts, p, jitter=0.05, kT=1e-4, seed=7)
    print(f"[case] full-size {name}: n={info['n']} cell_factor={cf}", flush=True)
    g = S.System(dict(p, cell_factor=cf), parts)
    o = oracle_lib.Oracle(p, parts)
    assert g.compute_forces(check=False) == 0
    assert o.compute_forces(check=False) == 0
    nnz = assert_same_neighbors(g, o)
    assert_scalar_fields(g, o, p)
    worst = {f: assert_force_field(g, o, f) for f in VECTOR_FIELDS}
    print("  nnz", nnz, {k: f"{v:.1e}" for k, v in worst.items()}, flush=True)


def test_full_dam_break_after_steps_with_reuse(S, oracle_lib):
    """The bench's headline system (cells of 0.55 h, skin 0.1 = h/15) after
    60 steps, its lists taken from the candidates since the last search:
    the oracle, made from its state, searches from scratch."""
    from test_gpu_reuse import _hand_over
    p, parts, info = W.CONFIGS["dam_break"]()
    print(f"[case] full-size dam break, 60 steps with reuse: n={info['n']}", flush=True)
    g = S.System(dict(p, cell_factor=0.55, skin=0.1), parts)
    g.step(60)
    inf = g.info()
    print(f"  {inf[13]} searches, {inf[14]} lists from candidates", flush=True)
    assert inf[14] >= 30
    _hand_over(S, oracle_lib, g, p, parts, VECTOR_FIELDS)


def test_full_scale_box_after_steps_with_reuse(S, oracle_lib):
    """The benchmark's periodic scale box (8,388,608 particles, kT = 1e-3,
    cells of 0.55 h, skin 0.1 = h/15) after 30 steps from a jittered
    lattice, every list since the first search taken from its candidates:
    the oracle, made from its state, searches from scratch."""
    from test_gpu_reuse import _hand_over
    p, parts, info = W.CONFIGS["periodic_scale"]()
    parts = W.perturb(parts, p, jitter=0.05, kT=1e-3, seed=11)
    print(f"[case] full-size scale box, 30 steps with reuse: n={info['n']}", flush=True)
    g = S.System(dict(p, cell_factor=0.55, skin=0.1), parts)
    g.step(30)
    inf = g.info()
    print(f"  {inf[13]} searches, {inf[14]} lists from candidates", flush=True)
    assert inf[14] >= 25
    _hand_over(S, oracle_lib, g, p, parts, VECTOR_FIELDS)


def test_full_viscometer_batch_sampled_boxes(S, oracle_lib):
    """The bench's batched viscometer (256 Lees-Edwards cells, 7,272,566
    particles, cells of 0.67 h): one force evaluation of the whole batch, and
    six of its boxes (the smallest, the largest and four drawn at random)
    evaluated one by one by the oracle; their rows must match the oracle's
    neighbours bit for bit and its force fields within the tolerances."""
    shared, cells = W.viscometer_batch(256, seed=0, steps=5000)
    parts, boxes, box_of = W.stack_cells(cells)
    print(f"[case] full viscometer batch n={parts['id'].shape[0]}", flush=True)
    g = S.System(dict(shared, cell_factor=0.67), parts, boxes=boxes, box_of=box_of)
    assert g.compute_forces(check=False) == 0
    rows, cols = g.read_neighbors()  # CSR: row starts (n + 1) and columns
    fields = {f: g.read_field(f) for f in VECTOR_FIELDS}
    sizes = np.array([c[2]["n"] for c in cells])
    offs = np.concatenate([[0], np.cumsum(sizes)])
    rng = np.random.default_rng(1)
    pick = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)),
                   *rng.choice(len(cells), 4, replace=False).tolist()})
    for b in pick:
        p, pp, info = cells[b]
        a, e = int(offs[b]), int(offs[b + 1])
        o = oracle_lib.Oracle(p, pp)
        assert o.compute_forces(check=False) == 0
        ro, co = o.read_neighbors()
        assert np.array_equal(rows[a:e + 1] - rows[a], ro), b
        assert np.array_equal(cols[rows[a]:rows[e]] - a, co), b
        for f in VECTOR_FIELDS:
            gv = fields[f][a:e]
            ov, sc = o.read_field(f), o.read_field(f + "_ABS")
            err = np.linalg.norm(gv - ov, axis=1)
            tiny = 1e-30 + 1e-12 * (sc.max() if sc.size else 0.0)
            assert np.all(err <= 1e-5 * sc + tiny), (b, f)
        print(f"  box {b}: n={e - a}, {int(ro[-1])} neighbour slots", flush=True)


def test_full_viscometer_batch_with_sheared_reuse(S, oracle_lib):
    """The batch as the benchmark's tuned shape runs it: eager steps with
    neighbour-candidate reuse under shear (skin 0.1 = h/15), 60 steps, so
    that the fastest-sheared cells search again while the rest take their
    lists from candidates.  Three boxes (the smallest, the largest and one
    drawn at random) then go to the oracle with their state, contacts and
    step number; the oracle searches from scratch."""
    shared, cells = W.viscometer_batch(256, seed=0, steps=5000)
    parts, boxes, box_of = W.stack_cells(cells)
    print(f"[case] full viscometer batch with reuse, n={parts['id'].shape[0]}", flush=True)
    g = S.System(dict(shared, cell_factor=0.67, skin=0.1), parts, boxes=boxes, box_of=box_of)
    assert g.step(60) == 0
    inf = g.info()
    print(f"  60 steps: {inf[13]} searches, {inf[14]} lists from candidates", flush=True)
    assert inf[13] >= 2 and inf[14] >= 30
    pos, vel, ang = (g.read_field(f) for f in ("POS", "VEL", "ANGVEL"))
    pairs, dts = g.read_contacts()
    assert g.compute_forces(check=False) == 0
    rows, cols = g.read_neighbors()
    fields = {f: g.read_field(f) for f in VECTOR_FIELDS}
    sizes = np.array([c[2]["n"] for c in cells])
    offs = np.concatenate([[0], np.cumsum(sizes)])
    rng = np.random.default_rng(2)
    pick = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)),
                   int(rng.integers(len(cells)))})
    for b in pick:
        p, pp, _info = cells[b]
        a, e = int(offs[b]), int(offs[b + 1])
        st = {k: np.array(v, copy=True) for k, v in pp.items()}
        st["pos"], st["vel"], st["angvel"] = pos[a:e], vel[a:e], ang[a:e]
        o = oracle_lib.Oracle(dict(p, itr_start=g.current_step), st)
        mine = np.all((pairs >= a) & (pairs < e), axis=1)
        if mine.any():
            o.load_contacts(pairs[mine] - a, dts[mine])
        assert o.compute_forces(check=False) == 0
        ro, co = o.read_neighbors()
        assert np.array_equal(rows[a:e + 1] - rows[a], ro), b
        assert np.array_equal(cols[rows[a]:rows[e]] - a, co), b
        worst = 0.0
        for f in VECTOR_FIELDS:
            ov, sc = o.read_field(f), o.read_field(f + "_ABS")
            err = np.linalg.norm(fields[f][a:e] - ov, axis=1)
            tiny = 1e-30 + 1e-12 * (sc.max() if sc.size else 0.0)
            assert np.all(err <= 1e-5 * sc + tiny), (b, f)
            worst = max(worst, float((err / (sc + tiny)).max()))
        print(f"  box {b}: n={e - a}, {int(ro[-1])} neighbour slots, worst rel {worst:.1e}",
              flush=True)
