"""The viscometer autotuner on the GPU: its trials, its choice, and the
launch shapes it chooses between leaving the measured viscosities alone."""
import numpy as np
import pytest

from paper_2002_03120_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def AT():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_03120_amd import autotune
    return autotune


def test_tuner_picks_the_fastest_predicted_shape(AT):
    _, cells = W.viscometer_batch(12, seed=4, side=(12, 20), steps=100)
    n = sum(c[2]["n"] for c in cells)
    print(f"[case] tune {len(cells)} cells, {n} particles", flush=True)
    res = AT.tune(cells, 1000, sample_steps=10, cell_factors=(0.5, 1.0, 1.3),
                  graph_steps=(10, 2, 0), tiles=(n // 3, 1 << 22))
    timed = [t for t in res["trials"] if "predicted_s" in t]
    assert len(timed) == 3 + 2 + 1
    assert res["predicted_s"] == min(t["predicted_s"] for t in timed)
    assert res["cell_factor"] in (0.5, 1.0, 1.3) and res["graph_steps"] in (0, 2, 10)
    assert res["tile"] in (n // 3, 1 << 22)
    assert all(t["step_ms"] > 0 and t["create_s"] > 0 for t in timed)
    h = cells[0][0]["h"]
    assert res["skin"] == (AT.REUSE_SKIN_H * h if res["graph_steps"] == 0 else 0.0)


def test_batch_tile_and_graph_length_do_not_change_results(AT):
    """Each cell owns its particle range, noise key and stress sums, so how
    the cells are packed into batches and how many steps a graph holds
    leave every measured value bit for bit the same."""
    from paper_2002_03120_amd import surrogate as SG
    _, cells = W.viscometer_batch(6, seed=5, side=(10, 14), steps=80)
    n = sum(c[2]["n"] for c in cells)
    print(f"[case] measure {len(cells)} cells two ways", flush=True)
    a = SG.measure(cells, 80, block=20)
    b = SG.measure(cells, 80, block=20,
                   tuning=dict(cell_factor=1.0, graph_steps=2, tile=n // 3))
    assert np.all(np.isfinite(a[1]))
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_eager_shape_with_reuse_measures_the_same_viscosities(AT):
    """The eager shape (graph length 0: neighbour-candidate reuse in the
    sheared cells) computes the same physics: the neighbour sets are exact,
    only the summation order differs, so over a short run each cell's
    viscosity agrees with the graph-replayed measurement to within the
    runs' own standard errors."""
    from paper_2002_03120_amd import surrogate as SG
    _, cells = W.viscometer_batch(6, seed=5, side=(10, 14), steps=200)
    n = sum(c[2]["n"] for c in cells)
    print(f"[case] measure {len(cells)} cells, graphs and eager with reuse", flush=True)
    a = SG.measure(cells, 200, block=20, tuning=dict(cell_factor=0.67, graph_steps=2, tile=n))
    b = SG.measure(cells, 200, block=20, tuning=dict(cell_factor=0.67, graph_steps=0, tile=n))
    assert np.all(np.isfinite(b[0])) and np.all(np.isfinite(b[1]))
    print("  eta", np.round(a[0], 3), np.round(b[0], 3), "se", np.round(a[1], 3), flush=True)
    assert np.all(np.abs(a[0] - b[0]) <= 3.0 * (a[1] + b[1]))


def test_single_system_tuner_picks_its_fastest_cell_size(AT):
    """tune_system, the search behind `bench.py --cell-factor 0`, on a small
    dam break: every admissible candidate is timed and the pick is the
    fastest of them."""
    p, parts, info = W.dam_break(tank=(48, 16, 32), column=(24, 16, 24), n_rigid=40, seed=2)
    print(f"[case] tune_system on n={info['n']}", flush=True)
    res = AT.tune_system(p, parts, sample_steps=4, cell_factors=(0.5, 1.0, 1.5))
    timed = [t for t in res["trials"] if "step_ms" in t]
    assert [t["cell_factor"] for t in timed] == [0.5, 1.0, 1.5]
    best = min(timed, key=lambda t: t["step_ms"])
    assert res["cell_factor"] == best["cell_factor"]
    assert res["step_ms"] == best["step_ms"]
