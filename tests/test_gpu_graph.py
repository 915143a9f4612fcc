"""Steps replayed from a captured HIP graph give the same bits as eager
steps: the step counter and Lees-Edwards offsets live in device memory,
the buffer swaps repeat with period two, and a graph records whether its
first pass refills the coupling slots.  Replays are
interleaved with eager work and reads, and cross the rigid activation."""
import numpy as np
import pytest

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


def state(g):
    return [g.read_field(k) for k in ("POS", "VEL", "ANGVEL", "F_SDPD", "F_DEM", "F_RXN")]


def run(S, p, parts, chunks, graph, stress=False, boxes=None, box_of=None):
    import torch
    st = torch.cuda.Stream() if graph else None
    g = S.System(p, parts, stream=st, boxes=boxes, box_of=box_of)
    if stress:
        g.set_stress(True)
    if graph:
        g.set_graph(graph)
    reads = []
    for c in chunks:
        g.step(c)
        reads.append(g.read_field("POS")[:5].copy())  # eager work between replays
    out = state(g)
    if stress:
        out.append(g.box_stress()[1])
    out.append(g.current_step)
    info = g.info()
    if graph:
        assert info[11] > 0, "no step was replayed from a graph"
    if np.any(parts["type"] == W.RIGID):
        assert info[12] == 1, "the contacts did not get the second stream"
    g.close()
    return out, reads


@pytest.mark.parametrize("kT,act", [(0.0, 0), (1e-3, 0), (0.0, 9)])
def test_dam_break_graph_equals_eager(S, kT, act):
    p, parts, _ = W.dam_break(tank=(40, 16, 32), column=(20, 16, 20), n_rigid=60, kBT=kT)
    p["itr_actv_rigid"] = act
    print(f"[case] dam break graph kT={kT} itr_actv_rigid={act}", flush=True)
    chunks = [1, 8, 3, 12, 4]
    a, ra = run(S, p, parts, chunks, 0)
    b, rb = run(S, p, parts, chunks, 4)
    for x, y in zip(a, b):
        assert np.array_equal(np.asarray(x), np.asarray(y))
    for x, y in zip(ra, rb):
        assert np.array_equal(x, y)


def test_sheared_batch_with_stress_graph_equals_eager(S):
    sh, cells = W.viscometer_batch(5, seed=9, side=(10, 13), steps=20)
    parts, boxes, box_of = W.stack_cells(cells)
    print(f"[case] sheared batch graph n={parts['id'].shape[0]}", flush=True)
    chunks = [2, 10, 7, 10]
    a, _ = run(S, sh, parts, chunks, 0, stress=True, boxes=boxes, box_of=box_of)
    b, _ = run(S, sh, parts, chunks, 10, stress=True, boxes=boxes, box_of=box_of)
    for x, y in zip(a, b):
        assert np.array_equal(np.asarray(x), np.asarray(y))


def test_graphs_on_the_null_stream_stay_eager(S):
    """Capture needs a stream of its own: on the null stream set_graph leaves
    every step eager (none replayed) and the results are those of a system
    without graphs.  (A capture that cannot start switches graphs off for
    the rest of the call instead of being tried again.)"""
    p, parts, _ = W.dam_break(tank=(40, 16, 30), column=(20, 16, 20), n_rigid=60, kBT=1e-4)
    print("[case] dam break, graphs asked for on the null stream", flush=True)
    a = S.System(p, parts)
    a.set_graph(4)
    a.step(9)
    assert a.info()[11] == 0
    b = S.System(p, parts)
    b.step(9)
    for k in ("POS", "VEL", "ANGVEL"):
        assert np.array_equal(a.read_field(k), b.read_field(k))
